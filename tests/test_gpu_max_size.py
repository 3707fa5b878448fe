"""The largest problem the boundary accepts, L = 14 (16385 x 16385 =
268,468,225 unknowns, about 58 GB of hierarchy), solved in mixed precision,
and the FP64 fused passes at that size (vectors over 2 GiB).

Too large for the oracle to solve, so the checks use properties that hold at
any size, on a random sample of nodes: each sampled row of the device
operator equals the sum of the oracle's element matrices of the four
elements around the node (coordinates from the published generator), and
the residual b - A x at the sampled nodes, evaluated on the host with those
rows, is consistent with the residual norm the solver reports.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

L = 14
N = (1 << L) + 1
A_JIT, GSEED, RSEED = 0.2, 1404, 2404


@pytest.fixture(scope="module")
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_0904_4152_amd as mg
    mg.lib()
    return mg


def node_xy(p):
    """Jittered coordinates of nodes p (the generator's draws 2p, 2p+1)."""
    p = np.asarray(p, dtype=np.int64)
    i, j = p % N, p // N
    h = 1.0 / (N - 1)
    x, y = i * h, j * h
    inner = (i > 0) & (j > 0) & (i < N - 1) & (j < N - 1)
    ux = synth.uniform(GSEED, (2 * p).astype(np.uint64))
    uy = synth.uniform(GSEED, (2 * p + 1).astype(np.uint64))
    x = np.where(inner, x + (2 * ux - 1) * A_JIT * h, x)
    y = np.where(inner, y + (2 * uy - 1) * A_JIT * h, y)
    return x, y


def rows_from_elements(orc, p):
    """The nine band entries of row p (interior, away from the boundary) as
    the sum of the oracle's element matrices of its four elements."""
    i, j = int(p % N), int(p // N)
    row = np.zeros(9)
    for ej in (j - 1, j):
        for ei in (i - 1, i):
            corners = [(ei, ej), (ei + 1, ej), (ei + 1, ej + 1), (ei, ej + 1)]
            q = np.array([cj * N + ci for ci, cj in corners])
            xq, yq = node_xy(q)
            K = orc.element_stiffness(xq, yq)
            a = corners.index((i, j))
            for c, (ci, cj) in enumerate(corners):
                k = (cj - j + 1) * 3 + (ci - i + 1)
                row[k] += K[a, c]
    return row


def test_level_14_mixed_solve(mg, orc):
    ctx = mg.Context(0)
    h = mg.Hierarchy(ctx, L, jitter=A_JIT, seed=GSEED)
    assert h.n == N * N
    b = torch.empty(h.n, dtype=torch.float64, device="cuda")
    h.rhs_uniform(RSEED, b)
    x = torch.zeros_like(b)
    st = h.solve(b, x, mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-8))
    print("L=14 mixed: outer %d inner %d rel_res %.3e %.1f ms"
          % (st.outer_steps, st.cycles, st.rel_res, st.seconds * 1e3))
    assert st.status == 0 and st.rel_res <= 1e-8
    # sampled interior nodes away from the boundary
    rng = np.random.default_rng(14)
    i = rng.integers(2, N - 2, size=400)
    j = rng.integers(2, N - 2, size=400)
    p = j * N + i
    offs = np.array([(k // 3 - 1) * N + (k % 3 - 1) for k in range(9)])
    nb = torch.from_numpy(p[:, None] + offs[None, :]).cuda()
    xs = x[nb].cpu().numpy()
    bs = b[torch.from_numpy(p).cuda()].cpu().numpy()
    # the right-hand side at those nodes is the generator's draw
    np.testing.assert_array_equal(bs, 2.0 * synth.uniform(RSEED, p.astype(np.uint64)) - 1.0)
    rows = np.array([rows_from_elements(orc, q) for q in p])
    # the device operator's rows at the sample (band k at index p)
    dev_rows = []
    for k in range(9):
        e = torch.zeros(h.n, dtype=torch.float64, device="cuda")
        e[nb[:, k]] = 1.0
        y = torch.empty_like(e)
        h.spmv(L, e, y)
        dev_rows.append(y[torch.from_numpy(p).cuda()].cpu().numpy())
        del e, y
    dev_rows = np.stack(dev_rows, axis=1)
    # sampled nodes are far apart (neighbourhoods do not overlap in practice);
    # where two overlap the unit vectors add, so compare only clean rows
    clean = np.ones(len(p), dtype=bool)
    allnb = nb.cpu().numpy().ravel()
    vals, counts = np.unique(allnb, return_counts=True)
    shared = set(vals[counts > 1])
    for s, q in enumerate(p):
        if any(int(v) in shared for v in (q + offs)):
            clean[s] = False
    scale = np.max(np.abs(rows), axis=1, keepdims=True)
    assert np.all(np.abs(dev_rows - rows)[clean] <= (64 * 2.0 ** -53 * scale)[clean])
    # residual at the sampled nodes against the reported norm: every entry is
    # below the whole norm, and the sampled root mean square extrapolates to
    # the reported norm within a factor of three
    r = bs - np.sum(rows * xs, axis=1)
    rnorm = st.rel_res * float(torch.linalg.vector_norm(b))
    assert np.all(np.abs(r) <= rnorm)
    est = np.sqrt(np.mean(r * r) * h.n)
    assert rnorm / 3 <= est <= 3 * rnorm, (est, rnorm)
    h.close()


def test_level_14_fp64_fused_passes_equal_separate_kernels(mg):
    """FP64 vectors at L = 14 hold 2,147,745,800 bytes, past 2^31: the fused
    passes' zero-returning loads (halo columns outside the grid, rows outside
    a tile's window) must still fall outside every buffer.  The pre pass
    equals two sweeps, the defect and the restriction, and the post pass the
    prolongation and two sweeps, bit for bit, as at small sizes."""
    ctx = mg.Context(0)
    h = mg.Hierarchy(ctx, L, jitter=A_JIT, seed=GSEED)
    n, nc = h.n, ((1 << (L - 1)) + 1) ** 2
    assert n * 8 > 2 ** 31
    g = torch.Generator(device="cuda")
    g.manual_seed(1414)
    b = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
    x = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
    xc = torch.randn(nc, dtype=torch.float64, device="cuda", generator=g)
    out = torch.empty_like(x)
    bc = torch.empty_like(xc)
    h.pre_smooth(L, b, x, out, bc)
    t1 = torch.empty_like(x)
    t2 = torch.empty_like(x)
    h.jacobi(L, b, x, t1, 0.7)
    h.jacobi(L, b, t1, t2, 0.7)
    assert torch.equal(out, t2)
    h.defect(L, b, t2, t1)
    bc2 = torch.empty_like(bc)
    h.restrict(L, t1, bc2)
    assert torch.equal(bc, bc2)
    nrm = h.post_smooth(L, b, x, xc, out, norm=True)
    t1.copy_(x)
    h.prolong(L, xc, t1)
    h.jacobi(L, b, t1, t2, 0.7)
    h.jacobi(L, b, t2, t1, 0.7)
    assert torch.equal(out, t1)
    # the norm sums in another order: rounding-level agreement
    ref = h.defect(L, b, t1, t2, norm=True)
    assert abs(nrm - ref) <= 1e-12 * ref
    del b, x, xc, out, bc, t1, t2, bc2
    h.close()
