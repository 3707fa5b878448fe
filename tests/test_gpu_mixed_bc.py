"""Parity of the HIP path with the oracle for mixed boundary conditions:
homogeneous Dirichlet conditions on a chosen set of sides, the natural
Neumann condition on the others (Sec. 2.1; Sec. 6.2.2 runs its performance
test with free Neumann and geometric Dirichlet sides).

Side masks: bit 1 x = 0, bit 2 x = 1, bit 4 y = 0, bit 8 y = 1.  The cases
cover one Dirichlet side (1), two adjacent sides (5), two opposite sides
(12), three sides (14) and every side (15, the default path, which must keep
its bits).  Tolerances are those of the all-Dirichlet parity tests: the
operations are the same, only the set of constrained nodes changes.
"""
import numpy as np
import pytest

import synth
from gpu_common import U32, U64, abs_band_product, assert_within, offsets

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MASKS = [1, 5, 12, 14]


@pytest.fixture(scope="module")
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_0904_4152_amd as mg
    mg.lib()
    return mg


@pytest.fixture(scope="module")
def ctx(mg):
    return mg.Context(0)


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def dirichlet_nodes(N, mask):
    ii = np.tile(np.arange(N), N)
    jj = np.repeat(np.arange(N), N)
    return (((ii == 0) & bool(mask & 1)) | ((ii == N - 1) & bool(mask & 2)) |
            ((jj == 0) & bool(mask & 4)) | ((jj == N - 1) & bool(mask & 8)))


@pytest.mark.parametrize("mask", MASKS)
@pytest.mark.parametrize("L,a,seed", [(5, 0.0, 0), (7, 0.25, 4100)])
def test_assembled_bands_match_oracle(mg, ctx, orc, mask, L, a, seed):
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed, dirichlet_sides=mask)
    oh = orc.Hierarchy(L, synth.coords(L, a, seed), Lc=1, dmask=mask)
    for l in range(1, L + 1):
        N = (1 << l) + 1
        ref = oh.bands(l)
        got = h.bands(l)
        scale = np.max(np.abs(ref), axis=0)
        for k in range(9):
            assert_within(got[k], ref[k], 64 * U64 * scale, "mask %d band %d level %d"
                          % (mask, k, l))
        np.testing.assert_array_equal(h.bands(l, torch.float32), got.astype(np.float32))
        n = N * N
        offs = offsets(N)
        for k in range(9):
            p = np.arange(n)
            q = p + offs[k]
            ok = (q >= 0) & (q < n)
            np.testing.assert_array_equal(got[k][p[ok]], got[8 - k][q[ok]])
        # Dirichlet rows are identity rows; Neumann rows keep their full
        # stencil and so sum to zero (constants lie in the Neumann kernel)
        dn = dirichlet_nodes(N, mask)
        assert np.all(got[4][dn] == 1.0)
        assert np.all(got[[0, 1, 2, 3, 5, 6, 7, 8]][:, dn] == 0.0)
        ii = np.tile(np.arange(N), N)
        jj = np.repeat(np.arange(N), N)
        touch = np.zeros(n, dtype=bool)
        for k in range(9):
            di, dj = k % 3 - 1, k // 3 - 1
            inside = (ii + di >= 0) & (ii + di < N) & (jj + dj >= 0) & (jj + dj < N)
            nb = np.where(inside, (jj + dj) * N + (ii + di), 0)
            touch |= inside & dn[nb] & (k != 4)
        free_rows = ~dn & ~touch
        rs = got.sum(axis=0)[free_rows]
        assert np.all(np.abs(rs) <= 64 * U64 * scale[free_rows])


@pytest.mark.parametrize("mask", MASKS + [15])
def test_device_rhs_uniform_equals_host_generator(mg, ctx, mask):
    L = 7
    h = mg.Hierarchy(ctx, L, jitter=0.1, seed=2, dirichlet_sides=mask)
    b = torch.empty(h.n, dtype=torch.float64, device="cuda")
    h.rhs_uniform(4242, b)
    np.testing.assert_array_equal(host(b), synth.rhs_uniform(L, 4242, mask))


@pytest.mark.parametrize("mask", MASKS)
@pytest.mark.parametrize("L", [2, 5, 9])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_restrict(mg, ctx, orc, mask, L, dtype):
    h = mg.Hierarchy(ctx, L, dirichlet_sides=mask)
    Nf, Nc = (1 << L) + 1, (1 << (L - 1)) + 1
    rng = np.random.default_rng(L + mask)
    np_dt = np.float64 if dtype == torch.float64 else np.float32
    u = U64 if dtype == torch.float64 else U32
    d = rng.standard_normal(Nf * Nf).astype(np_dt).astype(np.float64)
    bc = torch.empty(Nc * Nc, dtype=dtype, device="cuda")
    h.restrict(L, dev(d, dtype), bc)
    ref = orc.restrict(Nf, d, dmask=mask)
    sc = orc.restrict(Nf, np.abs(d), dmask=mask)
    # nine weighted terms (weights powers of two) summed in different orders
    # on the two sides: each within gamma_8 of the exact sum, so 16 u apart
    assert_within(host(bc), ref, 16 * u * sc, "restrict mask %d" % mask)


@pytest.mark.parametrize("mask", MASKS)
@pytest.mark.parametrize("Lc", [1, 2, 3, 4])
def test_coarse_direct_solve(mg, ctx, orc, mask, Lc):
    L = max(Lc, 4)
    h = mg.Hierarchy(ctx, L, coarse_level=Lc, jitter=0.2, seed=5, dirichlet_sides=mask)
    oh = orc.Hierarchy(L, synth.coords(L, 0.2, 5), Lc=Lc, dmask=mask)
    Nc = (1 << Lc) + 1
    A = oh.bands(Lc)
    b = synth.rhs_uniform(Lc, 9, mask).astype(np.float32).astype(np.float64)
    x = torch.zeros(Nc * Nc, dtype=torch.float64, device="cuda")
    h.coarse_solve(dev(b), x)
    xh = host(x)
    r = orc.defect(Nc, A, b, xh)
    assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(b), np.linalg.norm(r)
    assert np.all(xh[dirichlet_nodes(Nc, mask)] == 0.0)
    # the FP32 variant solves in FP64 and rounds once: the FP64 result rounded
    x32 = torch.zeros(Nc * Nc, dtype=torch.float32, device="cuda")
    h.coarse_solve(dev(b, torch.float32), x32)
    np.testing.assert_array_equal(host(x32), xh.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("mask", MASKS)
@pytest.mark.parametrize("L,a", [(3, 0.0), (6, 0.2), (9, 0.2)])
def test_vcycle_fp64_matches_oracle(mg, ctx, orc, mask, L, a):
    seed = 310 + L
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed, dirichlet_sides=mask)
    oh = orc.Hierarchy(L, synth.coords(L, a, seed), Lc=1, dmask=mask)
    b = synth.rhs_uniform(L, 7, mask)
    x0 = np.random.default_rng(3).standard_normal(b.size) * 0.1
    x0[~synth.free_mask(L, mask)] = 0.0
    xd = dev(x0)
    h.vcycle(L, dev(b), xd)
    ref = oh.vcycle(L, x0, b)
    err = np.linalg.norm(host(xd) - ref) / np.linalg.norm(ref)
    assert err <= 1e-13, err


@pytest.mark.parametrize("mask", MASKS)
@pytest.mark.parametrize("L,a", [(2, 0.0), (5, 0.2), (9, 0.25), (11, 0.2)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fused_cycle_equals_unfused_bitwise(mg, ctx, mask, L, a, dtype):
    h = mg.Hierarchy(ctx, L, jitter=a, seed=40 + L, dirichlet_sides=mask)
    b = dev(synth.rhs_uniform(L, 8, mask), dtype)
    x0 = np.random.default_rng(L).standard_normal(h.n) * 0.1
    x0[~synth.free_mask(L, mask)] = 0.0
    xf = dev(x0, dtype)
    xu = dev(x0, dtype)
    h.vcycle(L, b, xf, fused=True)
    h.vcycle(L, b, xu, fused=False)
    np.testing.assert_array_equal(host(xf), host(xu))


@pytest.mark.parametrize("mask", [5, 12])
@pytest.mark.parametrize("L,a", [(6, 0.2), (10, 0.2)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fused_pre_pass_matches_oracle(mg, ctx, orc, mask, L, a, dtype):
    """The pre pass on a mixed problem: two sweeps, defect, and the
    restriction whose coarse Neumann-side entries collect the defect of the
    fine nodes on that side."""
    h = mg.Hierarchy(ctx, L, jitter=a, seed=60 + L, dirichlet_sides=mask)
    N, Nc = (1 << L) + 1, (1 << (L - 1)) + 1
    np_dt = np.float64 if dtype == torch.float64 else np.float32
    u = U64 if dtype == torch.float64 else U32
    bands = h.bands(L, dtype).astype(np.float64)
    rng = np.random.default_rng(L + 17)
    free = synth.free_mask(L, mask)
    x = np.where(free, rng.standard_normal(N * N), 0.0).astype(np_dt).astype(np.float64)
    b = np.where(free, rng.standard_normal(N * N), 0.0).astype(np_dt).astype(np.float64)
    om = float(np_dt(0.7))
    x2 = torch.empty(N * N, dtype=dtype, device="cuda")
    bc = torch.empty(Nc * Nc, dtype=dtype, device="cuda")
    h.pre_smooth(L, dev(b, dtype), dev(x, dtype), x2, bc, omega=om)
    x2r = orc.jacobi(N, bands, b, orc.jacobi(N, bands, b, x, om), om)
    assert_within(host(x2), x2r, 64 * u * (np.max(np.abs(x2r)) + np.max(np.abs(b))), "pre x2")
    bcr = orc.restrict(N, orc.defect(N, bands, b, host(x2)), dmask=mask)
    sc = orc.restrict(N, np.abs(b) + abs_band_product(N, bands, host(x2)), dmask=mask)
    assert_within(host(bc), bcr, 16 * u * sc, "pre restriction")
    # the coarse Neumann sides carry nonzero restricted defects
    side = ~dirichlet_nodes(Nc, mask) & ~synth.interior_mask(L - 1)
    assert np.count_nonzero(host(bc)[side]) > 0


def _solve(mg, h, b, **kw):
    x = torch.zeros(b.numel(), dtype=torch.float64, device="cuda")
    st = h.solve(b, x, mg.default_opts(**kw))
    return host(x), st


@pytest.mark.parametrize("mask", MASKS)
@pytest.mark.parametrize("L", [8, 10])
def test_fp64_solve_matches_oracle_at_equal_cycles(mg, ctx, orc, mask, L):
    a, seed = 0.2, 1002
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed, dirichlet_sides=mask)
    oh = orc.Hierarchy(L, synth.coords(L, a, seed), Lc=1, dmask=mask)
    bh = synth.rhs_uniform(L, 2002, mask)
    xo, sto = oh.solve_fp64(bh, o=orc.opts(rel_tol=1e-8))
    assert sto.status == 0
    x, st = _solve(mg, h, dev(bh), rel_tol=1e-8)
    assert st.status == 0 and st.rel_res <= 1e-8
    assert abs(st.cycles - sto.cycles) <= 1
    xf, stf = _solve(mg, h, dev(bh), fixed_cycles=sto.cycles)
    assert np.linalg.norm(xf - xo) <= 1e-10 * np.linalg.norm(xo)
    np.testing.assert_allclose(stf.hist(), orc.hist(sto), rtol=1e-6)


@pytest.mark.parametrize("mask", MASKS)
def test_mixed_solve_reaches_1e8(mg, ctx, orc, mask):
    L, a, seed = 10, 0.2, 1002
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed, dirichlet_sides=mask)
    oh = orc.Hierarchy(L, synth.coords(L, a, seed), Lc=1, dmask=mask)
    bh = synth.rhs_uniform(L, 2002, mask)
    x, st = _solve(mg, h, dev(bh), rel_tol=1e-8, precision=mg.MG_PREC_MIXED)
    assert st.status == 0 and st.rel_res <= 1e-8
    N = (1 << L) + 1
    r = orc.norm2(orc.defect(N, oh.bands(L), bh, x)) / orc.norm2(bh)
    assert r <= 1.01e-8, r
    xo, _ = oh.solve_fp64(bh, o=orc.opts(rel_tol=1e-12))
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-6
    _, ste = oh.solve_mixed_emulated(bh, o=orc.opts(rel_tol=1e-8))
    assert abs(st.outer_steps - ste.outer_steps) <= 1


@pytest.mark.parametrize("mask,fn", [(12, 2), (5, 3)])
def test_manufactured_solution_error_matches_oracle(mg, ctx, orc, mask, fn):
    """u = cos(pi x) sin(pi y) (Dirichlet at y = 0, 1; Neumann at x = 0, 1)
    and u = sin(pi x / 2) sin(pi y / 2) (Dirichlet at x = 0 and y = 0;
    Neumann at x = 1 and y = 1): the device solution has the oracle's
    discretisation error, and that error falls by about four per level."""
    errs = []
    for L in (5, 6, 7):
        N = (1 << L) + 1
        xy = synth.coords(L)
        h = mg.Hierarchy(ctx, L, dirichlet_sides=mask)
        oh = orc.Hierarchy(L, xy, Lc=1, dmask=mask)
        b = orc.load_vector(N, xy, fn=fn, dmask=mask)
        x, st = _solve(mg, h, dev(b), rel_tol=1e-12)
        assert st.status == 0
        xo, _ = oh.solve_fp64(b, o=orc.opts(rel_tol=1e-12))
        e_gpu = orc.l2_error(N, xy, x, fn)
        e_or = orc.l2_error(N, xy, xo, fn)
        assert abs(e_gpu - e_or) <= 1e-6 * e_or
        errs.append(e_gpu)
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.5 <= e0 / e1 <= 4.5, errs


def test_batch_of_mixed_problems_equals_single_solves(mg, ctx):
    levels = [5, 7, 8, 6, 9, 4]
    masks = [1, 5, 12, 14, 15, 3]
    probs = []
    for k, (L, m) in enumerate(zip(levels, masks)):
        h = mg.Hierarchy(ctx, L, jitter=0.2, seed=700 + k, dirichlet_sides=m)
        b = torch.empty(h.n, dtype=torch.float64, device="cuda")
        h.rhs_uniform(800 + k, b)
        probs.append((h, b))
    opts = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-8)
    xs = [torch.zeros_like(b) for _, b in probs]
    stats = mg.solve_batch([p[0] for p in probs], [p[1] for p in probs], xs, opts)
    for k, (h, b) in enumerate(probs):
        x1 = torch.zeros_like(b)
        s1 = h.solve(b, x1, opts)
        assert stats[k].status == 0 and stats[k].rel_res <= 1e-8
        assert (stats[k].cycles, stats[k].outer_steps) == (s1.cycles, s1.outer_steps)
        np.testing.assert_array_equal(host(xs[k]), host(x1))
    for h, _ in probs:
        h.close()


def test_mask_arguments_checked(mg, ctx):
    for bad in (0, 16, -1):
        with pytest.raises(mg.MgError):
            mg.Hierarchy(ctx, 4, dirichlet_sides=bad)
    h = mg.Hierarchy(ctx, 4, dirichlet_sides=5)
    b = torch.empty(h.n, dtype=torch.float64, device="cuda")
    with pytest.raises(mg.MgError):
        h.rhs_sinsin(b)
    h.close()
