"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every comparison runs both sides on the same seeded inputs.  FP64 band
operations must agree within a forward-error bound of the 9-term sums
(gamma = 12 u_64 times sum |a||x|); FP32 operations are compared with the
oracle's FP64 evaluation of the same FP32 inputs within 12 u_32 times the
same scale.  Assembly is compared within 64 FP64 ulps of the row scale.
Sizes span L = 1 (9 unknowns, less than one tile) to L = 10 (1,050,625
unknowns: many tiles and an odd, ragged tail), plus sampled checks at the
full L = 12 workload.
"""
import numpy as np
import pytest

import synth
from gpu_common import U32, U64, abs_band_product, assert_within, offsets

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


_ORACLE_CACHE = {}


def oracle_hier(orc, L, a, seed, Lc=1):
    key = (L, a, seed, Lc)
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = orc.Hierarchy(L, synth.coords(L, a, seed), Lc=Lc)
    return _ORACLE_CACHE[key]


# ------------------------------------------------------------------ geometry


@pytest.mark.parametrize("L,a,seed", [(6, 0.2, 1002), (9, 0.25, 77)])
def test_device_jitter_equals_host_generator(mg, ctx, L, a, seed):
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed, assemble=False)
    got = h.coords(L)
    ref = synth.coords(L, a, seed).reshape(-1)
    np.testing.assert_array_equal(got, ref)
    # coarse levels are the fine coordinates sampled every 2^(L-l) nodes
    N = (1 << L) + 1
    c3 = h.coords(3).reshape(9, 9, 2)
    s = 1 << (L - 3)
    np.testing.assert_array_equal(c3, ref.reshape(N, N, 2)[::s, ::s])


# ------------------------------------------------------------------ assembly


@pytest.mark.parametrize("L,a,seed", [(5, 0.0, 0), (8, 0.2, 1002), (7, 0.25, 4100)])
def test_assembled_bands_match_oracle(mg, ctx, orc, L, a, seed):
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed)
    oh = oracle_hier(orc, L, a, seed)
    for l in range(1, L + 1):
        N = (1 << l) + 1
        ref = oh.bands(l)
        got = h.bands(l)
        # each entry sums up to 16 quadrature terms whose own evaluation (map
        # derivatives, cofactors, division by det J) costs ~10 roundings on
        # either side: 64 u times the row scale bounds the difference
        scale = np.max(np.abs(ref), axis=0)
        for k in range(9):
            assert_within(got[k], ref[k], 64 * U64 * scale, "band %d level %d" % (k, l))
        # FP32 copy is the round-to-nearest image of the FP64 bands
        got32 = h.bands(l, torch.float32)
        np.testing.assert_array_equal(got32, got.astype(np.float32))
        # symmetry: A[p][q] == A[q][p] bitwise (same element terms, same order)
        n = N * N
        offs = offsets(N)
        for k in range(9):
            p = np.arange(n)
            q = p + offs[k]
            ok = (q >= 0) & (q < n)
            np.testing.assert_array_equal(got[k][p[ok]], got[8 - k][q[ok]])


# ------------------------------------------------------------------ band ops


CASES = [(1, 0.0), (2, 0.25), (4, 0.2), (7, 0.2), (10, 0.2)]


@pytest.mark.parametrize("L,a", CASES)
def test_spmv_defect_jacobi_fp64(mg, ctx, orc, L, a):
    seed = 100 + L
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed)
    N = (1 << L) + 1
    bands = h.bands(L)  # the device operator; assembly parity is tested separately
    rng = np.random.default_rng(L)
    x = rng.standard_normal(N * N)
    b = rng.standard_normal(N * N)
    scale = abs_band_product(N, bands, x)
    xd, bd = dev(x), dev(b)
    y = torch.empty_like(xd)
    h.spmv(L, xd, y)
    assert_within(host(y), orc.spmv(N, bands, x), 12 * U64 * scale + 1e-300, "spmv64")
    d = torch.empty_like(xd)
    nrm = h.defect(L, bd, xd, d, norm=True)
    dref = orc.defect(N, bands, b, x)
    assert_within(host(d), dref, 12 * U64 * (scale + np.abs(b)), "defect64")
    assert abs(nrm - orc.norm2(dref)) <= 1e-13 * orc.norm2(dref)
    # norm-only variant (no d written)
    assert abs(h.defect(L, bd, xd, None, norm=True) - nrm) == 0.0
    xs = xd.clone()
    h.smooth(L, bd, xs, sweeps=1, omega=0.7)
    jref = orc.jacobi(N, bands, b, x, 0.7)
    diag = np.abs(bands[4])
    bound = 12 * U64 * (np.abs(x) + 0.7 * (scale + np.abs(b)) / diag)
    assert_within(host(xs), jref, bound, "jacobi64")
    xo = torch.empty_like(xd)
    h.jacobi(L, bd, xd, xo, 0.7)  # the single-kernel sweep
    np.testing.assert_array_equal(host(xo), host(xs))


@pytest.mark.parametrize("L,a", CASES)
def test_spmv_defect_jacobi_fp32(mg, ctx, orc, L, a):
    seed = 200 + L
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed)
    N = (1 << L) + 1
    b32 = h.bands(L, torch.float32)  # RNE of the device FP64 bands
    bands = b32.astype(np.float64)
    rng = np.random.default_rng(L + 50)
    x = rng.standard_normal(N * N).astype(np.float32).astype(np.float64)
    b = rng.standard_normal(N * N).astype(np.float32).astype(np.float64)
    scale = abs_band_product(N, bands, x)
    xd, bd = dev(x, torch.float32), dev(b, torch.float32)
    y = torch.empty_like(xd)
    h.spmv(L, xd, y)
    assert_within(host(y), orc.spmv(N, bands, x), 12 * U32 * scale, "spmv32")
    d = torch.empty_like(xd)
    h.defect(L, bd, xd, d)
    assert_within(host(d), orc.defect(N, bands, b, x), 12 * U32 * (scale + np.abs(b)),
                  "defect32")
    xs = xd.clone()
    h.smooth(L, bd, xs, sweeps=1, omega=0.7)
    jref = orc.jacobi(N, bands, b, x, float(np.float32(0.7)))
    bound = 16 * U32 * (np.abs(x) + 0.7 * (scale + np.abs(b)) / np.abs(bands[4]))
    assert_within(host(xs), jref, bound, "jacobi32")
    xo = torch.empty_like(xd)
    h.jacobi(L, bd, xd, xo, 0.7)
    np.testing.assert_array_equal(host(xo), host(xs))


@pytest.mark.parametrize("L", [2, 5, 9])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_restrict_prolong(mg, ctx, orc, L, dtype):
    h = mg.Hierarchy(ctx, L)
    Nf, Nc = (1 << L) + 1, (1 << (L - 1)) + 1
    rng = np.random.default_rng(L)
    np_dt = np.float64 if dtype == torch.float64 else np.float32
    u = U64 if dtype == torch.float64 else U32
    d = rng.standard_normal(Nf * Nf).astype(np_dt).astype(np.float64)
    xc = rng.standard_normal(Nc * Nc).astype(np_dt).astype(np.float64)
    xc[~synth.interior_mask(L - 1)] = 0.0  # coarse corrections vanish on the boundary
    xf = rng.standard_normal(Nf * Nf).astype(np_dt).astype(np.float64)
    bc = torch.empty(Nc * Nc, dtype=dtype, device="cuda")
    h.restrict(L, dev(d, dtype), bc)
    ref = orc.restrict(Nf, d, filter=True)
    sc = orc.restrict(Nf, np.abs(d), filter=True)
    # nine weighted terms (weights powers of two) summed in different orders
    # on the two sides: each within gamma_8 of the exact sum, so 16 u apart
    assert_within(host(bc), ref, 16 * u * sc, "restrict")
    xfd = dev(xf, dtype)
    h.prolong(L, dev(xc, dtype), xfd)
    ref = orc.prolong_add(Nf, xc, xf)
    sc = orc.prolong_add(Nf, np.abs(xc), np.abs(xf))
    assert_within(host(xfd), ref, 4 * u * sc, "prolong")


@pytest.mark.parametrize("Lc", [1, 2, 3, 4])
def test_coarse_direct_solve(mg, ctx, orc, Lc):
    L = max(Lc, 4)
    h = mg.Hierarchy(ctx, L, coarse_level=Lc, jitter=0.2, seed=5)
    oh = oracle_hier(orc, L, 0.2, 5, Lc=Lc)
    Nc = (1 << Lc) + 1
    A = oh.bands(Lc)
    b = synth.rhs_uniform(Lc, 9)
    x = torch.zeros(Nc * Nc, dtype=torch.float64, device="cuda")
    h.coarse_solve(dev(b), x)
    # x solves the coarse system: residual at rounding level
    r = orc.defect(Nc, A, b, host(x))
    assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(b)


# ------------------------------------------------------------------ cycles and solves


@pytest.mark.parametrize("L,a", [(3, 0.0), (6, 0.2), (9, 0.2)])
def test_vcycle_fp64_matches_oracle(mg, ctx, orc, L, a):
    seed = 300 + L
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed)
    oh = oracle_hier(orc, L, a, seed)
    b = synth.rhs_uniform(L, 7)
    x0 = np.random.default_rng(3).standard_normal(b.size) * 0.1
    x0[~synth.interior_mask(L)] = 0.0
    xd = dev(x0)
    h.vcycle(L, dev(b), xd)
    ref = oh.vcycle(L, x0, b)
    err = np.linalg.norm(host(xd) - ref) / np.linalg.norm(ref)
    assert err <= 1e-13, err


def _solve(mg, h, b, **kw):
    x = torch.zeros(b.numel(), dtype=torch.float64, device="cuda")
    st = h.solve(b, x, mg.default_opts(**kw))
    return host(x), st


def test_config0_fp64_sinsin_L6(mg, ctx, orc):
    """Plain FP64, uniform 65x65 grid, f = 2 pi^2 sin sin, V(2,2), omega 0.7,
    3x3 coarse direct solve, 1e-8 relative residual."""
    L = 6
    N = 65
    h = mg.Hierarchy(ctx, L)
    b = torch.empty(N * N, dtype=torch.float64, device="cuda")
    h.rhs_sinsin(b)
    bh = host(b)
    bref = orc.load_vector(N, synth.coords(L), fn=0)
    assert_within(bh, bref, 64 * U64 * np.max(np.abs(bref)), "load vector")
    oh = oracle_hier(orc, L, 0.0, 0)
    xo, sto = oh.solve_fp64(bref, o=orc.opts(rel_tol=1e-8))
    x, st = _solve(mg, h, b, rel_tol=1e-8)
    assert st.status == 0 and st.rel_res <= 1e-8
    assert st.cycles == sto.cycles
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
    # discretisation error as in the oracle
    e_gpu = orc.l2_error_sinsin(N, synth.coords(L), x)
    e_or = orc.l2_error_sinsin(N, synth.coords(L), xo)
    assert abs(e_gpu - e_or) <= 1e-8 * e_or


@pytest.mark.parametrize("L,a,seed", [(8, 0.2, 1002), (10, 0.2, 1002)])
def test_fp64_solve_matches_oracle_at_equal_cycles(mg, ctx, orc, L, a, seed):
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed)
    oh = oracle_hier(orc, L, a, seed)
    bh = synth.rhs_uniform(L, 2002)
    xo, sto = oh.solve_fp64(bh, o=orc.opts(rel_tol=1e-8))
    assert sto.status == 0
    x, st = _solve(mg, h, dev(bh), rel_tol=1e-8)
    assert st.status == 0 and st.rel_res <= 1e-8
    assert abs(st.cycles - sto.cycles) <= 1
    xf, stf = _solve(mg, h, dev(bh), fixed_cycles=sto.cycles)
    assert stf.cycles == sto.cycles
    assert np.linalg.norm(xf - xo) <= 1e-10 * np.linalg.norm(xo)
    # residual history agrees cycle by cycle
    np.testing.assert_allclose(stf.hist(), orc.hist(sto), rtol=1e-6)


@pytest.mark.parametrize("L,a,seed", [(7, 0.2, 11), (10, 0.2, 1002)])
def test_mixed_solve_reaches_1e8(mg, ctx, orc, L, a, seed):
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed)
    oh = oracle_hier(orc, L, a, seed)
    bh = synth.rhs_uniform(L, 2002)
    x, st = _solve(mg, h, dev(bh), rel_tol=1e-8, precision=mg.MG_PREC_MIXED)
    assert st.status == 0 and st.rel_res <= 1e-8
    # independent check of the residual with the oracle's operator
    N = (1 << L) + 1
    r = orc.norm2(orc.defect(N, oh.bands(L), bh, x)) / orc.norm2(bh)
    assert r <= 1.01e-8, r
    # error against the FP64 oracle solution, stated per result
    xo, _ = oh.solve_fp64(bh, o=orc.opts(rel_tol=1e-12))
    rel_err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print("L=%d mixed: outer %d inner %d relres %.3e error vs FP64 oracle %.3e"
          % (L, st.outer_steps, st.cycles, st.rel_res, rel_err))
    assert rel_err <= 1e-6
    # the emulated mixed oracle needs a similar amount of work
    _, ste = oh.solve_mixed_emulated(bh, o=orc.opts(rel_tol=1e-8))
    assert abs(st.outer_steps - ste.outer_steps) <= 1


def test_graph_replay_equals_direct_launches(mg, ctx):
    L = 8
    h = mg.Hierarchy(ctx, L, jitter=0.2, seed=3)
    b = dev(synth.rhs_uniform(L, 4))
    for prec in (mg.MG_PREC_FP64, mg.MG_PREC_MIXED):
        xg, sg = _solve(mg, h, b, precision=prec, use_graph=1)
        xe, se = _solve(mg, h, b, precision=prec, use_graph=0)
        xg2, _ = _solve(mg, h, b, precision=prec, use_graph=1)
        np.testing.assert_array_equal(xg, xe)
        np.testing.assert_array_equal(xg, xg2)
        assert sg.cycles == se.cycles


def test_warm_start_and_zero_rhs(mg, ctx):
    L = 6
    h = mg.Hierarchy(ctx, L, jitter=0.1, seed=1)
    b = dev(synth.rhs_uniform(L, 5))
    x, st = _solve(mg, h, b, rel_tol=1e-10)
    xw = dev(x)
    st2 = h.solve(b, xw, mg.default_opts(rel_tol=1e-10))
    assert st2.cycles == 0 and st2.rel_res <= 1e-10
    z = torch.zeros_like(b)
    xz = torch.ones_like(b)
    st3 = h.solve(z, xz, mg.default_opts())
    assert st3.status == 0 and torch.count_nonzero(xz).item() == 0


def test_level_one_is_a_direct_solve(mg, ctx, orc):
    h = mg.Hierarchy(ctx, 1)
    b = np.zeros(9)
    b[4] = 1.0
    x, st = _solve(mg, h, dev(b), rel_tol=1e-12)
    assert st.cycles == 1 and st.rel_res < 1e-15
    A = orc.assemble(3, synth.coords(1))
    assert abs(x[4] - 1.0 / A[4][4]) < 1e-16


def test_error_paths(mg, ctx):
    with pytest.raises(mg.MgError) as e:
        mg.Hierarchy(ctx, 15)
    assert e.value.status == mg.MG_ERR_INVALID
    with pytest.raises(mg.MgError) as e:
        mg.Hierarchy(ctx, 4, coarse_level=5)
    assert e.value.status == mg.MG_ERR_INVALID
    h = mg.Hierarchy(ctx, 6, jitter=0.2, seed=2)
    b = dev(synth.rhs_uniform(6, 1))
    x = torch.zeros_like(b)
    st = h.solve(b, x, mg.default_opts(rel_tol=1e-14, max_cycles=1), raise_on_error=False)
    assert st.status == mg.MG_ERR_NOCONV and st.cycles == 1
    bn = b.clone()
    bn[100] = float("nan")
    st = h.solve(bn, x, mg.default_opts(), raise_on_error=False)
    assert st.status == mg.MG_ERR_NUMERIC
    with pytest.raises(mg.MgError) as e:
        h.spmv(9, b, x)
    assert e.value.status == mg.MG_ERR_INVALID


def test_budget_exhaustion_is_clean(mg):
    need = mg.Hierarchy.bytes_needed(9)
    c = mg.Context(0, budget_bytes=need + mg.Hierarchy.bytes_needed(5))
    h1 = mg.Hierarchy(c, 9, assemble=False)
    with pytest.raises(mg.MgError) as e:
        mg.Hierarchy(c, 9, assemble=False)
    assert e.value.status == mg.MG_ERR_NOMEM
    assert c.memory()[0] == need
    h1.close()
    assert c.memory()[0] == 0
    h2 = mg.Hierarchy(c, 9, assemble=False)  # the freed budget is usable again
    h2.close()


# ------------------------------------------------------------------ full-size workload


def test_full_size_L12_spmv_and_mixed_solve(mg, ctx, orc):
    """L = 12 (16,785,409 unknowns), jitter 0.2 h, Gaussian RHS: the FP32 and
    FP64 band products at full size against the oracle's operator, and the
    mixed solve's residual checked independently on the host."""
    L, N = 12, 4097
    xy = synth.coords(L, 0.2, 1003)
    h = mg.Hierarchy(ctx, L, jitter=0.2, seed=1003)
    dbands = h.bands(L)
    rng = np.random.default_rng(12)
    idx = rng.integers(0, N * N, size=200000)
    x = rng.standard_normal(N * N)
    xd = dev(x)
    y = torch.empty_like(xd)
    h.spmv(L, xd, y)
    yr = orc.spmv(N, dbands, x)
    scale = abs_band_product(N, dbands, x)
    assert_within(host(y)[idx], yr[idx], (12 * U64 * scale)[idx], "spmv64 L12")
    # the FP64 defect and its norm at full size (every row and strip tile)
    bvec = rng.standard_normal(N * N)
    d = torch.empty_like(xd)
    nrm = h.defect(L, dev(bvec), xd, d, norm=True)
    dref = orc.defect(N, dbands, bvec, x)
    assert_within(host(d)[idx], dref[idx], (12 * U64 * (scale + np.abs(bvec)))[idx],
                  "defect64 L12")
    assert abs(nrm - orc.norm2(dref)) <= 1e-13 * orc.norm2(dref)
    del dbands, yr, scale, dref, d
    x32 = x.astype(np.float32)
    y32 = torch.empty(N * N, dtype=torch.float32, device="cuda")
    h.spmv(L, dev(x32, torch.float32), y32)
    b32 = h.bands(L, torch.float32).astype(np.float64)
    x64 = x32.astype(np.float64)
    assert_within(host(y32)[idx], orc.spmv(N, b32, x64)[idx],
                  (12 * U32 * abs_band_product(N, b32, x64))[idx], "spmv32 L12")
    del b32
    bands = orc.assemble(N, xy)
    b = synth.rhs_gaussian(L, 2003)
    xs, st = _solve(mg, h, dev(b), precision=mg.MG_PREC_MIXED, rel_tol=1e-8)
    assert st.status == 0 and st.rel_res <= 1e-8
    r = orc.norm2(orc.defect(N, bands, b, xs)) / orc.norm2(b)
    assert r <= 1.05e-8, r


@pytest.mark.parametrize("L,a", [(2, 0.0), (5, 0.2), (9, 0.25), (11, 0.2)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fused_cycle_equals_unfused_bitwise(mg, ctx, L, a, dtype):
    """The fused smoothing passes (two sweeps + defect + restriction; 
    prolongation + two sweeps) perform each node's arithmetic exactly as the
    separate kernels do, so a V(2,2) cycle gives identical bits; L = 11 spans
    many strips and row chunks, L = 2 less than one tile."""
    h = mg.Hierarchy(ctx, L, jitter=a, seed=40 + L)
    n = h.n
    b = dev(synth.rhs_uniform(L, 8), dtype)
    x0 = np.random.default_rng(L).standard_normal(n) * 0.1
    x0[~synth.interior_mask(L)] = 0.0
    xf = dev(x0, dtype)
    xu = dev(x0, dtype)
    h.vcycle(L, b, xf, fused=True)
    h.vcycle(L, b, xu, fused=False)
    np.testing.assert_array_equal(host(xf), host(xu))
    # and from a zero iterate (first sweep from zero on the finest level too)
    st_f = h.solve(b.double(), torch.zeros(n, dtype=torch.float64, device="cuda"),
                   mg.default_opts(precision=mg.MG_PREC_MIXED, fixed_cycles=2))
    assert st_f.status == 0


@pytest.mark.parametrize("L,a", [(2, 0.0), (6, 0.2), (10, 0.2)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fused_passes_match_oracle(mg, ctx, orc, L, a, dtype):
    """Pre pass = two damped Jacobi sweeps, defect, restriction with boundary
    filter; post pass = prolongation/correction and two sweeps (+ residual
    norm); each against the oracle's operators on the device bands."""
    h = mg.Hierarchy(ctx, L, jitter=a, seed=60 + L)
    N, Nc = (1 << L) + 1, (1 << (L - 1)) + 1
    np_dt = np.float64 if dtype == torch.float64 else np.float32
    u = U64 if dtype == torch.float64 else U32
    bands = h.bands(L, dtype).astype(np.float64)
    rng = np.random.default_rng(L + 7)
    x = rng.standard_normal(N * N).astype(np_dt).astype(np.float64)
    b = rng.standard_normal(N * N).astype(np_dt).astype(np.float64)
    om = float(np_dt(0.7))
    # pre pass against oracle operators (FP64 evaluation of the same inputs)
    x2 = torch.empty(N * N, dtype=dtype, device="cuda")
    bc = torch.empty(Nc * Nc, dtype=dtype, device="cuda")
    h.pre_smooth(L, dev(b, dtype), dev(x, dtype), x2, bc, omega=om)
    x1 = orc.jacobi(N, bands, b, x, om)
    x2r = orc.jacobi(N, bands, b, x1, om)
    scale = np.max(np.abs(x2r)) + np.max(np.abs(b))
    assert_within(host(x2), x2r, 64 * u * scale, "pre x2")
    bcr = orc.restrict(N, orc.defect(N, bands, b, host(x2)), filter=True)
    sc = orc.restrict(N, np.abs(b) + abs_band_product(N, bands, host(x2)), filter=True)
    assert_within(host(bc), bcr, 16 * u * sc, "pre restriction")
    # from a zero iterate
    h.pre_smooth(L, dev(b, dtype), dev(x, dtype), x2, bc, x_zero=True, omega=om)
    x2z = orc.jacobi(N, bands, b, orc.jacobi(N, bands, b, np.zeros(N * N), om), om)
    assert_within(host(x2), x2z, 64 * u * (np.max(np.abs(x2z)) + np.max(np.abs(b))), "pre zero")
    # post pass
    xc = rng.standard_normal(Nc * Nc).astype(np_dt).astype(np.float64)
    xc[~synth.interior_mask(L - 1)] = 0.0
    xo = torch.empty(N * N, dtype=dtype, device="cuda")
    nrm = h.post_smooth(L, dev(b, dtype), dev(x, dtype), dev(xc, dtype), xo, omega=om, norm=True)
    xp = orc.prolong_add(N, xc, x)
    xr = orc.jacobi(N, bands, b, orc.jacobi(N, bands, b, xp, om), om)
    assert_within(host(xo), xr, 64 * u * (np.max(np.abs(xr)) + np.max(np.abs(b))), "post")
    dref = orc.norm2(orc.defect(N, bands, b, host(xo)))
    assert abs(nrm - dref) <= 64 * u * (orc.norm2(b) + orc.norm2(abs_band_product(N, bands, host(xo))))
