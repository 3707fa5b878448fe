"""Multigrid-preconditioned CG on the GPU (Sec. 4.1: a solver plugged into
another as its preconditioner; the V(2,2) cycle of Sec. 6.2) against the
oracle's preconditioned CG.

The device and the oracle sum their dot products in different orders, so
iterates agree to rounding amplified by the few CG steps compared (a
fixed number of steps, so no stop decision sits on a rounding boundary).
"""
import numpy as np
import pytest

import synth

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


def _solve(mg, h, b, x0=None, **kw):
    x = torch.zeros(b.numel(), dtype=torch.float64, device="cuda") if x0 is None else x0.clone()
    st = h.solve(b, x, mg.default_opts(**kw))
    return host(x), st


@pytest.mark.parametrize("L,mask", [(6, 15), (9, 15), (9, 5)])
@pytest.mark.parametrize("mixed", [False, True])
def test_pcg_steps_match_oracle(mg, ctx, orc, L, mask, mixed):
    a, seed = 0.2, 400 + L
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed, dirichlet_sides=mask)
    oh = orc.Hierarchy(L, synth.coords(L, a, seed), dmask=mask)
    bh = synth.rhs_uniform(L, 33, mask)
    prec = mg.MG_PREC_MIXED if mixed else mg.MG_PREC_FP64
    for k in (1, 2, 4):
        x, st = _solve(mg, h, dev(bh), krylov=1, precision=prec, fixed_cycles=k)
        xo, sto = oh.solve_pcg(bh, o=orc.opts(fixed_cycles=k), precond32=mixed)
        assert st.status == 0 and st.cycles == k == sto.cycles
        # FP64 cycle: rounding-level agreement; FP32 cycle: the preconditioner
        # itself differs at FP32 rounding between the two sides, which CG
        # passes on to the iterate at about that level
        tol = 1e-6 if mixed else 1e-11
        assert np.linalg.norm(x - xo) <= tol * np.linalg.norm(xo), (k, np.linalg.norm(x - xo))
        np.testing.assert_allclose(st.hist(), orc.hist(sto), rtol=100 * tol)
        assert abs(st.rel_res - sto.rel_res) <= 100 * tol * sto.rel_res


@pytest.mark.parametrize("L", [8, 10])
@pytest.mark.parametrize("mixed", [False, True])
def test_pcg_reaches_1e8(mg, ctx, orc, L, mixed):
    a, seed = 0.2, 1002
    h = mg.Hierarchy(ctx, L, jitter=a, seed=seed)
    oh = orc.Hierarchy(L, synth.coords(L, a, seed))
    bh = synth.rhs_uniform(L, 2002)
    prec = mg.MG_PREC_MIXED if mixed else mg.MG_PREC_FP64
    x, st = _solve(mg, h, dev(bh), krylov=1, precision=prec, rel_tol=1e-8)
    assert st.status == 0 and st.rel_res <= 1.05e-8
    _, sto = oh.solve_pcg(bh, o=orc.opts(rel_tol=1e-8), precond32=mixed)
    assert abs(st.cycles - sto.cycles) <= 1
    N = (1 << L) + 1
    r = orc.norm2(orc.defect(N, oh.bands(L), bh, x)) / orc.norm2(bh)
    assert abs(r - st.rel_res) <= 1e-3 * r
    # fewer steps than plain multigrid cycles
    _, smg = _solve(mg, h, dev(bh), rel_tol=1e-8)
    assert st.cycles < smg.cycles
    xo, _ = oh.solve_fp64(bh, o=orc.opts(rel_tol=1e-12))
    assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)


def test_pcg_graph_replay_equals_direct_launches(mg, ctx):
    L = 8
    h = mg.Hierarchy(ctx, L, jitter=0.2, seed=3)
    b = dev(synth.rhs_uniform(L, 4))
    for prec in (mg.MG_PREC_FP64, mg.MG_PREC_MIXED):
        xg, sg = _solve(mg, h, b, krylov=1, precision=prec, use_graph=1)
        xe, se = _solve(mg, h, b, krylov=1, precision=prec, use_graph=0)
        np.testing.assert_array_equal(xg, xe)
        assert sg.cycles == se.cycles and sg.rel_res == se.rel_res
        # and again from the cached graph
        xg2, _ = _solve(mg, h, b, krylov=1, precision=prec, use_graph=1)
        np.testing.assert_array_equal(xg2, xg)


def test_pcg_with_other_cycles_and_coarse_cg(mg, ctx, orc):
    L = 7
    h = mg.Hierarchy(ctx, L, coarse_level=3, jitter=0.2, seed=8, dirichlet_sides=12)
    oh = orc.Hierarchy(L, synth.coords(L, 0.2, 8), Lc=3, dmask=12)
    bh = synth.rhs_uniform(L, 9, 12)
    # V(1,1) runs the unfused cycle
    x, st = _solve(mg, h, dev(bh), krylov=1, nu_pre=1, nu_post=1, rel_tol=1e-9)
    assert st.status == 0 and st.rel_res <= 1.05e-9
    _, sto = oh.solve_pcg(bh, o=orc.opts(nu_pre=1, nu_post=1, rel_tol=1e-9))
    assert abs(st.cycles - sto.cycles) <= 1
    # with the CG coarse solver
    h.set_coarse_solver(mg.MG_COARSE_CG, tol=1e-12, max_iter=200)
    x2, st2 = _solve(mg, h, dev(bh), krylov=1, rel_tol=1e-9)
    assert st2.status == 0 and st2.rel_res <= 1.05e-9
    xo, _ = oh.solve_fp64(bh, o=orc.opts(rel_tol=1e-12))
    assert np.linalg.norm(x2 - xo) <= 1e-7 * np.linalg.norm(xo)


def test_pcg_warm_start_zero_rhs_and_limits(mg, ctx):
    L = 6
    h = mg.Hierarchy(ctx, L, jitter=0.1, seed=1)
    b = dev(synth.rhs_uniform(L, 2))
    x, st = _solve(mg, h, b, krylov=1, rel_tol=1e-10)
    assert st.status == 0
    x2, st2 = _solve(mg, h, b, x0=dev(x), krylov=1, rel_tol=1e-8)
    assert st2.status == 0 and st2.cycles == 0
    z, sz = _solve(mg, h, torch.zeros_like(b), krylov=1)
    assert sz.status == 0 and not z.any()
    xn = torch.zeros_like(b)
    sn = h.solve(b, xn, mg.default_opts(krylov=1, rel_tol=1e-14, max_cycles=2),
                 raise_on_error=False)
    assert sn.status == mg.MG_ERR_NOCONV and sn.cycles == 2
    with pytest.raises(mg.MgError):
        _solve(mg, h, b, krylov=2)
    xs = [torch.zeros_like(b)]
    with pytest.raises(mg.MgError):
        mg.solve_batch([h], [b], xs, mg.default_opts(precision=mg.MG_PREC_MIXED, krylov=1))
