"""The start of a solve on the device.

A zero initial iterate (the usual start) makes the first defect b itself;
the solvers then form it from b alone with the defect kernel's tiles and
norm partials.  Its norm must be the same bits as the full defect kernel's
on x = 0 (mg_defect), including sizes whose last tile is partial, in the FP64
and in the mixed solver.  A nonzero initial iterate takes the full defect;
the mixed solver's warm start is checked with the oracle's operator.
"""
import numpy as np
import pytest

import synth
from gpu_common import U64, abs_band_product

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


FP64_TILE = 512  # rows of one FP64 defect tile (256 threads x 2 rows)


@pytest.mark.parametrize("L", [3, 5, 9, 12])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_zero_iterate_first_residual_is_the_defect_kernels(mg, ctx, L, prec):
    n = ((1 << L) + 1) ** 2
    if L in (3, 5, 9):
        assert n % FP64_TILE != 0  # the last tile is partial
    h = mg.Hierarchy(ctx, L, jitter=0.2, seed=1000 + L)
    b = torch.from_numpy(synth.rhs_uniform(L, 2000 + L)).cuda()
    zero = torch.zeros_like(b)
    r0 = h.defect(L, b, zero, norm=True)
    # a tolerance above 1 stops before the first cycle: the reported residual
    # is the first defect's norm over ||b||
    o = mg.default_opts(precision=mg.MG_PREC_FP64 if prec == "fp64" else mg.MG_PREC_MIXED,
                        rel_tol=10.0)
    x = torch.zeros_like(b)
    st = h.solve(b, x, o)
    assert st.status == 0 and st.cycles == 0 and st.outer_steps == 0
    assert st.rel_res == r0 / st.bnorm
    assert float(np.linalg.norm(x.cpu().numpy())) == 0.0
    h.close()


def test_zero_iterate_shortcut_does_not_change_the_solve(mg, ctx):
    """x0 = 0 (shortcut) and x0 = +0 written by hand are the same input: same
    bits; a tiny nonzero x0 takes the full defect and still converges."""
    L = 7
    h = mg.Hierarchy(ctx, L, jitter=0.2, seed=77)
    b = torch.from_numpy(synth.rhs_uniform(L, 78)).cuda()
    for prec in (mg.MG_PREC_FP64, mg.MG_PREC_MIXED):
        o = mg.default_opts(precision=prec, rel_tol=1e-8)
        x1 = torch.zeros_like(b)
        s1 = h.solve(b, x1, o)
        x2 = torch.full_like(b, 0.0)
        s2 = h.solve(b, x2, o)
        np.testing.assert_array_equal(x1.cpu().numpy(), x2.cpu().numpy())
        assert (s1.cycles, s1.outer_steps, s1.rel_res) == (s2.cycles, s2.outer_steps, s2.rel_res)
        x3 = torch.zeros_like(b)
        x3[h.n // 2] = 1e-300  # one nonzero entry: the full defect
        s3 = h.solve(b, x3, o)
        assert s3.status == 0 and s3.rel_res <= 1e-8
    h.close()


@pytest.mark.parametrize("L", [6, 10])
def test_mixed_warm_start_checked_by_oracle(mg, ctx, orc, L):
    """Mixed solve from a nonzero iterate (a partly converged FP64 solve plus
    noise): reaches 1e-8 by the oracle's operator, and its first reported
    residual equals the full defect kernel's on that iterate."""
    a, gs, rs = 0.2, 3000 + L, 4000 + L
    N = (1 << L) + 1
    h = mg.Hierarchy(ctx, L, jitter=a, seed=gs)
    bh = synth.rhs_uniform(L, rs)
    b = torch.from_numpy(bh).cuda()
    x = torch.zeros_like(b)
    h.solve(b, x, mg.default_opts(precision=mg.MG_PREC_FP64, fixed_cycles=2))
    rng = np.random.default_rng(L)
    x0 = x.cpu().numpy() + 1e-3 * rng.standard_normal(h.n) * synth.free_mask(L)
    xd = torch.from_numpy(x0).cuda()
    r0 = h.defect(L, b, xd, norm=True)
    st0 = h.solve(b, xd.clone(), mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=10.0))
    assert st0.cycles == 0 and st0.rel_res == r0 / st0.bnorm
    st = h.solve(b, xd, mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-8))
    assert st.status == 0 and st.outer_steps >= 1
    xs = xd.cpu().numpy()
    bands = orc.assemble(N, synth.coords(L, a, gs))
    r = orc.norm2(orc.defect(N, bands, bh, xs)) / orc.norm2(bh)
    assert r <= 1.05e-8, r
    scale = np.linalg.norm(abs_band_product(N, bands, xs) + np.abs(bh))
    assert abs(r - st.rel_res) * orc.norm2(bh) <= 80 * U64 * scale
    h.close()


def _garbage(b, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.randn(b.shape, dtype=b.dtype, device="cuda", generator=g) * 1e3


@pytest.mark.parametrize("L", [5, 7, 10])
def test_zero_guess_equals_a_zeroed_iterate(mg, ctx, L):
    """opts.zero_guess: x's contents are not read; the solve equals the one
    from a zeroed x bit for bit (FP64, mixed under device control and with
    the host loop, with and without graphs, preconditioned CG)."""
    h = mg.Hierarchy(ctx, L, jitter=0.2, seed=90 + L)
    b = torch.from_numpy(synth.rhs_uniform(L, 91 + L)).cuda()
    cases = [dict(precision=mg.MG_PREC_FP64),
             dict(precision=mg.MG_PREC_MIXED),
             dict(precision=mg.MG_PREC_MIXED, use_graph=0),
             dict(precision=mg.MG_PREC_MIXED, inner_max_cycles=1000),  # host-driven loop
             dict(precision=mg.MG_PREC_MIXED, fixed_cycles=1),
             dict(precision=mg.MG_PREC_FP64, krylov=1),
             dict(precision=mg.MG_PREC_MIXED, krylov=1)]
    for k, kw in enumerate(cases):
        o_ref = mg.default_opts(rel_tol=1e-9, **kw)
        x_ref = torch.zeros_like(b)
        s_ref = h.solve(b, x_ref, o_ref)
        o = mg.default_opts(rel_tol=1e-9, zero_guess=1, **kw)
        x = _garbage(b, 100 * L + k)
        s = h.solve(b, x, o)
        torch.cuda.synchronize()
        assert s_ref.status == 0 and s.status == 0, kw
        np.testing.assert_array_equal(x.cpu().numpy(), x_ref.cpu().numpy())
        assert (s.cycles, s.outer_steps, s.rel_res, s.bnorm) == \
            (s_ref.cycles, s_ref.outer_steps, s_ref.rel_res, s_ref.bnorm), kw
        assert s.hist() == s_ref.hist(), kw
    # a tolerance met before any update: the result is x = 0
    for prec in (mg.MG_PREC_FP64, mg.MG_PREC_MIXED):
        x = _garbage(b, 7)
        s = h.solve(b, x, mg.default_opts(precision=prec, rel_tol=10.0, zero_guess=1))
        torch.cuda.synchronize()
        assert s.status == 0 and s.cycles == 0 and s.outer_steps == 0
        assert not x.cpu().numpy().any()
    with pytest.raises(mg.MgError):
        h.solve(b, x, mg.default_opts(zero_guess=2))
    h.close()


def test_zero_guess_in_a_batch(mg, ctx):
    """The batched solver with zero_guess equals the batch from zeroed
    iterates bit for bit, and never reads the callers' x."""
    levels = [5, 7, 6, 8]
    hs = [mg.Hierarchy(ctx, L, jitter=0.2, seed=60 + i) for i, L in enumerate(levels)]
    bs = [torch.from_numpy(synth.rhs_uniform(L, 70 + i)).cuda() for i, L in enumerate(levels)]
    o_ref = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-9)
    xr = [torch.zeros_like(b) for b in bs]
    sr = mg.solve_batch(hs, bs, xr, o_ref)
    o = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-9, zero_guess=1)
    xs = [_garbage(b, 50 + i) for i, b in enumerate(bs)]
    ss = mg.solve_batch(hs, bs, xs, o)
    torch.cuda.synchronize()
    for a, c, s1, s2 in zip(xs, xr, ss, sr):
        assert s1.status == 0 and s2.status == 0
        np.testing.assert_array_equal(a.cpu().numpy(), c.cpu().numpy())
        assert (s1.cycles, s1.outer_steps, s1.rel_res) == (s2.cycles, s2.outer_steps, s2.rel_res)
    for h in hs:
        h.close()


@pytest.mark.parametrize("k", [-60, 45])
def test_solution_scales_exactly_with_b(mg, ctx, k):
    """Powers of two scale exactly in binary arithmetic, and the mixed
    scheme brings defects into FP32 range by a power of two from ||b||: the
    solve for 2^k b is exactly 2^k times the solve for b (same residuals
    and cycle counts) in every solver path."""
    L = 9
    h = mg.Hierarchy(ctx, L, jitter=0.2, seed=120)
    b = torch.from_numpy(synth.rhs_uniform(L, 121)).cuda()
    # 2^k b formed on the host (np.ldexp is exact)
    bk = torch.from_numpy(np.ldexp(b.cpu().numpy(), k)).cuda()
    for kw in (dict(precision=mg.MG_PREC_FP64), dict(precision=mg.MG_PREC_MIXED),
               dict(precision=mg.MG_PREC_MIXED, inner_max_cycles=1000),
               dict(precision=mg.MG_PREC_MIXED, krylov=1)):
        o = mg.default_opts(rel_tol=1e-9, zero_guess=1, **kw)
        x1 = torch.empty_like(b)
        s1 = h.solve(b, x1, o)
        x2 = torch.empty_like(b)
        s2 = h.solve(bk, x2, o)
        torch.cuda.synchronize()
        assert s1.status == 0 and s2.status == 0, kw
        np.testing.assert_array_equal(x2.cpu().numpy(), np.ldexp(x1.cpu().numpy(), k),
                                      err_msg=str(kw))
        assert s2.bnorm == np.ldexp(s1.bnorm, k)
        assert (s2.rel_res, s2.cycles, s2.outer_steps) == (s1.rel_res, s1.cycles, s1.outer_steps), kw
    h.close()
