"""The mixed solve's inner loop under device control (Sec. 6.2.2: FP32
cycles until the FP32 residual has dropped by the requested factor).

With the fused V(2,2) cycle the FP32 cycles an outer step took in the
previous solve are queued at once, each returning at once after a control
kernel has found the loop over; the update and the next FP64 defect wait on
the device for the loop's end.  The decisions are the host loop's, so every
bit must equal the host-driven loop (taken here with a cycle cap of 1000,
which disables device control and binds no loop), whether the queued count
is right, too high (cycles skipped) or too low (single cycles queued after),
with graphs or direct launches.
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


def run(mg, h, b, **kw):
    x = torch.zeros_like(b)
    o = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-10, **kw)
    st = h.solve(b, x, o)
    torch.cuda.synchronize()
    return x.cpu().numpy(), st


def same(a, b):
    xa, sa = a
    xb, sb = b
    np.testing.assert_array_equal(xa, xb)
    assert (sa.status, sa.cycles, sa.outer_steps) == (sb.status, sb.cycles, sb.outer_steps)
    assert sa.rel_res == sb.rel_res and sa.bnorm == sb.bnorm
    assert sa.hist() == sb.hist()


@pytest.mark.parametrize("L", [6, 7, 10])
def test_device_control_equals_host_loop(mg, ctx, L):
    h = mg.Hierarchy(ctx, L, jitter=0.2, seed=800 + L)
    b = torch.from_numpy(synth.rhs_uniform(L, 810 + L)).cuda()
    ref = run(mg, h, b, inner_max_cycles=1000)  # host-driven loop
    assert ref[1].status == 0 and ref[1].rel_res <= 1e-10
    # no inner loop came near the cap of 8 the device-controlled runs use
    assert ref[1].cycles <= 6 * ref[1].outer_steps
    first = run(mg, h, b)            # no history yet: 2 cycles queued per loop
    same(first, ref)
    again = run(mg, h, b)            # queued counts exact
    same(again, ref)
    direct = run(mg, h, b, use_graph=0)
    same(direct, ref)
    # history from loops that took more cycles: queued counts too high
    run(mg, h, b, inner_reduction=1e-4)
    same(run(mg, h, b), ref)
    # and from loops of one cycle: too low
    run(mg, h, b, inner_reduction=0.9)
    same(run(mg, h, b), ref)
    h.close()


def test_device_control_warm_start_and_cap(mg, ctx):
    """A warm start (the full first defect) equals the host loop bit for
    bit; a cap of one cycle binds every loop on the device as on the host."""
    L = 8
    h = mg.Hierarchy(ctx, L, jitter=0.15, seed=830)
    b = torch.from_numpy(synth.rhs_uniform(L, 831)).cuda()
    x0 = np.random.default_rng(832).standard_normal(h.n) * 0.01
    x0[~synth.interior_mask(L)] = 0.0

    def warm(**kw):
        x = torch.from_numpy(x0.copy()).cuda()
        o = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-9, **kw)
        st = h.solve(b, x, o)
        torch.cuda.synchronize()
        return x.cpu().numpy(), st

    ref = warm(inner_max_cycles=1000)
    assert ref[1].status == 0 and ref[1].rel_res <= 1e-9
    same(warm(), ref)
    same(warm(), ref)
    x1, s1 = warm(inner_max_cycles=1)
    assert s1.status == 0 and s1.rel_res <= 1e-9
    assert s1.cycles == s1.outer_steps  # one cycle per outer step
    assert s1.outer_steps > ref[1].outer_steps
    h.close()


def test_device_control_step_limits(mg, ctx):
    """fixed_cycles and an exhausted max_cycles end the outer loop at the
    same step, with the same status, iterate and statistics, on the device
    as on the host."""
    L = 7
    h = mg.Hierarchy(ctx, L, jitter=0.2, seed=840)
    b = torch.from_numpy(synth.rhs_uniform(L, 841)).cuda()

    def solve(**kw):
        x = torch.zeros_like(b)
        o = mg.default_opts(precision=mg.MG_PREC_MIXED, **kw)
        st = h.solve(b, x, o, raise_on_error=False)
        torch.cuda.synchronize()
        return x.cpu().numpy(), st

    for kw in (dict(fixed_cycles=2), dict(fixed_cycles=5, rel_tol=1e-3),
               dict(max_cycles=2, rel_tol=1e-14)):
        ref = solve(inner_max_cycles=1000, **kw)
        got = solve(**kw)
        same(got, ref)
        if "max_cycles" in kw:
            assert got[1].status == mg.MG_ERR_NOCONV
        else:
            assert got[1].status == 0 and got[1].outer_steps == kw["fixed_cycles"]
    h.close()


def test_solve_is_ordered_on_the_callers_stream(mg, ctx):
    """The solve waits on the device for work queued before it on the
    caller's stream, and work queued after it on that stream sees the
    solution, without the host blocking in between."""
    L = 9
    h = mg.Hierarchy(ctx, L, jitter=0.2, seed=850)
    b = torch.from_numpy(synth.rhs_uniform(L, 851)).cuda()
    o = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-9)
    x_ref = torch.zeros_like(b)
    h.solve(b, x_ref, o)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        x = torch.full_like(b, 7.0)
        x.zero_()                       # queued on s before the solve
        h.solve(b, x, o, stream=s)
        out = x * 1.0                   # queued on s after it
    s.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), x_ref.cpu().numpy())
    h.close()
