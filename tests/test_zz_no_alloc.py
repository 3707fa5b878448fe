"""mg_dot_noalloc (the dot product for callers that cannot allocate) against
mg_dot: the same kernels and summation order, so the same bits, on two calls
in a row (the second with a smaller input, so the first call's partials are
still in the library's fixed device array), in FP64 and FP32, for ragged
lengths, n = 0, and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FP64_MAX = 1 << 27  # the fixed array holds 2^17 tile partials of 1024 FP64 elements
FP32_MAX = 1 << 28  # or of 2048 FP32 elements


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_0904_4152_amd as mg
    return mg, torch, mg.Context(0)


def _vec(torch, n, dtype, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    return torch.randn(n, generator=g, device="cuda", dtype=torch.float64).to(dtype)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_noalloc_dot_equals_dot_on_two_calls(env, dt):
    mg, torch, ctx = env
    dtype = torch.float64 if dt == "f64" else torch.float32
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    # a large ragged length (several reduction segments), then a smaller one
    for n, seed in ((20_000_003, 1), (4_099, 2)):
        print("noalloc dot: dtype=%s n=%d" % (dt, n), flush=True)
        x = _vec(torch, n, dtype, seed)
        y = _vec(torch, n, dtype, seed + 10)
        ref = ctx.dot(x, y)
        ctx.dot_noalloc(x, y, out)
        torch.cuda.synchronize()
        got = float(out[0].item())
        assert got == ref, (n, got, ref)
        assert np.isnan(float(out[1].item()))  # only out[0] is written
        # against an FP64 sum on the host (independent of the kernels)
        xd = x.double().cpu().numpy()
        yd = y.double().cpu().numpy()
        exact = float(np.dot(xd, yd))
        bound = 2 * n * 2.0 ** -53 * float(np.abs(xd) @ np.abs(yd))
        assert abs(got - exact) <= bound


def test_noalloc_dot_at_the_limit_and_beyond(env):
    mg, torch, ctx = env
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    x = torch.ones(FP32_MAX, dtype=torch.float32, device="cuda")
    print("noalloc dot: dtype=f32 n=%d (the limit)" % FP32_MAX, flush=True)
    ctx.dot_noalloc(x, x, out)
    torch.cuda.synchronize()
    assert float(out.item()) == float(FP32_MAX) == ctx.dot(x, x)
    x1 = torch.ones(FP32_MAX + 1, dtype=torch.float32, device="cuda")
    with pytest.raises(mg.MgError) as e:
        ctx.dot_noalloc(x1, x1, out)
    assert e.value.status == mg.MG_ERR_INVALID
    del x, x1
    xd = torch.ones(FP64_MAX + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(mg.MgError) as e:
        ctx.dot_noalloc(xd, xd, out)
    assert e.value.status == mg.MG_ERR_INVALID
    del xd
    torch.cuda.empty_cache()


def test_noalloc_dot_of_empty_vectors(env):
    mg, torch, ctx = env
    out = torch.full((1,), 5.0, dtype=torch.float64, device="cuda")
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    ctx.dot_noalloc(e, e, out)
    torch.cuda.synchronize()
    assert float(out.item()) == 0.0 == ctx.dot(e, e)
