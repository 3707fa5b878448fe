"""BLAS level-1 operations on the GPU (Sec. 6.1: axpy and the other
vector-vector operations) against the oracle.

Lengths cover the empty vector, less than one 16-byte vector, ragged tails
of every kind, one and many tiles, and more tiles than one reduction
segment holds (the two-stage reduction).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U64 = 2.0 ** -53
U32 = 2.0 ** -24
SIZES = [0, 1, 3, 17, 1000, 2047, 2048, 2049, (1 << 20) + 5, (1 << 24) + 3]


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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_axpy(mg, ctx, orc, n, dtype):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n).astype(dtype)
    y = rng.standard_normal(n).astype(dtype)
    alpha = -0.37
    yd = dev(y)
    ctx.axpy(alpha, dev(x), yd)
    got = host(yd).astype(np.float64)
    ref = orc.axpy(alpha, x, y).astype(np.float64)
    if dtype == np.float64:
        # one fused rounding against the oracle's two: within 2 u of the terms
        bound = 2 * U64 * (np.abs(alpha * x) + np.abs(y))
    else:
        # both are the FP32 rounding of nearly the same FP64 value: 1 ulp
        bound = 2 * U32 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_dot_and_norm(mg, ctx, orc, n, dtype):
    rng = np.random.default_rng(n + 1)
    x = rng.standard_normal(n).astype(dtype)
    y = rng.standard_normal(n).astype(dtype)
    xd, yd = dev(x), dev(y)
    d = ctx.dot(xd, yd)
    ref = orc.dot(x, y)
    scale = orc.dot(np.abs(x), np.abs(y))
    # both sum FP64 products (exact for FP32 inputs) in different orders
    assert abs(d - ref) <= 2 * (n + 1) * U64 * scale + 1e-300
    nr = ctx.norm2(xd)
    nref = orc.norm2(x.astype(np.float64))
    assert abs(nr - nref) <= 2 * (n + 1) * U64 * nref + 1e-300
    # a result depends only on the data
    assert ctx.dot(xd, yd) == d and ctx.norm2(xd) == nr
    if n == 0:
        assert d == 0.0 and nr == 0.0


def test_blas1_arguments_checked(mg, ctx):
    x = torch.zeros(64, dtype=torch.float32, device="cuda")
    y = torch.zeros(64, dtype=torch.float32, device="cuda")
    with pytest.raises(mg.MgError):
        ctx.axpy(1.0, x, x)  # aliasing
    with pytest.raises(mg.MgError):
        ctx.axpy(1.0, x[1:], y[1:])  # not 16-byte aligned
    with pytest.raises(mg.MgError):
        ctx.dot(x[1:], y[1:])
    out = mg._binding._d()
    st = mg.lib().mg_dot(ctx.handle, mg.MG_F32, -1, mg._binding._ptr(x), mg._binding._ptr(y),
                         mg._binding.ctypes.byref(out), None)
    assert st == mg.MG_ERR_INVALID


def test_blas1_scratch_is_charged_to_the_budget(mg):
    small = mg.Context(0, budget_bytes=4096)
    x = torch.ones(1 << 20, dtype=torch.float64, device="cuda")
    with pytest.raises(mg.MgError) as e:
        small.norm2(x)
    assert e.value.status == mg.MG_ERR_NOMEM
    roomy = mg.Context(0, budget_bytes=1 << 20)
    assert roomy.norm2(x) == 1024.0
    used, _ = roomy.memory()
    assert 0 < used <= 1 << 20
