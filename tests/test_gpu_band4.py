"""The four-band combination of the shallow-water prediction step (Sec.
2.2: u_new = u + M1 v + M2 w + M3 u + M4 u + S(u), each M_i with four
bands) on the GPU against the oracle.

FP64: both sides add the same terms in the same order, the device with one
fused rounding per term, so they agree within a few ulps of the sum of the
terms' magnitudes.  FP32: the device result against the oracle's FP64
evaluation of the same FP32 inputs, within 20 FP32 roundings of that scale.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U64 = 2.0 ** -53
U32 = 2.0 ** -24


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
    return t.cpu().numpy().astype(np.float64)


def swe_offsets(N):
    return [(-2, -1, 1, 2), (-2 * N, -N, N, 2 * N), (-1, 1, -N, N), (-N - 1, -N + 1, N - 1, N + 1)]


@pytest.mark.parametrize("N", [1, 3, 17, 100, 1025])
@pytest.mark.parametrize("m", [1, 2, 4])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("with_source", [False, True])
def test_band4_matches_oracle(mg, ctx, orc, N, m, dtype, with_source):
    n = N * N
    rng = np.random.default_rng(N * 10 + m)
    offs = [tuple(max(-n + 1, min(n - 1, o)) for o in row) for row in swe_offsets(N)[:m]]
    bands = [rng.standard_normal((4, n)).astype(dtype) for _ in range(m)]
    u = rng.standard_normal(n).astype(dtype)
    vs = [rng.standard_normal(n).astype(dtype) for _ in range(m - 1)] + [u]  # M_m acts on u
    s = rng.standard_normal(n).astype(dtype) if with_source else None
    out = torch.empty(n, dtype=torch.float64 if dtype == np.float64 else torch.float32,
                      device="cuda")
    dvs = [dev(v) for v in vs[:-1]]
    du = dev(u)
    ctx.band4_combine([dev(b) for b in bands], offs, dvs + [du], du, out,
                      s=None if s is None else dev(s))
    ref = orc.band4_combine(bands, offs, vs, u, s)
    scale = orc.band4_combine([np.abs(b) for b in bands], offs, [np.abs(v) for v in vs],
                              np.abs(u), None if s is None else np.abs(s))
    u_ = U64 if dtype == np.float64 else U32
    bound = (4 * m + 4) * u_ * scale + 1e-300
    got = host(out)
    assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) - bound))


def test_band4_band_stride_and_far_offsets(mg, ctx, orc):
    n, stride = 1000, 1088
    rng = np.random.default_rng(7)
    full = rng.standard_normal((4, stride))
    offs = [(-999, -500, 500, 999)]
    u = rng.standard_normal(n)
    v = rng.standard_normal(n)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.band4_combine([dev(full)], offs, [dev(v)], dev(u), out)
    ref = orc.band4_combine([full[:, :n]], offs, [v], u)
    assert np.max(np.abs(host(out) - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_band4_arguments_checked(mg, ctx):
    n = 16
    b = torch.zeros((4, n), dtype=torch.float64, device="cuda")
    u = torch.zeros(n, dtype=torch.float64, device="cuda")
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(mg.MgError):
        ctx.band4_combine([b], [(0, 1, 2, n)], [u], u, out)  # offset out of (-n, n)
    with pytest.raises(mg.MgError):
        ctx.band4_combine([b] * 5, [(0, 1, 2, 3)] * 5, [u] * 5, u, out)  # m > 4
    with pytest.raises(mg.MgError):
        ctx.band4_combine([b], [(0, 1, 2, 3)], [u], u, u)  # output aliases u
