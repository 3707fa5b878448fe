"""Shared helpers of the GPU parity tests (tolerances derived from the
arithmetic of each operation)."""
import numpy as np

U64 = 2.0 ** -53   # unit roundoff, FP64
U32 = 2.0 ** -24   # unit roundoff, FP32


def offsets(N):
    return [(k // 3 - 1) * N + (k % 3 - 1) for k in range(9)]


def abs_band_product(N, bands, x):
    """sum_k |band_k[p]| |x[p + off_k]|: the scale of the rounding error of a
    9-term band product (a forward error bound is gamma_9 times this)."""
    n = N * N
    ax = np.abs(x)
    out = np.zeros(n)
    ii = np.tile(np.arange(N), N)
    jj = np.repeat(np.arange(N), N)
    for k in range(9):
        di, dj = k % 3 - 1, k // 3 - 1
        ok = (ii + di >= 0) & (ii + di < N) & (jj + dj >= 0) & (jj + dj < N)
        p = np.nonzero(ok)[0]
        out[p] += np.abs(bands[k][p]) * ax[p + dj * N + di]
    return out


def assert_within(got, ref, bound, what):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(got - ref)
    bad = err > bound
    if np.any(bad):
        k = int(np.argmax(err - bound))
        raise AssertionError("%s: %d of %d entries outside the bound; worst at %d: got %r ref %r "
                             "bound %r" % (what, int(bad.sum()), err.size, k, got[k], ref[k],
                                           bound[k] if np.ndim(bound) else bound))
