// Linear combination of four-band products (Sec. 2.2: the shallow-water
// prediction step adds to u the products of up to four banded matrices of
// four bands each with the step's vectors, plus a source term).  One fused
// pass: every band value, every vector element and the result cross HBM
// once; neighbour reads of the shifted bands hit the same cache lines as
// the adjacent threads' own reads.
#include <hip/hip_runtime.h>

#include <string>

#include "device_ops.h"
#include "mg_internal.h"

namespace mg {

namespace {

using dev::BLOCK;

constexpr int B4_MAX_TERMS = 4;
constexpr int B4_PER_THREAD = 2;  // elements per thread, BLOCK apart

template <typename T>
struct Band4Args {
    const T* bands[B4_MAX_TERMS];  // band k of term i at bands[i] + k * bs
    const T* v[B4_MAX_TERMS];
    int off[B4_MAX_TERMS][4];
    const T* u;
    const T* s;  // nullable
    T* out;
    int64_t n;
    int64_t bs;
    int m;
};

// out[p] = u[p] + sum_i sum_k band_i,k[p] v_i[p + off_i,k] (+ s[p]); the
// terms are added in (i, k) order after u, the source last.
template <typename T, int M>
__global__ __launch_bounds__(BLOCK) void k_band4(Band4Args<T> a) {
    const int64_t base = (int64_t)blockIdx.x * BLOCK * B4_PER_THREAD + threadIdx.x;
#pragma unroll
    for (int e = 0; e < B4_PER_THREAD; ++e) {
        const int64_t p = base + (int64_t)e * BLOCK;
        if (p >= a.n) return;
        T acc = a.u[p];
#pragma unroll
        for (int i = 0; i < M; ++i) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t q = p + a.off[i][k];
                const T vq = (q >= 0 && q < a.n) ? a.v[i][q] : T(0);
                acc = fma(__builtin_nontemporal_load(a.bands[i] + k * a.bs + p), vq, acc);
            }
        }
        if (a.s) acc += a.s[p];
        a.out[p] = acc;
    }
}

template <typename T>
hipError_t launch_band4(const Band4Args<T>& a, hipStream_t st) {
    const unsigned g = (unsigned)((a.n + BLOCK * B4_PER_THREAD - 1) / (BLOCK * B4_PER_THREAD));
    switch (a.m) {
        case 1: hipLaunchKernelGGL((k_band4<T, 1>), dim3(g), dim3(BLOCK), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_band4<T, 2>), dim3(g), dim3(BLOCK), 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_band4<T, 3>), dim3(g), dim3(BLOCK), 0, st, a); break;
        default: hipLaunchKernelGGL((k_band4<T, 4>), dim3(g), dim3(BLOCK), 0, st, a); break;
    }
    return hipGetLastError();
}

template <typename T>
mg_status band4(int64_t n, int m, const void* const* bands, int64_t bs, const int* offsets,
                const void* const* v, const void* u, const void* s, void* out, hipStream_t st) {
    Band4Args<T> a{};
    for (int i = 0; i < m; ++i) {
        a.bands[i] = (const T*)bands[i];
        a.v[i] = (const T*)v[i];
        for (int k = 0; k < 4; ++k) a.off[i][k] = offsets[4 * i + k];
    }
    a.u = (const T*)u;
    a.s = (const T*)s;
    a.out = (T*)out;
    a.n = n;
    a.bs = bs;
    a.m = m;
    MG_HIP(launch_band4<T>(a, st));
    return MG_OK;
}

}  // namespace

}  // namespace mg

using namespace mg;

extern "C" mg_status mg_band4_combine(mg_context* ctx, mg_dtype dtype, int64_t n, int m,
                                      const void* const* bands, int64_t band_stride,
                                      const int* offsets, const void* const* v, const void* u,
                                      const void* s, void* u_new, void* stream) {
    if (!ctx) return fail(MG_ERR_INVALID, "null context");
    if (dtype != MG_F64 && dtype != MG_F32) return fail(MG_ERR_INVALID, "unknown dtype");
    if (n < 0 || n > ((int64_t)1 << 32))
        return fail(MG_ERR_INVALID, "n=" + std::to_string(n) + " outside [0, 2^32]");
    if (m < 1 || m > B4_MAX_TERMS) return fail(MG_ERR_INVALID, "m must lie in [1, 4]");
    if (band_stride < n) return fail(MG_ERR_INVALID, "band_stride must be >= n");
    if (n == 0) return MG_OK;
    if (!bands || !offsets || !v || !u || !u_new)
        return fail(MG_ERR_INVALID, "null argument");
    for (int i = 0; i < m; ++i) {
        if (!bands[i] || !v[i]) return fail(MG_ERR_INVALID, "null band or vector pointer");
        for (int k = 0; k < 4; ++k) {
            const int o = offsets[4 * i + k];
            if ((int64_t)o <= -n || (int64_t)o >= n)
                return fail(MG_ERR_INVALID, "band offset " + std::to_string(o) +
                                                " outside (-n, n)");
        }
        if (v[i] == u_new) return fail(MG_ERR_INVALID, "u_new must not alias an input vector");
    }
    if (u_new == u || (s && u_new == s))
        return fail(MG_ERR_INVALID, "u_new must not alias an input vector");
    MG_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == MG_F64) return band4<double>(n, m, bands, band_stride, offsets, v, u, s, u_new, st);
    return band4<float>(n, m, bands, band_stride, offsets, v, u, s, u_new, st);
}
