// BLAS level-1 vector operations (Sec. 6.1: axpy and the other
// vector-vector operations, purely bandwidth bound, as the basic
// architecture comparison): y = alpha x + y, x . y and ||x||_2 on device
// vectors of any length.  Every thread moves 16 bytes per stream and step;
// the reductions sum in FP64 in one fixed order (per tile, then the tiles
// through the library's deterministic two-stage reduction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "device_ops.h"
#include "mg_internal.h"

namespace mg {

namespace {

using dev::BLOCK;
using dev::V16;

// 16-byte vectors per thread and tile.
constexpr int BLAS_UNROLL = 2;

template <typename T>
constexpr int64_t blas_tile() {
    return (int64_t)BLOCK * V16<T>::W * BLAS_UNROLL;
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_axpy(int64_t n, T alpha, const T* __restrict__ x,
                                                T* __restrict__ y) {
    constexpr int W = V16<T>::W;
    typedef typename V16<T>::type VT;
    const int64_t base = (int64_t)blockIdx.x * blas_tile<T>();
    VT xv[BLAS_UNROLL], yv[BLAS_UNROLL];
    bool full[BLAS_UNROLL];
#pragma unroll
    for (int u = 0; u < BLAS_UNROLL; ++u) {
        const int64_t p = base + ((int64_t)u * BLOCK + threadIdx.x) * W;
        full[u] = p + W <= n;
        if (full[u]) {
            xv[u] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(x + p));
            yv[u] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(y + p));
        }
    }
#pragma unroll
    for (int u = 0; u < BLAS_UNROLL; ++u) {
        const int64_t p = base + ((int64_t)u * BLOCK + threadIdx.x) * W;
        if (full[u]) {
            VT r;
#pragma unroll
            for (int e = 0; e < W; ++e) r[e] = fma(alpha, xv[u][e], yv[u][e]);
            __builtin_nontemporal_store(r, reinterpret_cast<VT*>(y + p));
        } else {
            for (int e = 0; e < W; ++e)
                if (p + e < n) y[p + e] = fma(alpha, x[p + e], y[p + e]);
        }
    }
}

// Partial sums of x_i y_i (SQUARE: x_i^2) in FP64 per tile: each thread sums
// its elements in index order, then the block in its fixed order.
template <typename T, bool SQUARE>
__global__ __launch_bounds__(BLOCK) void k_dot_tiles(int64_t n, const T* __restrict__ x,
                                                     const T* __restrict__ y,
                                                     double* __restrict__ partials) {
    constexpr int W = V16<T>::W;
    typedef typename V16<T>::type VT;
    const int64_t base = (int64_t)blockIdx.x * blas_tile<T>();
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < BLAS_UNROLL; ++u) {
        const int64_t p = base + ((int64_t)u * BLOCK + threadIdx.x) * W;
        if (p + W <= n) {
            const VT xv = __builtin_nontemporal_load(reinterpret_cast<const VT*>(x + p));
            VT yv = xv;
            if (!SQUARE) yv = __builtin_nontemporal_load(reinterpret_cast<const VT*>(y + p));
#pragma unroll
            for (int e = 0; e < W; ++e) s += (double)xv[e] * (double)yv[e];
        } else {
            for (int e = 0; e < W; ++e)
                if (p + e < n) s += (double)x[p + e] * (double)(SQUARE ? x[p + e] : y[p + e]);
        }
    }
    const double t = dev::block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

inline unsigned tiles_of(int64_t n, int64_t tile) { return (unsigned)((n + tile - 1) / tile); }

mg_status check_vectors(const mg_context* ctx, mg_dtype dtype, int64_t n, const void* x,
                        const void* y) {
    if (!ctx) return fail(MG_ERR_INVALID, "null context");
    if (dtype != MG_F64 && dtype != MG_F32) return fail(MG_ERR_INVALID, "unknown dtype");
    if (n < 0 || n > MG_BLAS_MAX_N)
        return fail(MG_ERR_INVALID, "n=" + std::to_string(n) + " outside [0, 2^33]");
    if (n > 0 && (!x || !y || ((uintptr_t)x & 15) || ((uintptr_t)y & 15)))
        return fail(MG_ERR_INVALID, "vectors must be non-null and 16-byte aligned");
    return MG_OK;
}

// The context's reduction scratch: the reduction ticket, partials of n
// elements (one per tile), room for the segment sums, two result doubles, and
// a pinned mirror.  Zeroed when allocated (the ticket starts at zero).
mg_status blas_scratch(mg_context* ctx, int64_t tiles) {
    const size_t need =
        (size_t)(PARTIALS_FRONT + (tiles + 63) / 64 * 64 + dev::RED_MAX_SEGS + 64) * sizeof(double);
    if (ctx->blas_bytes >= need && ctx->blas_host) return MG_OK;
    if (!ctx->blas_host) {
        if (hipHostMalloc((void**)&ctx->blas_host, 64 * sizeof(double), hipHostMallocDefault) !=
            hipSuccess) {
            ctx->blas_host = nullptr;
            return fail(MG_ERR_NOMEM, "pinned host allocation failed");
        }
    }
    if (ctx->blas_bytes >= need) return MG_OK;
    if (!ctx->reserve(need)) return fail(MG_ERR_NOMEM, "reduction scratch over the context budget");
    void* p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) {
        (void)hipGetLastError();
        ctx->release(need);
        return fail(MG_ERR_NOMEM, "hipMalloc failed for the reduction scratch");
    }
    if (hipMemset(p, 0, need) != hipSuccess) {
        (void)hipFree(p);
        ctx->release(need);
        return fail(MG_ERR_DEVICE, "hipMemset failed for the reduction scratch");
    }
    if (ctx->blas_scratch) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->blas_scratch);
        ctx->release(ctx->blas_bytes);
    }
    ctx->blas_scratch = (double*)p;
    ctx->blas_bytes = need;
    return MG_OK;
}

template <typename T, bool SQUARE>
mg_status blas_reduce(mg_context* ctx, int64_t n, const T* x, const T* y, double* host_out,
                      hipStream_t st, bool root) {
    const int64_t tiles = std::max<int64_t>(1, (n + blas_tile<T>() - 1) / blas_tile<T>());
    if (mg_status s = blas_scratch(ctx, tiles)) return s;
    double* partials = ctx->blas_scratch + PARTIALS_FRONT;
    // two result slots after the partials and the segment sums
    double* scal = partials + (tiles + 63) / 64 * 64 + dev::RED_MAX_SEGS;
    if (n == 0) {
        *host_out = 0.0;
        return MG_OK;
    }
    hipLaunchKernelGGL((k_dot_tiles<T, SQUARE>), dim3(tiles_of(n, blas_tile<T>())), dim3(BLOCK),
                       0, st, n, x, y, partials);
    MG_HIP(hipGetLastError());
    MG_HIP(launch_reduce(partials, tiles, scal, 0, ctx->blas_host, st));
    MG_HIP(hipStreamSynchronize(st));
    *host_out = ((volatile double*)ctx->blas_host)[root ? 1 : 0];
    return MG_OK;
}

// ---- the dot product without allocation (mg_dot_noalloc)
// Tile partials of one call live in a file-scope device array instead of the
// context's grown-on-demand scratch: 2^17 partials (1 MiB) cover 2^27 FP64 or
// 2^28 FP32 elements.  Each device that runs the call holds its own copy of
// the array until the process ends.  In host code the name `scratch` is only
// a host-side stand-in: kernels get the device address looked up once per
// device (noalloc_scratch).
constexpr int64_t NOALLOC_MAX_TILES = int64_t(1) << 17;
static __device__ __align__(256) double scratch[NOALLOC_MAX_TILES];

constexpr int MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on `device` (current on entry), looked up on
// the first call on that device and kept.
mg_status noalloc_scratch(int device, double** out) {
    if (device < 0 || device >= MAX_DEVICES)
        return fail(MG_ERR_INVALID, "device " + std::to_string(device) + " outside [0, 64)");
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MG_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                           hipGetErrorString(e));
        g_noalloc_ptr[device] = (double*)p;
    }
    *out = g_noalloc_ptr[device];
    return MG_OK;
}

// out[0] = the fixed-order sum of np partials (dev::reduce_partials, the
// order of launch_reduce), in one workgroup.
__global__ __launch_bounds__(BLOCK) void k_reduce_one(const double* __restrict__ partials,
                                                      int64_t np, double* __restrict__ out) {
    const double s = dev::reduce_partials(partials, np);
    if (threadIdx.x == 0) out[0] = s;
}

template <typename T>
mg_status dot_noalloc(int device, int64_t n, const T* x, const T* y, double* dev_out,
                      hipStream_t st) {
    const int64_t tiles = (n + blas_tile<T>() - 1) / blas_tile<T>();
    if (tiles > NOALLOC_MAX_TILES)
        return fail(MG_ERR_INVALID,
                    "n=" + std::to_string(n) + " above the no-allocation limit of " +
                        std::to_string(NOALLOC_MAX_TILES * blas_tile<T>()) + " elements");
    double* partials = nullptr;
    if (mg_status s = noalloc_scratch(device, &partials)) return s;
    // every partial the reduction reads is written by this call first, so
    // nothing is cleared (n = 0 reduces no partials: out = 0)
    if (tiles > 0) {
        hipLaunchKernelGGL((k_dot_tiles<T, false>), dim3((unsigned)tiles), dim3(BLOCK), 0, st, n,
                           x, y, partials);
        MG_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_reduce_one, dim3(1), dim3(BLOCK), 0, st, partials, tiles, dev_out);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

}  // namespace

}  // namespace mg

using namespace mg;

extern "C" mg_status mg_axpy(mg_context* ctx, mg_dtype dtype, int64_t n, double alpha,
                             const void* x, void* y, void* stream) {
    if (mg_status s = check_vectors(ctx, dtype, n, x, y)) return s;
    if (n > 0 && x == y) return fail(MG_ERR_INVALID, "x and y must not alias");
    MG_HIP(hipSetDevice(ctx->device));
    if (n == 0) return MG_OK;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == MG_F64)
        hipLaunchKernelGGL(k_axpy<double>, dim3(tiles_of(n, blas_tile<double>())), dim3(BLOCK), 0,
                           st, n, alpha, (const double*)x, (double*)y);
    else
        hipLaunchKernelGGL(k_axpy<float>, dim3(tiles_of(n, blas_tile<float>())), dim3(BLOCK), 0,
                           st, n, (float)alpha, (const float*)x, (float*)y);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

extern "C" mg_status mg_dot(mg_context* ctx, mg_dtype dtype, int64_t n, const void* x,
                            const void* y, double* host_out, void* stream) {
    if (mg_status s = check_vectors(ctx, dtype, n, x, y)) return s;
    if (!host_out) return fail(MG_ERR_INVALID, "null output");
    MG_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->blas_mu);
    if (dtype == MG_F64)
        return blas_reduce<double, false>(ctx, n, (const double*)x, (const double*)y, host_out,
                                          (hipStream_t)stream, false);
    return blas_reduce<float, false>(ctx, n, (const float*)x, (const float*)y, host_out,
                                     (hipStream_t)stream, false);
}

extern "C" mg_status mg_norm2(mg_context* ctx, mg_dtype dtype, int64_t n, const void* x,
                              double* host_out, void* stream) {
    if (mg_status s = check_vectors(ctx, dtype, n, x, x)) return s;
    if (!host_out) return fail(MG_ERR_INVALID, "null output");
    MG_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->blas_mu);
    if (dtype == MG_F64)
        return blas_reduce<double, true>(ctx, n, (const double*)x, nullptr, host_out,
                                         (hipStream_t)stream, true);
    return blas_reduce<float, true>(ctx, n, (const float*)x, nullptr, host_out,
                                    (hipStream_t)stream, true);
}

extern "C" mg_status mg_dot_noalloc(mg_context* ctx, mg_dtype dtype, int64_t n, const void* x,
                                    const void* y, double* dev_out, void* stream) {
    if (mg_status s = check_vectors(ctx, dtype, n, x, y)) return s;
    if (!dev_out || ((uintptr_t)dev_out & 7))
        return fail(MG_ERR_INVALID, "dev_out must be an 8-byte aligned device pointer");
    MG_HIP(hipSetDevice(ctx->device));
    if (dtype == MG_F64)
        return dot_noalloc<double>(ctx->device, n, (const double*)x, (const double*)y, dev_out,
                                   (hipStream_t)stream);
    return dot_noalloc<float>(ctx->device, n, (const float*)x, (const float*)y, dev_out,
                              (hipStream_t)stream);
}
