// Device arithmetic of the hot path, per tile or per element.  The
// single-problem kernels (kernels.hip) and the batched persistent kernels
// (batch.hip) call exactly these functions with the same tiling, so a
// problem's results do not depend on which other problems share a launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mg {
namespace dev {

constexpr int BLOCK = 256;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T>
struct V16;
template <>
struct V16<float> {
    typedef f32x4 type;
    static constexpr int W = 4;
};
template <>
struct V16<double> {
    typedef f64x2 type;
    static constexpr int W = 2;
};

// Rows per stencil tile: 16 bytes of every band per thread.
template <typename T>
constexpr int tile_rows() {
    return BLOCK * V16<T>::W;
}

// Elements per reduction tile of a plain vector norm.
constexpr int NORM_TILE = BLOCK * 4;

// The damped Jacobi correction num / a_pp (num = omega (b - A x)): FP64
// divides; FP32 multiplies by the hardware reciprocal of a_pp (within one
// ulp of it; the FP32 sweeps are the inner solver of the mixed scheme, whose
// result the FP64 defect correction checks and corrects).  Every FP32
// Jacobi sweep (tile kernels, fused passes, coarse tail, batch) uses it, so
// they all give the same bits.
template <typename T>
__device__ __forceinline__ T jacobi_div(T num, T diag) {
    return num / diag;
}
template <>
__device__ __forceinline__ float jacobi_div<float>(float num, float diag) {
    return num * __builtin_amdgcn_rcpf(diag);
}

// Deterministic block sum (wave shuffles, then the waves in order); the
// result is valid in thread 0.  Every thread of the block must call it; it
// may be called repeatedly in a loop.
template <int NT = BLOCK>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double ws[NT / 64];
    __syncthreads();
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += ws[w];
    }
    return s;
}

enum { OP_SPMV = 0, OP_DEFECT = 1, OP_JACOBI = 2 };

// s + r * r in two roundings (product, then sum).  The norm partials of the
// stencil tile kinds must agree bit for bit, and whether the compiler fuses
// a product and a sum into one fma depends on the code around them, so it
// is not left to it here.
__device__ __forceinline__ double add_sq(double s, double r) {
#pragma clang fp contract(off)
    return s + r * r;
}

// The mixed scheme rounds each FP64 defect to FP32 after scaling it by a
// power of two fixed per solve by ||b||: 2^-e for ||b|| = m 2^e with m in
// [0.5, 1) (e clamped so that 2^e and 2^-e stay normal), and scales the FP32
// correction back by 2^e.  Scaling by a power of two is exact in binary
// floating point, so the FP32 inner solve computes the same digits whatever
// e is; the scale only keeps the FP32 values in range.
__host__ __device__ inline int pow2_exponent(double v) {
    int e = 0;
    (void)frexp(v, &e);
    return e < -1020 ? -1020 : (e > 1020 ? 1020 : e);
}
__host__ __device__ inline double pow2_scale(double v) { return ldexp(1.0, -pow2_exponent(v)); }
__host__ __device__ inline double pow2_unscale(double v) { return ldexp(1.0, pow2_exponent(v)); }

// Destination of a defect tile's values rounded to FP32 after scaling by sc
// (the mixed scheme's FP32 right-hand side), written in place of the FP64
// values when a tile function's CAST is set.
struct Cast32 {
    float* out = nullptr;
    double sc = 1.0;
};

// W consecutive floats at p (p aligned to W floats) in one store.
template <int W>
__device__ __forceinline__ void store_floats(float* __restrict__ p, const float* f) {
    typedef float VF __attribute__((ext_vector_type(W)));
    VF v;
    __builtin_memcpy(&v, f, sizeof(VF));
    *reinterpret_cast<VF*>(p) = v;
}

// One stencil tile: rows [blo, blo + tile_rows) of y = A x (SPMV),
// d = b - A x (DEFECT) or x' = x + omega (b - A x) / a_pp (JACOBI).  Each
// thread owns W consecutive rows.  Tiles at least N+1 rows away from both
// ends of the vector read the x halo without bounds checks.  Returns the
// thread's sum of squares of its outputs when NORM.  With CAST (FP64 only)
// STORE writes float(v sc) to cast.out instead of v to out.
//
// SYM: the matrix is symmetric bit for bit, so the lower bands at p are
// read as upper bands of the neighbours (band 8 at p-N-1, 7 at p-N, 6 at
// p-N+1, 5 at p-1; zero before the first row, as stored).  Those rows were
// streamed by the tiles just before (same XCD), so the shifted reads are
// served by the cache and HBM sees 5 band streams instead of 9.  Same
// values, same results.
template <typename T, int OP, bool NORM, bool STORE, bool SYM = false, bool CAST = false>
__device__ __forceinline__ double stencil_tile(const T* __restrict__ bands, int64_t bs, int N,
                                               int64_t n, const T* __restrict__ x,
                                               const T* __restrict__ b, T* __restrict__ out,
                                               T omega, int64_t blo, Cast32 cast = Cast32{}) {
    static_assert(!CAST || (sizeof(T) == 8 && OP == OP_DEFECT), "CAST: FP64 defects");
    constexpr int W = V16<T>::W;
    typedef typename V16<T>::type VT;
    const int64_t p0 = blo + (int64_t)threadIdx.x * W;
    const bool fast = (blo - N - 1 >= 0) && (blo + tile_rows<T>() + N + 1 <= n);
    double sq = 0.0;
    if (p0 >= n) return sq;
    T xv[3][W + 2];
    if (fast) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const T* xp = x + p0 + (int64_t)(r - 1) * N - 1;
#pragma unroll
            for (int e = 0; e < W + 2; ++e) xv[r][e] = xp[e];
        }
    } else {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int e = 0; e < W + 2; ++e) {
                const int64_t q = p0 + (int64_t)(r - 1) * N - 1 + e;
                xv[r][e] = (q >= 0 && q < n) ? x[q] : T(0);
            }
        }
    }
    T bk[9][W];
#pragma unroll
    for (int k = SYM ? 4 : 0; k < 9; ++k) {
        // band arrays are padded beyond n, so the vector load stays in bounds;
        // with SYM the bands read again by later tiles stay cacheable
        const VT* src = reinterpret_cast<const VT*>(bands + k * bs + p0);
        VT v = (!SYM || k == 4) ? __builtin_nontemporal_load(src) : *src;
        __builtin_memcpy(bk[k], &v, sizeof(VT));
    }
    if (SYM) {
        const int64_t sh[4] = {-(int64_t)N - 1, -(int64_t)N, -(int64_t)N + 1, -1};
        const int up[4] = {8, 7, 6, 5};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T* src = bands + up[k] * bs + p0 + sh[k];
#pragma unroll
            for (int v = 0; v < W; ++v)
                bk[k][v] = (fast || p0 + v + sh[k] >= 0) ? src[v] : T(0);
        }
    }
    T res[W];
#pragma unroll
    for (int v = 0; v < W; ++v) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) acc = fma(bk[k][v], xv[k / 3][v + k % 3], acc);
        res[v] = acc;
    }
    if (OP != OP_SPMV) {
        T bb[W];
        if (fast) {
            VT v = *reinterpret_cast<const VT*>(b + p0);
            __builtin_memcpy(bb, &v, sizeof(VT));
        } else {
#pragma unroll
            for (int v = 0; v < W; ++v) bb[v] = (p0 + v < n) ? b[p0 + v] : T(0);
        }
#pragma unroll
        for (int v = 0; v < W; ++v) {
            if (OP == OP_DEFECT)
                res[v] = bb[v] - res[v];
            else
                res[v] = xv[1][v + 1] + jacobi_div(omega * (bb[v] - res[v]), bk[4][v]);
        }
    }
    if (NORM) {
#pragma unroll
        for (int v = 0; v < W; ++v)
            if (p0 + v < n) sq = add_sq(sq, (double)res[v]);
    }
    if (STORE && CAST) {
        float f[W];
#pragma unroll
        for (int v = 0; v < W; ++v) f[v] = (float)((double)res[v] * cast.sc);
        if (fast) {
            store_floats<W>(cast.out + p0, f);
        } else {
#pragma unroll
            for (int v = 0; v < W; ++v)
                if (p0 + v < n) cast.out[p0 + v] = f[v];
        }
    } else if (STORE) {
        if (fast) {
            VT v;
            __builtin_memcpy(&v, res, sizeof(VT));
            *reinterpret_cast<VT*>(out + p0) = v;
        } else {
#pragma unroll
            for (int v = 0; v < W; ++v)
                if (p0 + v < n) out[p0 + v] = res[v];
        }
    }
    return sq;
}

// stencil_tile with SYM on an interior tile (every neighbour inside the
// vector), its scattered loads staged through LDS: each workgroup loads the
// three rows of x and the previous row's bands 6, 7 and 8 that the tile
// touches with aligned 16-byte loads (one or two per thread and row) and
// passes band 5 to the next node through LDS, instead of per-element loads
// of every neighbour.  Every node's operands and fma chain are those of
// stencil_tile, so the results are the same bits.  Tiles at either end of
// the vector take stencil_tile itself.  Every thread of the workgroup must
// call it (barriers inside).
template <typename T, int OP, bool NORM, bool STORE, bool CAST = false>
__device__ __forceinline__ double stencil_tile_staged(const T* __restrict__ bands, int64_t bs,
                                                      int N, int64_t n,
                                                      const T* __restrict__ x,
                                                      const T* __restrict__ b,
                                                      T* __restrict__ out, T omega, int64_t blo,
                                                      Cast32 cast = Cast32{}) {
    constexpr int W = V16<T>::W, R = tile_rows<T>();
    constexpr int SL = R + 2 * W;  // elements of one staged segment
    typedef typename V16<T>::type VT;
    // segment starts, rounded down to a vector: x rows at offsets -N-1, -1,
    // N-1 and the previous row's bands at -N-1 (floor division)
    auto seg0 = [&](int64_t o) -> int64_t {
        const int64_t q = blo + o;
        return (q >= 0 ? q / W : -((-q + W - 1) / W)) * W;
    };
    const int64_t ax[3] = {seg0(-(int64_t)N - 1), seg0(-1), seg0((int64_t)N - 1)};
    const int64_t ab = ax[0];
    const bool inner = ab - W >= 0 && ax[2] + SL <= n;  // uniform per tile
    if (!inner)
        return stencil_tile<T, OP, NORM, STORE, true, CAST>(bands, bs, N, n, x, b, out, omega, blo,
                                                             cast);
    __shared__ T sx[3][SL];
    __shared__ T sb[3][SL];      // bands 8, 7, 6 of the previous row
    __shared__ T s5[R + W];      // band 5 at blo - W .. blo + R - 1
    const int t = threadIdx.x;
    const int64_t p0 = blo + (int64_t)t * W;
    // this thread's own band vectors (diagonal and upper bands) and b
    T bk[9][W];
#pragma unroll
    for (int k = 4; k < 9; ++k) {
        const VT* src = reinterpret_cast<const VT*>(bands + k * bs + p0);
        VT v = k == 4 ? __builtin_nontemporal_load(src) : *src;
        __builtin_memcpy(bk[k], &v, sizeof(VT));
    }
    T bb[W];
    if (OP != OP_SPMV) {
        VT v = *reinterpret_cast<const VT*>(b + p0);
        __builtin_memcpy(bb, &v, sizeof(VT));
    }
    __syncthreads();  // a previous tile of this workgroup is done with LDS
    // staged segments: vector j of each, j = t and (t < SL/W - BLOCK) t + BLOCK
#pragma unroll
    for (int rep = 0; rep < 2; ++rep) {
        const int j = t + rep * BLOCK;
        if (rep == 0 || j < SL / W) {
#pragma unroll
            for (int r = 0; r < 3; ++r)
                *reinterpret_cast<VT*>(&sx[r][j * W]) =
                    *reinterpret_cast<const VT*>(x + ax[r] + (int64_t)j * W);
            const int up[3] = {8, 7, 6};
#pragma unroll
            for (int k = 0; k < 3; ++k)
                *reinterpret_cast<VT*>(&sb[k][j * W]) =
                    *reinterpret_cast<const VT*>(bands + up[k] * bs + ab + (int64_t)j * W);
        }
    }
    *reinterpret_cast<VT*>(&s5[W + t * W]) = *reinterpret_cast<const VT*>(bk[5]);
    if (t == 0) *reinterpret_cast<VT*>(&s5[0]) = *reinterpret_cast<const VT*>(bands + 5 * bs + blo - W);
    __syncthreads();
    T xv[3][W + 2];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int o = (int)(p0 + (int64_t)(r - 1) * N - 1 - ax[r]);
#pragma unroll
        for (int e = 0; e < W + 2; ++e) xv[r][e] = sx[r][o + e];
    }
    {
        // A[p][p-N-1] = band 8 at p-N-1, A[p][p-N] = band 7 at p-N,
        // A[p][p-N+1] = band 6 at p-N+1, A[p][p-1] = band 5 at p-1
        const int o = (int)(p0 - (int64_t)N - 1 - ab);
#pragma unroll
        for (int v = 0; v < W; ++v) {
            bk[0][v] = sb[0][o + v];
            bk[1][v] = sb[1][o + v + 1];
            bk[2][v] = sb[2][o + v + 2];
            bk[3][v] = s5[W + t * W + v - 1];
        }
    }
    T res[W];
#pragma unroll
    for (int v = 0; v < W; ++v) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) acc = fma(bk[k][v], xv[k / 3][v + k % 3], acc);
        res[v] = acc;
    }
    double sq = 0.0;
    if (OP != OP_SPMV) {
#pragma unroll
        for (int v = 0; v < W; ++v) {
            if (OP == OP_DEFECT)
                res[v] = bb[v] - res[v];
            else
                res[v] = xv[1][v + 1] + jacobi_div(omega * (bb[v] - res[v]), bk[4][v]);
        }
    }
    if (NORM) {
#pragma unroll
        for (int v = 0; v < W; ++v) sq = add_sq(sq, (double)res[v]);
    }
    if (STORE && CAST) {
        float f[W];
#pragma unroll
        for (int v = 0; v < W; ++v) f[v] = (float)((double)res[v] * cast.sc);
        store_floats<W>(cast.out + p0, f);
    } else if (STORE) {
        VT v;
        __builtin_memcpy(&v, res, sizeof(VT));
        *reinterpret_cast<VT*>(out + p0) = v;
    }
    return sq;
}

// The defect tile of a zero iterate, d = b on rows [blo, blo + tile_rows):
// the same nodes per thread as stencil_tile and the thread's sum of squares
// in the same order, so the bits equal stencil_tile's OP_DEFECT with x = 0
// (b - 0 is b).  out may be null (norm only).  With CAST the values go to
// cast.out as stencil_tile's CAST writes them (out is not used).
template <typename T, bool CAST = false>
__device__ __forceinline__ double copy_tile_sumsq(const T* __restrict__ b, T* __restrict__ out,
                                                  int64_t n, int64_t blo, Cast32 cast = Cast32{}) {
    constexpr int W = V16<T>::W;
    const int64_t p0 = blo + (int64_t)threadIdx.x * W;
    double sq = 0.0;
#pragma unroll
    for (int v = 0; v < W; ++v) {
        if (p0 + v < n) {
            const T r = b[p0 + v];
            sq = add_sq(sq, (double)r);
            if (CAST)
                cast.out[p0 + v] = (float)((double)r * cast.sc);
            else if (out)
                out[p0 + v] = r;
        }
    }
    return sq;
}

// Damped Jacobi sweep from a zero iterate: x' = omega b / a_pp.
template <typename T>
__device__ __forceinline__ void jacobi_zero_elem(const T* __restrict__ diag,
                                                 const T* __restrict__ b, T* __restrict__ xo,
                                                 int64_t p, T omega) {
    xo[p] = jacobi_div(omega * b[p], diag[p]);
}

// Dirichlet sides (bit 1: x = 0, bit 2: x = 1, bit 4: y = 0, bit 8: y = 1);
// the other sides carry the natural homogeneous Neumann condition.
constexpr int ALL_DIRICHLET = 15;

// Evaluated without short-circuits, so callers get straight-line selects.
__host__ __device__ __forceinline__ bool is_dirichlet(int N, int i, int j, int dmask) {
    const unsigned side = (unsigned)(i == 0) | (unsigned)(i == N - 1) << 1 |
                          (unsigned)(j == 0) << 2 | (unsigned)(j == N - 1) << 3;
    return (side & (unsigned)dmask) != 0;
}

// b_c(I,J) = P^T d_f: weights 1 (centre), 1/2 (edges), 1/4 (corners) over the
// 3x3 fine neighbourhood of (2I, 2J), terms outside the grid absent (zero);
// zero at coarse Dirichlet nodes.
template <typename T>
__device__ __forceinline__ void restrict_elem(int Nf, const T* __restrict__ d,
                                              T* __restrict__ bc, int I, int J, int dmask) {
    const int Nc = (Nf >> 1) + 1;
    T s = T(0);
    if (!is_dirichlet(Nc, I, J, dmask)) {
        const int i = 2 * I, j = 2 * J;
        auto at = [&](int di, int dj) -> T {
            const int ii = i + di, jj = j + dj;
            return (ii >= 0 && ii < Nf && jj >= 0 && jj < Nf) ? d[(int64_t)jj * Nf + ii] : T(0);
        };
        const T corner = (at(-1, -1) + at(1, -1)) + (at(-1, 1) + at(1, 1));
        const T edge = (at(0, -1) + at(0, 1)) + (at(-1, 0) + at(1, 0));
        s = at(0, 0) + T(0.5) * edge + T(0.25) * corner;
    }
    bc[(int64_t)J * Nc + I] = s;
}

// x_f(i,j) += bilinear interpolation (index space) of x_c at fine node (i,j).
template <typename T>
__device__ __forceinline__ void prolong_elem(int Nf, const T* __restrict__ xc,
                                             T* __restrict__ xf, int i, int j) {
    const int Nc = (Nf >> 1) + 1;
    const int I = i >> 1, J = j >> 1;
    const T* c = xc + (int64_t)J * Nc + I;
    T v;
    if (!(i & 1) && !(j & 1))
        v = c[0];
    else if (!(j & 1))
        v = T(0.5) * (c[0] + c[1]);
    else if (!(i & 1))
        v = T(0.5) * (c[0] + c[Nc]);
    else
        v = T(0.25) * ((c[0] + c[1]) + (c[Nc] + c[Nc + 1]));
    xf[(int64_t)j * Nf + i] += v;
}

// Coarsest level: at most 17 x 17 nodes (level 4).
constexpr int COARSE_MAX_LEVEL = 4;
constexpr int COARSE_MAX_N = (1 << COARSE_MAX_LEVEL) + 1;
constexpr int COARSE_MAX_UNKNOWNS = COARSE_MAX_N * COARSE_MAX_N;
// LDS doubles of a coarse solve: CG keeps x, r, q and p (p with N+1 zeros on
// either side for the band product); Cholesky needs m values and m indices.
constexpr int COARSE_LDS = 4 * COARSE_MAX_UNKNOWNS + 2 * (COARSE_MAX_N + 1);
static_assert(COARSE_LDS >= COARSE_MAX_UNKNOWNS + (COARSE_MAX_UNKNOWNS + 1) / 2,
              "Cholesky scratch fits");

// How the coarsest level is solved (always in FP64).
struct CoarseSolver {
    const double* chol;    // m x m Cholesky factor of the unknowns' block
    const double* bands;   // FP64 bands of the coarsest level (stride bs)
    int64_t bs;
    int m;                 // unknowns: the nodes off the Dirichlet sides
    int dmask;             // Dirichlet sides
    int cg;                // 1: conjugate gradients; 0: Cholesky
    int max_iter;          // CG step limit
    double tol;            // CG: stop once ||r|| <= tol ||b||
};

// Dirichlet rows are identity rows; the other nodes are solved with the
// Cholesky factor of their block (thread 0; forward and back substitution).
template <typename T>
__device__ __forceinline__ void coarse_cholesky(const CoarseSolver& cs, int Nc,
                                                const T* __restrict__ b, T* __restrict__ x,
                                                double* __restrict__ w) {
    double* z = w;
    int* node = reinterpret_cast<int*>(w + COARSE_MAX_UNKNOWNS);
    const int m = cs.m;
    for (int p = threadIdx.x; p < Nc * Nc; p += blockDim.x)
        if (is_dirichlet(Nc, p % Nc, p / Nc, cs.dmask)) x[p] = b[p];
    if (threadIdx.x == 0) {
        int r = 0;
        for (int p = 0; p < Nc * Nc; ++p)
            if (!is_dirichlet(Nc, p % Nc, p / Nc, cs.dmask)) node[r++] = p;
        // the factor is banded (unknowns in node order: nothing more than
        // Nc + 1 off the diagonal), so the sums run over the band only; the
        // terms left out are exact zeros
        const int bw = Nc + 1;
        for (int r = 0; r < m; ++r) {
            double s = (double)b[node[r]];
            for (int k = max(0, r - bw); k < r; ++k) s -= cs.chol[r * m + k] * z[k];
            z[r] = s / cs.chol[r * m + r];
        }
        for (int r = m - 1; r >= 0; --r) {
            double s = z[r];
            for (int k = r + 1; k < min(m, r + bw + 1); ++k) s -= cs.chol[k * m + r] * z[k];
            z[r] = s / cs.chol[r * m + r];
        }
        for (int r = 0; r < m; ++r) x[node[r]] = (T)z[r];
    }
}

// u . v over n nodes in one fixed order for any workgroup size: lane l of
// wavefront 0 sums the nodes p = l mod 64 in index order, then the lanes
// combine in a fixed butterfly and lane 0's total is broadcast through
// *slot.  Every thread of the workgroup must call it.
__device__ __forceinline__ double cg_dot(const double* __restrict__ u,
                                         const double* __restrict__ v, int n, double* slot) {
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int p = threadIdx.x; p < n; p += 64) s += u[p] * v[p];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (threadIdx.x == 0) *slot = s;
    }
    __syncthreads();
    return *slot;
}

// Unpreconditioned conjugate gradients (Hestenes and Stiefel) on the
// coarsest level from a zero iterate, in FP64: q = A p, alpha = (r.r)/(p.q),
// x += alpha p, r -= alpha q, beta = (r'.r')/(r.r), p = r' + beta p; stops
// before a step once ||r|| <= tol ||b|| or after max_iter steps.  Dirichlet
// rows keep their zero start (identity rows, zero right-hand side).  The
// results do not depend on the workgroup size.
template <typename T>
__device__ __forceinline__ void coarse_cg(const CoarseSolver& cs, int N, const T* __restrict__ b,
                                          T* __restrict__ x, double* __restrict__ w) {
    __shared__ double red[2];
    const int n = N * N;
    double* xs = w;
    double* r = xs + n;
    double* q = r + n;
    double* p = q + n + (N + 1);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double bi = (double)b[i];
        xs[i] = 0.0;
        r[i] = bi;
        p[i] = bi;
    }
    for (int e = threadIdx.x; e < N + 1; e += blockDim.x) p[-N - 1 + e] = p[n + e] = 0.0;
    __syncthreads();
    double rr = cg_dot(r, r, n, &red[0]);
    const double stop = cs.tol * sqrt(rr);
    for (int k = 0; k < cs.max_iter && sqrt(rr) > stop; ++k) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            double acc = 0.0;
#pragma unroll
            for (int kb = 0; kb < 9; ++kb)
                acc = fma(cs.bands[kb * cs.bs + i], p[i + (kb / 3 - 1) * N + (kb % 3 - 1)], acc);
            q[i] = acc;
        }
        __syncthreads();
        const double alpha = rr / cg_dot(p, q, n, &red[1]);
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            xs[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        __syncthreads();
        const double rr_new = cg_dot(r, r, n, &red[0]);
        const double beta = rr_new / rr;
        for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = r[i] + beta * p[i];
        __syncthreads();
        rr = rr_new;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = (T)xs[i];
}

// The coarsest solve by the configured method, one workgroup; x complete
// for every thread on return.
template <typename T>
__device__ __forceinline__ void coarse_block(const CoarseSolver& cs, int Nc, const T* b, T* x) {
    __shared__ double w[COARSE_LDS];
    __syncthreads();
    if (cs.cg)
        coarse_cg<T>(cs, Nc, b, x, w);
    else
        coarse_cholesky<T>(cs, Nc, b, x, w);
    __syncthreads();
}

// Sum of squares of one norm tile (elements base + e*BLOCK + tid, e < 4,
// added in e order).  The four loads go out together (a lane past n reads
// element 0 and adds zero, which leaves the sum unchanged).
template <typename T>
__device__ __forceinline__ double sumsq_tile(const T* __restrict__ v, int64_t n, int64_t base) {
    T w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t p = base + (int64_t)e * BLOCK + threadIdx.x;
        w[e] = v[p < n ? p : 0];
    }
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t p = base + (int64_t)e * BLOCK + threadIdx.x;
        s += p < n ? (double)w[e] * (double)w[e] : 0.0;
    }
    return s;
}

constexpr int64_t RED_SEG = 8192;  // partials per first-stage segment
constexpr int RED_MAX_SEGS = 2048;  // so at most 16M partials

// Thread-strided sum of p[lo, hi) then block_sum; valid in thread 0.  Each
// thread adds its elements in index order; eight loads are in flight at a
// time, so a long sum costs a few memory latencies rather than one per
// element.
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int64_t lo,
                                              int64_t hi) {
    constexpr int U = 8;
    double s = 0.0;
    int64_t i = lo + threadIdx.x;
    for (; i + (int64_t)(U - 1) * BLOCK < hi; i += (int64_t)U * BLOCK) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = p[i + (int64_t)u * BLOCK];
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u];
    }
    for (; i < hi; i += BLOCK) s += p[i];
    return block_sum(s);
}

// Fixed-order sum of np partials (one block); valid in thread 0.  Up to
// RED_SEG partials take one strided pass; more are summed in segments of
// RED_SEG whose sums are then summed the same way, which a grid of segment
// blocks followed by one final block reproduces bit for bit.
__device__ __forceinline__ double reduce_partials(const double* __restrict__ partials,
                                                  int64_t np) {
    if (np <= RED_SEG) return strided_sum(partials, 0, np);
    __shared__ double segs[RED_MAX_SEGS];
    const int64_t ns = (np + RED_SEG - 1) / RED_SEG;
    for (int64_t sg = 0; sg < ns; ++sg) {
        const double v = strided_sum(partials, sg * RED_SEG, min(np, (sg + 1) * RED_SEG));
        if (threadIdx.x == 0) segs[sg] = v;
    }
    __syncthreads();
    return strided_sum(segs, 0, ns);
}

}  // namespace dev
}  // namespace mg
