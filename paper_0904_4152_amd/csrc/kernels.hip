// gfx950 kernels of the Q1 multigrid Poisson hot path: grid and band
// assembly, the 9-band product family (SpMV, defect with norm, damped
// Jacobi), grid transfers, coarse direct solve and the mixed-precision
// cast / update steps.
//
// All band-streaming kernels are HBM-bandwidth bound (about 0.2-0.4 flop per
// byte), so they use no matrix cores: each thread owns 16 contiguous bytes of
// every band (4 floats or 2 doubles), bands are read with non-temporal loads
// (single use), the x halo of the three grid rows comes through L1/L2, and
// workgroups are renumbered so that each XCD walks a contiguous part of the
// grid (its L2 then sees the row reuse of x).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "device_ops.h"
#include "fused_ops.h"
#include "mg_internal.h"

namespace mg {

namespace {

using dev::BLOCK;
using dev::OP_DEFECT;
using dev::OP_JACOBI;
using dev::OP_SPMV;

// Hardware dispatches consecutive workgroups round-robin over the 8 XCDs.
// Renumber so that XCD k processes the k-th contiguous eighth of the grid;
// the launch grid is a multiple of 8 and surplus groups return at once.
__device__ __forceinline__ int64_t xcd_block(int64_t nblk) {
    const int64_t per = gridDim.x >> 3;
    const int64_t b = blockIdx.x;
    const int64_t lb = (b & 7) * per + (b >> 3);
    return lb < nblk ? lb : -1;
}

inline unsigned grid8(int64_t nblk) { return (unsigned)((nblk + 7) / 8 * 8); }

// Kernels of a guarded sequence (the mixed solve under device control, see
// red_control) take a guard pointer: a nonzero *guard makes the whole
// launch return at once.  Null: no guard.
__device__ __forceinline__ bool skipped(const double* guard) { return guard && *guard != 0.0; }

// Device control of the mixed solve (Sec. 6.2.2), taken by the thread that
// has just written a norm r = scal[slot + 1] (see RedCtl):
//   RED_OUTER (the FP64 defect of an outer step): the solve is over when r
//     is not finite, above c.div ||b|| (diverged), at most c.thr ||b||,
//     zero, or when c.cap is set (the step count is used up) -- the host
//     driver's own tests on the same values (||b|| = scal[SC_B + 1]).  Then
//     SC_CONV, SC_STOP and SC_WAIT are set, so everything queued after
//     returns at once.  Otherwise, with c.reset, the step's inner loop
//     starts: reduction factor c.ithr, cycle cap c.icap, no cycle run yet,
//     and the norm it is relative to, that of the scaled defect
//     (pow2_scale(||b||) r), into scal[SC_D32 + 1].
//   RED_ZFLAG (the count of nonzero initial iterate elements):
//     scal[SC_XZ] = 1 if the iterate is zero, else 0.
//   RED_STEP (an inner cycle's FP32 residual): count the cycle; the loop is
//     over when the residual is not finite, at most c.thr (= scal[SC_RED])
//     times the scaled defect's norm (scal[SC_D32 + 1]), or the cap is
//     reached.  The host mirror
//     gets the count, plus ITER_DONE once the loop is over, in one store.
__device__ void red_control(const RedCtl& c, double* __restrict__ scal, double* __restrict__ host,
                            double r) {
    if (c.mode == RED_OUTER) {
        const double bn = scal[SC_B + 1];
        const bool conv =
            !isfinite(r) || r > c.div * bn || r <= c.thr * bn || r == 0.0 || c.cap != 0;
        scal[SC_CONV] = conv ? 1.0 : 0.0;
        if (conv) {
            scal[SC_STOP] = 1.0;
            scal[SC_WAIT] = 1.0;
        } else if (c.reset) {
            scal[SC_STOP] = 0.0;
            scal[SC_WAIT] = 1.0;
            scal[SC_ITER] = 0.0;
            scal[SC_RED] = c.ithr;
            scal[SC_CAP] = (double)c.icap;
            scal[SC_D32 + 1] = dev::pow2_scale(bn) * r;
        }
    } else if (c.mode == RED_ZFLAG) {
        scal[SC_XZ] = r == 0.0 ? 1.0 : 0.0;
    } else if (c.mode == RED_STEP) {
        const double it = scal[SC_ITER] + 1.0;
        const bool done = !isfinite(r) || r <= scal[SC_RED] * scal[SC_D32 + 1] || it >= scal[SC_CAP];
        scal[SC_ITER] = it;
        scal[SC_STOP] = done ? 1.0 : 0.0;
        scal[SC_WAIT] = done ? 0.0 : 1.0;
        if (host) host[SC_ITER] = done ? it + ITER_DONE : it;
    }
}

// One tile per workgroup of the band product family (see dev::stencil_tile).
template <typename T, int OP, bool NORM, bool STORE, bool SYM = false>
__global__ __launch_bounds__(BLOCK) void k_stencil(const T* __restrict__ bands, int64_t bs,
                                                   int N, int64_t n, const T* __restrict__ x,
                                                   const T* __restrict__ b,
                                                   T* __restrict__ out, T omega,
                                                   double* __restrict__ partials, int64_t nblk,
                                                   const double* __restrict__ guard) {
    const int64_t lb = xcd_block(nblk);
    if (lb < 0 || skipped(guard)) return;
    const int64_t blo = lb * (int64_t)dev::tile_rows<T>();
    double sq;
    if constexpr (SYM)
        sq = dev::stencil_tile_staged<T, OP, NORM, STORE>(bands, bs, N, n, x, b, out, omega, blo);
    else
        sq = dev::stencil_tile<T, OP, NORM, STORE, SYM>(bands, bs, N, n, x, b, out, omega, blo);
    if (NORM) {
        const double s = dev::block_sum(sq);
        if (threadIdx.x == 0) partials[lb] = s;
    }
}

// The mixed scheme's FP64 defect (k_stencil's SYM defect with the norm),
// d written as float(d sc) into the FP32 right-hand side, sc =
// pow2_scale(||b||).
__global__ __launch_bounds__(BLOCK) void k_defect_cast(const double* __restrict__ bands,
                                                       int64_t bs, int N, int64_t n,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ b,
                                                       float* __restrict__ d32,
                                                       const double* __restrict__ scal,
                                                       double* __restrict__ partials,
                                                       int64_t nblk,
                                                       const double* __restrict__ guard) {
    const int64_t lb = xcd_block(nblk);
    if (lb < 0 || skipped(guard)) return;
    const dev::Cast32 cast{d32, dev::pow2_scale(scal[SC_B + 1])};
    const double sq = dev::stencil_tile_staged<double, OP_DEFECT, true, true, true>(
        bands, bs, N, n, x, b, nullptr, 0.0, lb * (int64_t)dev::tile_rows<double>(), cast);
    const double s = dev::block_sum(sq);
    if (threadIdx.x == 0) partials[lb] = s;
}

__global__ __launch_bounds__(BLOCK) void k_reduce_final(const double* __restrict__ partials,
                                                        int64_t np, double* __restrict__ scal,
                                                        int slot, double* __restrict__ host,
                                                        const double* __restrict__ guard,
                                                        RedCtl ctl) {
    if (skipped(guard)) return;
    const double s = dev::reduce_partials(partials, np);
    if (threadIdx.x == 0) {
        scal[slot] = s;
        scal[slot + 1] = sqrt(s);
        red_control(ctl, scal, host, sqrt(s));
        if (host) {
            host[slot] = s;
            host[slot + 1] = sqrt(s);
            __threadfence_system();
        }
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_jacobi_zero(const T* __restrict__ diag,
                                                       const T* __restrict__ b,
                                                       T* __restrict__ xo, int64_t n, T omega) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p < n) dev::jacobi_zero_elem(diag, b, xo, p, omega);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_restrict(int Nf, const T* __restrict__ d,
                                                    T* __restrict__ bc, int dmask) {
    const int Nc = (Nf >> 1) + 1;
    const int I = blockIdx.x * BLOCK + threadIdx.x;
    if (I < Nc) dev::restrict_elem(Nf, d, bc, I, (int)blockIdx.y, dmask);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_prolong(int Nf, const T* __restrict__ xc,
                                                   T* __restrict__ xf) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i < Nf) dev::prolong_elem(Nf, xc, xf, i, (int)blockIdx.y);
}

// Segmented reduction in one launch: one block per RED_SEG partials writes
// its segment's sum; the block that finishes last (an integer ticket counts
// the finished blocks) sums the segment sums as k_reduce_final would, and
// resets the ticket for the next reduction.  The fences order each block's
// segment sum before its ticket and the last block's reads after it, across
// the XCDs' caches.
__global__ __launch_bounds__(BLOCK) void k_reduce_segs(const double* __restrict__ partials,
                                                       int64_t np, double* __restrict__ segs,
                                                       unsigned* __restrict__ ticket,
                                                       double* __restrict__ scal, int slot,
                                                       double* __restrict__ host,
                                                       const double* __restrict__ guard,
                                                       RedCtl ctl) {
    if (skipped(guard)) return;
    const int64_t sg = blockIdx.x;
    const double v = dev::strided_sum(partials, sg * dev::RED_SEG,
                                      std::min<int64_t>(np, (sg + 1) * dev::RED_SEG));
    __shared__ unsigned last;
    if (threadIdx.x == 0) {
        segs[sg] = v;
        __threadfence();
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    const double s = dev::strided_sum(segs, 0, gridDim.x);
    if (threadIdx.x == 0) {
        scal[slot] = s;
        scal[slot + 1] = sqrt(s);
        red_control(ctl, scal, host, sqrt(s));
        *ticket = 0u;
        if (host) {
            host[slot] = s;
            host[slot + 1] = sqrt(s);
            __threadfence_system();
        }
    }
}


template <typename T>
__global__ void k_coarse(dev::CoarseSolver cs, int Nc, const T* __restrict__ b,
                         T* __restrict__ x) {
    dev::coarse_block<T>(cs, Nc, b, x);
}

// Fused pre-smoothing pass: one (strip, chunk) tile per workgroup of BT
// threads.
template <typename T, bool XZERO, int BT>
__global__ __launch_bounds__(BT) void k_pre(const T* __restrict__ bands, int64_t bs, int N,
                                            const T* __restrict__ x, const T* __restrict__ b,
                                            T omega, T* __restrict__ x2out, T* __restrict__ bc,
                                            int dmask, dev::FusedGeom g,
                                            const double* __restrict__ guard) {
    const int64_t lb = xcd_block((int64_t)g.nstrips * g.nchunks);
    if (lb < 0 || skipped(guard)) return;
    dev::pre_tile<T, XZERO, BT>(bands, bs, N, x, b, omega, x2out, bc, dmask,
                                (int)(lb % g.nstrips), (int)(lb / g.nstrips), g.rh, g.cw);
}

// Fused post-smoothing pass; with NORM the residual partials of
// dev::post_tile (one per group of F_NORM_ROWS rows and F_NORM_COLS
// columns, dev::fused_norm_parts(N) in all).
template <typename T, bool NORM, int BT>
__global__ __launch_bounds__(BT) void k_post(const T* __restrict__ bands, int64_t bs, int N,
                                             const T* __restrict__ x, const T* __restrict__ xc,
                                             const T* __restrict__ b, T omega,
                                             T* __restrict__ xout, double* __restrict__ partials,
                                             dev::FusedGeom g, const double* __restrict__ guard) {
    const int64_t lb = xcd_block((int64_t)g.nstrips * g.nchunks);
    if (lb < 0 || skipped(guard)) return;
    dev::post_tile<T, NORM, BT>(bands, bs, N, x, xc, b, omega, xout, partials,
                                (int)(lb % g.nstrips), (int)(lb / g.nstrips), g.rh, g.cw);
}

// The same passes in block tiles of BR x BC owned nodes.
template <typename T, bool XZERO, int BR, int BC>
__global__ __launch_bounds__(dev::BLK_THREADS) void k_pre_blk(
    const T* __restrict__ bands, int64_t bs, int N, const T* __restrict__ x,
    const T* __restrict__ b, T omega, T* __restrict__ x2out, T* __restrict__ bc, int dmask,
    dev::FusedGeom g, const double* __restrict__ guard) {
    const int64_t lb = xcd_block((int64_t)g.nstrips * g.nchunks);
    if (lb < 0 || skipped(guard)) return;
    __shared__ dev::BlockLds<T, BR, BC> s;
    dev::pre_block<T, XZERO, BR, BC>(s, bands, bs, N, x, b, omega, x2out, bc, dmask,
                                     (int)(lb % g.nstrips), (int)(lb / g.nstrips));
}

template <typename T, bool NORM, int BR, int BC>
__global__ __launch_bounds__(dev::BLK_THREADS) void k_post_blk(
    const T* __restrict__ bands, int64_t bs, int N, const T* __restrict__ x,
    const T* __restrict__ xc, const T* __restrict__ b, T omega, T* __restrict__ xout,
    double* __restrict__ partials, dev::FusedGeom g, const double* __restrict__ guard) {
    const int64_t lb = xcd_block((int64_t)g.nstrips * g.nchunks);
    if (lb < 0 || skipped(guard)) return;
    __shared__ dev::BlockLds<T, BR, BC> s;
    dev::post_block<T, NORM, BR, BC>(s, bands, bs, N, x, xc, b, omega, xout, partials,
                                     (int)(lb % g.nstrips), (int)(lb / g.nstrips));
}

// Coarse tail: the V(2,2) sub-cycle over levels top..Lc in one workgroup.
template <typename T>
__global__ __launch_bounds__(dev::TAIL_THREADS) void k_tail(dev::TailLevels<T> tl, T omega,
                                                             const double* __restrict__ guard) {
    if (skipped(guard)) return;
    dev::tail_cycle<T>(tl, omega);
}

// Dense Cholesky factor (lower triangle, row-major m x m) of the coarsest
// level's operator restricted to its unknowns, by one wavefront.  Unknowns
// are numbered in node order, so the matrix, and with it the factor, is
// banded: entries more than bw = Nc + 1 below the diagonal are zero and
// stay zero.  Column by column: lane 0 forms the pivot, then the lanes form
// the band's rows below it, each row's sum in increasing k as a plain dense
// factorisation would (the terms skipped below the band are exact zeros).
// At most 289 unknowns (level 4); flag = 1 if a pivot is not positive.
__global__ __launch_bounds__(64) void k_chol_factor(const double* __restrict__ bands, int64_t bs,
                                                    int Nc, int dmask, double* __restrict__ A,
                                                    int* __restrict__ flag) {
    __shared__ int idx[dev::COARSE_MAX_UNKNOWNS];  // node -> unknown (LDS: no scratch)
    __shared__ int m_s, bad_s;
    __shared__ double piv_s;
    const int tid = threadIdx.x;
    if (tid == 0) {
        int m = 0;
        for (int p = 0; p < Nc * Nc; ++p)
            idx[p] = dev::is_dirichlet(Nc, p % Nc, p / Nc, dmask) ? -1 : m++;
        m_s = m;
        bad_s = 0;
    }
    __syncthreads();
    const int m = m_s;
    const int bw = Nc + 1;
    for (int r = tid; r < m * m; r += 64) A[r] = 0.0;
    __syncthreads();
    for (int p = tid; p < Nc * Nc; p += 64) {
        const int r = idx[p];
        if (r < 0) continue;
        const int i = p % Nc, j = p / Nc;
        for (int k = 0; k < 9; ++k) {
            const int ii = i + k % 3 - 1, jj = j + k / 3 - 1;
            if (ii < 0 || jj < 0 || ii > Nc - 1 || jj > Nc - 1) continue;
            const int c = idx[jj * Nc + ii];
            if (c >= 0) A[r * m + c] = bands[k * bs + p];
        }
    }
    __syncthreads();
    for (int c = 0; c < m; ++c) {
        if (tid == 0) {
            double d = A[c * m + c];
            for (int k = max(0, c - bw); k < c; ++k) d -= A[c * m + k] * A[c * m + k];
            if (!(d > 0.0)) {
                bad_s = 1;
            } else {
                d = sqrt(d);
                A[c * m + c] = d;
                piv_s = d;
            }
        }
        __syncthreads();
        if (bad_s) break;
        const double d = piv_s;
        for (int r = c + 1 + tid; r < m && r <= c + bw; r += 64) {
            double t = A[r * m + c];
            for (int k = max(0, r - bw); k < c; ++k) t -= A[r * m + k] * A[c * m + k];
            A[r * m + c] = t / d;
        }
        __syncthreads();
    }
    if (tid == 0) *flag = bad_s;
}

// ---------------------------------------------------------------- geometry

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform01(uint64_t seed, uint64_t k) {
    return (double)(splitmix64(seed, k) >> 11) * 0x1.0p-53;
}

// Finest-level coordinates: uniform grid, interior nodes moved by
// (2u-1)*jitter*h in each direction.  Explicitly rounded operations keep
// the result identical to a host evaluation of the same formula.
__device__ __forceinline__ void coords_node(double* __restrict__ xy, int N, double jitter,
                                            uint64_t seed, int i, int j) {
    const int64_t p = (int64_t)j * N + i;
    const double h = 1.0 / (double)(N - 1);
    double x = __dmul_rn((double)i, h), y = __dmul_rn((double)j, h);
    if (jitter != 0.0 && i > 0 && j > 0 && i < N - 1 && j < N - 1) {
        const double ux = uniform01(seed, 2ull * (uint64_t)p);
        const double uy = uniform01(seed, 2ull * (uint64_t)p + 1ull);
        const double dx = __dmul_rn(__dmul_rn(__dadd_rn(2.0 * ux, -1.0), jitter), h);
        const double dy = __dmul_rn(__dmul_rn(__dadd_rn(2.0 * uy, -1.0), jitter), h);
        x = __dadd_rn(x, dx);
        y = __dadd_rn(y, dy);
    }
    xy[2 * p] = x;
    xy[2 * p + 1] = y;
}

__global__ __launch_bounds__(BLOCK) void k_coords(double* __restrict__ xy, int N, double jitter,
                                                  uint64_t seed) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i < N) coords_node(xy, N, jitter, seed, i, (int)blockIdx.y);
}

// Bilinear map of one quadrilateral written as
//   x(xi,eta) = ax0 + ax1 xi + ax2 eta + ax3 xi eta   (same for y),
// corners counter-clockwise (-1,-1), (1,-1), (1,1), (-1,1).
struct Quad {
    double ax[4], ay[4];
    __device__ void set(const double* cx, const double* cy) {
        ax[0] = 0.25 * ((cx[0] + cx[1]) + (cx[2] + cx[3]));
        ax[1] = 0.25 * ((cx[1] - cx[0]) + (cx[2] - cx[3]));
        ax[2] = 0.25 * ((cx[2] - cx[1]) + (cx[3] - cx[0]));
        ax[3] = 0.25 * ((cx[0] - cx[1]) + (cx[2] - cx[3]));
        ay[0] = 0.25 * ((cy[0] + cy[1]) + (cy[2] + cy[3]));
        ay[1] = 0.25 * ((cy[1] - cy[0]) + (cy[2] - cy[3]));
        ay[2] = 0.25 * ((cy[2] - cy[1]) + (cy[3] - cy[0]));
        ay[3] = 0.25 * ((cy[0] - cy[1]) + (cy[2] - cy[3]));
    }
};

__device__ __constant__ double kSX[4] = {-1.0, 1.0, 1.0, -1.0};
__device__ __constant__ double kSY[4] = {-1.0, -1.0, 1.0, 1.0};

// Element stiffness matrix (2x2 Gauss):
//   K[a][b] = sum_q (G_a G_b + H_a H_b) / det J_q
// with G = det J * d(phi)/dx and H = det J * d(phi)/dy expressed through
// the cofactors of J (one reciprocal of det J per quadrature point).  Each
// entry with b >= a is computed once and mirrored, so K is symmetric bit
// for bit.
__device__ void element_matrix(const Quad& q, double (&K)[4][4]) {
    const double g = 0.57735026918962576451;  // 1/sqrt(3)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) K[a][b] = 0.0;
#pragma unroll
    for (int qp = 0; qp < 4; ++qp) {
        const double xi = (qp & 1) ? g : -g;
        const double eta = (qp & 2) ? g : -g;
        const double xx = q.ax[1] + q.ax[3] * eta, xe = q.ax[2] + q.ax[3] * xi;
        const double yx = q.ay[1] + q.ay[3] * eta, ye = q.ay[2] + q.ay[3] * xi;
        const double det = xx * ye - xe * yx;
        const double inv = 1.0 / det;
        double G[4], H[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double dxi = 0.25 * kSX[c] * (1.0 + kSY[c] * eta);
            const double deta = 0.25 * kSY[c] * (1.0 + kSX[c] * xi);
            G[c] = ye * dxi - yx * deta;
            H[c] = xx * deta - xe * dxi;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = a; b < 4; ++b) K[a][b] += (G[a] * G[b] + H[a] * H[b]) * inv;
    }
#pragma unroll
    for (int a = 1; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < a; ++b) K[a][b] = K[b][a];
}

__device__ __forceinline__ void level_xy(const double* __restrict__ xyf, int Nf, int s, int i,
                                         int j, double* x, double* y) {
    const int64_t pf = (int64_t)(j * s) * Nf + (int64_t)(i * s);
    *x = xyf[2 * pf];
    *y = xyf[2 * pf + 1];
}

// All levels Lc..L of a hierarchy in one launch.  A workgroup assembles a
// tile of ATX x ATY nodes of one level: it first computes the stiffness
// matrices of the (ATX+1) x (ATY+1) elements touching the tile into LDS (one
// element per thread), then each of the first ATX*ATY threads sums the
// entries of its node's nine bands over the four elements around the node
// in lexicographic order and applies the Dirichlet treatment.  Writes FP64
// bands and their round-to-nearest FP32 copies; a tile row is 63
// consecutive nodes, so the band writes are long contiguous runs.  Level l
// owns the workgroups [first[l], first[l + 1]).
constexpr int ATX = 63, ATY = 3;
static_assert((ATX + 1) * (ATY + 1) == BLOCK, "one thread per element of a tile");

struct AssembleLevels {
    double* b64[MG_MAX_LEVEL + 1];
    float* b32[MG_MAX_LEVEL + 1];
    int64_t bs[MG_MAX_LEVEL + 1];
    int64_t first[MG_MAX_LEVEL + 2];
    int Lc, L;
    int dmask;  // Dirichlet sides
};

__global__ __launch_bounds__(BLOCK) void k_assemble(const double* __restrict__ xyf,
                                                    AssembleLevels a) {
    __shared__ double Ke[(ATX + 1) * (ATY + 1)][16];
    const int64_t blk = blockIdx.x;
    int l = a.Lc;
    while (l < a.L && blk >= a.first[l + 1]) ++l;
    const int N = (1 << l) + 1, Nf = (1 << a.L) + 1, s = 1 << (a.L - l);
    const int tiles_x = (N + ATX - 1) / ATX;
    const int64_t local = blk - a.first[l];
    const int i0 = (int)(local % tiles_x) * ATX, j0 = (int)(local / tiles_x) * ATY;
    {
        const int e = threadIdx.x;
        const int ei = i0 - 1 + e % (ATX + 1), ej = j0 - 1 + e / (ATX + 1);
        if (ei >= 0 && ej >= 0 && ei < N - 1 && ej < N - 1) {
            double cx[4], cy[4];
            level_xy(xyf, Nf, s, ei, ej, &cx[0], &cy[0]);
            level_xy(xyf, Nf, s, ei + 1, ej, &cx[1], &cy[1]);
            level_xy(xyf, Nf, s, ei + 1, ej + 1, &cx[2], &cy[2]);
            level_xy(xyf, Nf, s, ei, ej + 1, &cx[3], &cy[3]);
            Quad q;
            q.set(cx, cy);
            double K[4][4];
            element_matrix(q, K);
#pragma unroll
            for (int r = 0; r < 16; ++r) Ke[e][r] = K[r / 4][r % 4];
        }
    }
    __syncthreads();
    if ((int)threadIdx.x >= ATX * ATY) return;
    const int i = i0 + (int)threadIdx.x % ATX, j = j0 + (int)threadIdx.x / ATX;
    if (i >= N || j >= N) return;
    const int64_t p = (int64_t)j * N + i;
    double band[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) band[k] = 0.0;
    if (dev::is_dirichlet(N, i, j, a.dmask)) {
        band[4] = 1.0;
    } else {
        // element (ei,ej) = (i-1+ex, j-1+ey); this node is its corner c_node.
        // Elements outside the grid (nodes on a Neumann side) are absent.
        const int corner_of[4] = {2, 3, 1, 0};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ex = e & 1, ey = e >> 1;
            const int ei = i - 1 + ex, ej = j - 1 + ey;
            if (ei < 0 || ej < 0 || ei > N - 2 || ej > N - 2) continue;
            const double* K = Ke[(ej - j0 + 1) * (ATX + 1) + (ei - i0 + 1)];
            const int c_node = corner_of[e];
            // corner c sits at (ei + ox[c], ej + oy[c]); this node at (i, j)
            const int ox[4] = {0, 1, 1, 0}, oy[4] = {0, 0, 1, 1};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int di = ei + ox[c] - i, dj = ej + oy[c] - j;
                band[(dj + 1) * 3 + (di + 1)] += K[c_node * 4 + c];
            }
        }
        // couplings to Dirichlet nodes move to the right-hand side (zero
        // data); a select per band, with no divergent branch around it
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int ii = i + k % 3 - 1, jj = j + k / 3 - 1;
            const bool drop = k != 4 && dev::is_dirichlet(N, ii, jj, a.dmask);
            band[k] = drop ? 0.0 : band[k];
        }
    }
    double* b64 = a.b64[l];
    float* b32 = a.b32[l];
    const int64_t bs = a.bs[l];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        b64[k * bs + p] = band[k];
        b32[k * bs + p] = (float)band[k];
    }
}

// Load vector of f = 2 pi^2 sin(pi x) sin(pi y), 3x3 Gauss per element,
// node-centric over the four elements around each interior node.
__global__ __launch_bounds__(BLOCK) void k_rhs_sinsin(const double* __restrict__ xy, int N,
                                                      double* __restrict__ bout) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= N) return;
    const int64_t p = (int64_t)j * N + i;
    if (i == 0 || j == 0 || i == N - 1 || j == N - 1) {
        bout[p] = 0.0;
        return;
    }
    const double pi = 3.14159265358979323846;
    const double gp[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
    const double gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    const int corner_of[4] = {2, 3, 1, 0};
    double sum = 0.0;
    for (int e = 0; e < 4; ++e) {
        const int ei = i - 1 + (e & 1), ej = j - 1 + (e >> 1);
        double cx[4], cy[4];
        level_xy(xy, N, 1, ei, ej, &cx[0], &cy[0]);
        level_xy(xy, N, 1, ei + 1, ej, &cx[1], &cy[1]);
        level_xy(xy, N, 1, ei + 1, ej + 1, &cx[2], &cy[2]);
        level_xy(xy, N, 1, ei, ej + 1, &cx[3], &cy[3]);
        Quad q;
        q.set(cx, cy);
        const int a = corner_of[e];
        for (int qj = 0; qj < 3; ++qj) {
            for (int qi = 0; qi < 3; ++qi) {
                const double xi = gp[qi], eta = gp[qj];
                const double px = q.ax[0] + q.ax[1] * xi + q.ax[2] * eta + q.ax[3] * xi * eta;
                const double py = q.ay[0] + q.ay[1] * xi + q.ay[2] * eta + q.ay[3] * xi * eta;
                const double xx = q.ax[1] + q.ax[3] * eta, xe = q.ax[2] + q.ax[3] * xi;
                const double yx = q.ay[1] + q.ay[3] * eta, ye = q.ay[2] + q.ay[3] * xi;
                const double det = xx * ye - xe * yx;
                const double phi = 0.25 * (1.0 + kSX[a] * xi) * (1.0 + kSY[a] * eta);
                const double f = 2.0 * pi * pi * sin(pi * px) * sin(pi * py);
                sum += gw[qi] * gw[qj] * det * f * phi;
            }
        }
    }
    bout[p] = sum;
}

// Seeded uniform right-hand side (zero on the Dirichlet sides); with x0 also
// a zero initial iterate.
__device__ __forceinline__ void rhs_uniform_node(int N, uint64_t seed, int dmask,
                                                 double* __restrict__ bout,
                                                 double* __restrict__ x0, int i, int j) {
    const int64_t p = (int64_t)j * N + i;
    double v = 0.0;
    if (!dev::is_dirichlet(N, i, j, dmask)) v = 2.0 * uniform01(seed, (uint64_t)p) - 1.0;
    bout[p] = v;
    if (x0) x0[p] = 0.0;
}

__global__ __launch_bounds__(BLOCK) void k_rhs_uniform(int N, uint64_t seed, int dmask,
                                                       double* __restrict__ bout,
                                                       double* __restrict__ x0) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i < N) rhs_uniform_node(N, seed, dmask, bout, x0, i, (int)blockIdx.y);
}

// Both of the above in one launch (a served request's problem set-up).
__global__ __launch_bounds__(BLOCK) void k_coords_rhs(double* __restrict__ xy, int N,
                                                      double jitter, uint64_t gseed,
                                                      uint64_t rseed, int dmask,
                                                      double* __restrict__ bout,
                                                      double* __restrict__ x0) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= N) return;
    coords_node(xy, N, jitter, gseed, i, (int)blockIdx.y);
    rhs_uniform_node(N, rseed, dmask, bout, x0, i, (int)blockIdx.y);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_copy(const T* __restrict__ s, T* __restrict__ d,
                                                int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p < n) d[p] = s[p];
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_sumsq(const T* __restrict__ v, int64_t n,
                                                 double* __restrict__ partials, int64_t nblk) {
    const int64_t lb = xcd_block(nblk);
    if (lb < 0) return;
    const double s = dev::block_sum(dev::sumsq_tile(v, n, lb * (int64_t)dev::NORM_TILE));
    if (threadIdx.x == 0) partials[lb] = s;
}

// Number of nonzero elements per norm tile (as a double: exact).
__global__ __launch_bounds__(BLOCK) void k_count_nonzero(const double* __restrict__ v, int64_t n,
                                                         double* __restrict__ partials,
                                                         int64_t nblk) {
    const int64_t lb = xcd_block(nblk);
    if (lb < 0) return;
    double c = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t p = lb * (int64_t)dev::NORM_TILE + (int64_t)e * BLOCK + threadIdx.x;
        c += (p < n && v[p < n ? p : 0] != 0.0) ? 1.0 : 0.0;
    }
    const double s = dev::block_sum(c);
    if (threadIdx.x == 0) partials[lb] = s;
}

// The defect d = b - A x of a zero iterate, d = b, with the tiling, stores
// and norm partials of k_stencil<T, OP_DEFECT, NORM, STORE>: with x = 0 every
// band product sums exact zeros to +0 and b - (+0) = b, so the results are
// the same bits without reading the bands or x.
template <typename T, bool NORM, bool STORE>
__global__ __launch_bounds__(BLOCK) void k_defect_zero_x(int64_t n, const T* __restrict__ b,
                                                         T* __restrict__ out,
                                                         double* __restrict__ partials,
                                                         int64_t nblk,
                                                         const double* __restrict__ guard) {
    const int64_t lb = xcd_block(nblk);
    if (lb < 0 || skipped(guard)) return;
    const double sq =
        dev::copy_tile_sumsq<T>(b, STORE ? out : nullptr, n, lb * (int64_t)dev::tile_rows<T>());
    if (NORM) {
        const double s = dev::block_sum(sq);
        if (threadIdx.x == 0) partials[lb] = s;
    }
}

// k_defect_cast for a zero iterate (d = b).
__global__ __launch_bounds__(BLOCK) void k_defect_zero_x_cast(int64_t n,
                                                              const double* __restrict__ b,
                                                              float* __restrict__ d32,
                                                              const double* __restrict__ scal,
                                                              double* __restrict__ partials,
                                                              int64_t nblk,
                                                              const double* __restrict__ guard) {
    const int64_t lb = xcd_block(nblk);
    if (lb < 0 || skipped(guard)) return;
    const dev::Cast32 cast{d32, dev::pow2_scale(scal[SC_B + 1])};
    const double sq = dev::copy_tile_sumsq<double, true>(
        b, nullptr, n, lb * (int64_t)dev::tile_rows<double>(), cast);
    const double s = dev::block_sum(sq);
    if (threadIdx.x == 0) partials[lb] = s;
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fill(T* __restrict__ v, int64_t n, T value) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p < n) v[p] = value;
}

__global__ __launch_bounds__(BLOCK) void k_cast_scaled(const double* __restrict__ d,
                                                       float* __restrict__ d32, int64_t n,
                                                       const double* __restrict__ scal, int slot) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= n) return;
    const double s = scal[slot + 1];
    d32[p] = s > 0.0 ? (float)(d[p] / s) : 0.0f;
}

// x += u double(c), u = pow2_unscale(||b||): u c is exact, so the sum is
// the one rounding.  ZERO: x is taken as zero and not read (0.0 + u c, the
// same bits as the sum with a zeroed x, the sign of a zero included).
template <bool ZERO>
__global__ __launch_bounds__(BLOCK) void k_update(double* __restrict__ x,
                                                  const float* __restrict__ c, int64_t n,
                                                  const double* __restrict__ scal,
                                                  const double* __restrict__ guard) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= n || skipped(guard)) return;
    const double xo = ZERO ? 0.0 : x[p];
    x[p] = xo + dev::pow2_unscale(scal[SC_B + 1]) * (double)c[p];
}


// ---------------------------------------------------------------- Krylov
// Vector kernels of the preconditioned CG solver.  A preconditioned vector
// z is FP64, or an FP32 cycle result c with z = s double(c), s =
// scal[zslot + 1] (zslot >= 0).
template <typename TZ>
__device__ __forceinline__ double z_value(const TZ* __restrict__ z, int64_t p, double s) {
    return s * (double)z[p];
}
template <>
__device__ __forceinline__ double z_value<double>(const double* __restrict__ z, int64_t p,
                                                  double) {
    return z[p];
}

// Partial sums of u . z per norm tile.
template <typename TZ>
__global__ __launch_bounds__(BLOCK) void k_dot(const double* __restrict__ u,
                                               const TZ* __restrict__ z, int64_t n,
                                               const double* __restrict__ scal, int zslot,
                                               double* __restrict__ partials, int64_t nblk) {
    const int64_t lb = xcd_block(nblk);
    if (lb < 0) return;
    const double s = zslot >= 0 ? scal[zslot + 1] : 1.0;
    // loads first (lanes past n read element 0 and add zero), then the sum
    // in e order
    double uv[4], zv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t p = lb * (int64_t)dev::NORM_TILE + (int64_t)e * BLOCK + threadIdx.x;
        const int64_t q = p < n ? p : 0;
        uv[e] = u[q];
        zv[e] = z_value(z, q, s);
    }
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t p = lb * (int64_t)dev::NORM_TILE + (int64_t)e * BLOCK + threadIdx.x;
        acc += p < n ? uv[e] * zv[e] : 0.0;
    }
    const double t = dev::block_sum(acc);
    if (threadIdx.x == 0) partials[lb] = t;
}

// p = z + beta p, beta = scal[s_new] / scal[s_old] (0 for the first
// direction, where scal[s_old] is +inf).
template <typename TZ>
__global__ __launch_bounds__(BLOCK) void k_pcg_dir(double* __restrict__ pv,
                                                   const TZ* __restrict__ z, int64_t n,
                                                   const double* __restrict__ scal, int zslot,
                                                   int s_new, int s_old) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= n) return;
    const double s = zslot >= 0 ? scal[zslot + 1] : 1.0;
    const double beta = scal[s_new] / scal[s_old];
    pv[p] = z_value(z, p, s) + beta * pv[p];
}

// alpha = scal[s_num] / scal[s_den]; x += alpha p; r -= alpha q; partial
// sums of the new r^2 per norm tile.
__global__ __launch_bounds__(BLOCK) void k_pcg_step(double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ pv,
                                                    const double* __restrict__ q, int64_t n,
                                                    const double* __restrict__ scal, int s_num,
                                                    int s_den, double* __restrict__ partials,
                                                    int64_t nblk) {
    const int64_t lb = xcd_block(nblk);
    if (lb < 0) return;
    const double alpha = scal[s_num] / scal[s_den];
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t p = lb * (int64_t)dev::NORM_TILE + (int64_t)e * BLOCK + threadIdx.x;
        if (p < n) {
            x[p] += alpha * pv[p];
            const double rn = r[p] - alpha * q[p];
            r[p] = rn;
            acc += rn * rn;
        }
    }
    const double t = dev::block_sum(acc);
    if (threadIdx.x == 0) partials[lb] = t;
}

// scal[to], scal[to + 1] = scal[from], scal[from + 1] (one thread).
__global__ void k_scalar_copy(double* __restrict__ scal, int from, int to) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        scal[to] = scal[from];
        scal[to + 1] = scal[from + 1];
    }
}

inline unsigned blocks1d(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

}  // namespace

// scal[slot] = sum of the np partials (the order of dev::reduce_partials),
// scal[slot + 1] = its square root; the same into host[slot..] if not null.
// Segment sums go right after the partials, which the partials buffer leaves
// room for; the word before the buffer is the ticket of k_reduce_segs.
hipError_t launch_reduce(double* partials, int64_t np, double* scal, int slot, double* host,
                         hipStream_t st, const double* guard, RedCtl ctl) {
    if (np <= dev::RED_SEG) {
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(BLOCK), 0, st, partials, np, scal, slot,
                           host, guard, ctl);
        return hipGetLastError();
    }
    const int64_t ns = (np + dev::RED_SEG - 1) / dev::RED_SEG;
    if (ns > dev::RED_MAX_SEGS) return hipErrorInvalidValue;
    double* segs = partials + (np + 63) / 64 * 64;
    unsigned* ticket = reinterpret_cast<unsigned*>(partials - 1);
    hipLaunchKernelGGL(k_reduce_segs, dim3(ns), dim3(BLOCK), 0, st, partials, np, segs, ticket,
                       scal, slot, host, guard, ctl);
    return hipGetLastError();
}

int64_t stencil_blocks(int64_t n, int elem_bytes) {
    const int64_t per = (int64_t)BLOCK * (16 / elem_bytes);
    return (n + per - 1) / per;
}

int64_t norm_blocks(int64_t n) { return (n + dev::NORM_TILE - 1) / dev::NORM_TILE; }

hipError_t launch_coords(double* xy, int L, double jitter, uint64_t seed, hipStream_t st) {
    const int N = (1 << L) + 1;
    hipLaunchKernelGGL(k_coords, dim3(blocks1d(N), N), dim3(BLOCK), 0, st, xy, N, jitter, seed);
    return hipGetLastError();
}

hipError_t launch_coords_rhs(double* xy, int L, double jitter, uint64_t geom_seed,
                             uint64_t rhs_seed, int dmask, double* b, double* x0,
                             hipStream_t st) {
    const int N = (1 << L) + 1;
    hipLaunchKernelGGL(k_coords_rhs, dim3(blocks1d(N), N), dim3(BLOCK), 0, st, xy, N, jitter,
                       geom_seed, rhs_seed, dmask, b, x0);
    return hipGetLastError();
}

hipError_t launch_assemble(const double* xy_fine, const Level* lv, int Lc, int L, int dmask,
                           hipStream_t st) {
    AssembleLevels a{};
    a.Lc = Lc;
    a.L = L;
    a.dmask = dmask;
    int64_t nb = 0;
    for (int l = Lc; l <= L; ++l) {
        const int64_t N = (int64_t(1) << l) + 1;
        a.b64[l] = lv[l].bands64;
        a.b32[l] = lv[l].bands32;
        a.bs[l] = lv[l].bs;
        a.first[l] = nb;
        nb += ((N + ATX - 1) / ATX) * ((N + ATY - 1) / ATY);
    }
    a.first[L + 1] = nb;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)nb), dim3(BLOCK), 0, st, xy_fine, a);
    return hipGetLastError();
}

hipError_t launch_chol_factor(const Level& lc, int dmask, double* chol, int* flag,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_chol_factor, dim3(1), dim3(64), 0, st, lc.bands64, lc.bs, lc.N, dmask,
                       chol, flag);
    return hipGetLastError();
}

hipError_t launch_rhs_sinsin(const double* xy, int N, double* b, hipStream_t st) {
    hipLaunchKernelGGL(k_rhs_sinsin, dim3(blocks1d(N), N), dim3(BLOCK), 0, st, xy, N, b);
    return hipGetLastError();
}

hipError_t launch_rhs_uniform(int N, uint64_t seed, int dmask, double* b, double* x0,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_rhs_uniform, dim3(blocks1d(N), N), dim3(BLOCK), 0, st, N, seed, dmask,
                       b, x0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spmv(const Level& lv, const T* bands, const T* x, T* y, hipStream_t st,
                       bool sym) {
    const int64_t nb = stencil_blocks(lv.n, sizeof(T));
    if (sym)
        hipLaunchKernelGGL((k_stencil<T, OP_SPMV, false, true, true>), dim3(grid8(nb)),
                           dim3(BLOCK), 0, st, bands, lv.bs, lv.N, lv.n, x, (const T*)nullptr, y,
                           T(0), (double*)nullptr, nb, (const double*)nullptr);
    else
        hipLaunchKernelGGL((k_stencil<T, OP_SPMV, false, true>), dim3(grid8(nb)), dim3(BLOCK), 0,
                           st, bands, lv.bs, lv.N, lv.n, x, (const T*)nullptr, y, T(0),
                           (double*)nullptr, nb, (const double*)nullptr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_defect(const Level& lv, const T* bands, const T* b, const T* x, T* d,
                         double* partials, double* scal, int slot, double* host, hipStream_t st,
                         const double* guard, RedCtl ctl) {
    const int64_t nb = stencil_blocks(lv.n, sizeof(T));
    const dim3 g(grid8(nb)), blk(BLOCK);
    if (partials && d)
        hipLaunchKernelGGL((k_stencil<T, OP_DEFECT, true, true, true>), g, blk, 0, st, bands,
                           lv.bs, lv.N, lv.n, x, b, d, T(0), partials, nb, guard);
    else if (partials)
        hipLaunchKernelGGL((k_stencil<T, OP_DEFECT, true, false, true>), g, blk, 0, st, bands,
                           lv.bs, lv.N, lv.n, x, b, (T*)nullptr, T(0), partials, nb, guard);
    else
        hipLaunchKernelGGL((k_stencil<T, OP_DEFECT, false, true, true>), g, blk, 0, st, bands,
                           lv.bs, lv.N, lv.n, x, b, d, T(0), (double*)nullptr, nb, guard);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !partials) return e;
    return launch_reduce(partials, nb, scal, slot, host, st, guard, ctl);
}

template <typename T>
hipError_t launch_jacobi(const Level& lv, const T* bands, const T* b, const T* x, T* xo,
                         T omega, hipStream_t st) {
    const int64_t nb = stencil_blocks(lv.n, sizeof(T));
    hipLaunchKernelGGL((k_stencil<T, OP_JACOBI, false, true>), dim3(grid8(nb)), dim3(BLOCK), 0,
                       st, bands, lv.bs, lv.N, lv.n, x, b, xo, omega, (double*)nullptr, nb,
                       (const double*)nullptr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jacobi_zero(const Level& lv, const T* bands, const T* b, T* xo, T omega,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_jacobi_zero<T>, dim3(blocks1d(lv.n)), dim3(BLOCK), 0, st,
                       bands + 4 * lv.bs, b, xo, lv.n, omega);
    return hipGetLastError();
}

static int env_int(const char* name, int dflt) {
    const char* e = getenv(name);
    return e ? atoi(e) : dflt;
}

// Workgroup width of the fused passes on a level with N nodes per side: the
// width that covers a row with the fewest threads, ties to the wider one.
// MG_FUSED_BT (64, 128, 192 or 256) forces one width for every level.
int fused_bt(int N) {
    static const int forced = env_int("MG_FUSED_BT", 0);
    if (forced == 64 || forced == 128 || forced == 192 || forced == 256) return forced;
    int best = dev::F_MAX_THREADS;
    int64_t best_threads = INT64_MAX;
    for (int bt = dev::F_MAX_THREADS; bt >= dev::F_MIN_THREADS; bt -= 64) {
        const int64_t th = (int64_t)dev::fused_geom(N, bt, 2).nstrips * bt;
        if (th < best_threads) {
            best_threads = th;
            best = bt;
        }
    }
    return best;
}

int64_t fused_max_norm_parts(int N) { return dev::fused_norm_parts(N); }

// Owned rows per chunk of a fused pass over `count` problems on a level with
// N nodes per side: the longest chunk (a power of two from 64 down to 4)
// that still gives at least MG_FUSED_WAVES (default 3500, about 14 per
// compute unit) wavefronts, so that levels with little work keep the device
// busy and their marching pipelines short, and levels with much work waste
// little on the recomputed halo rows.  Chunk heights are multiples of
// F_NORM_ROWS.
int fused_rh(int N, int bt, int64_t count) {
    static const int64_t target = std::max(1, env_int("MG_FUSED_WAVES", 3500));
    const int64_t per_chunk = count * dev::fused_geom(N, bt, 4).nstrips * (bt / 64);
    int rh = 64;
    while (rh > 4 && per_chunk * ((N + rh - 1) / rh) < target) rh /= 2;
    return rh;
}

// The autotuner's trial of one level (per thread: the tuner launches from
// the calling thread only).
static thread_local int t_trial_N = 0, t_trial_rows = 0, t_trial_bt = 0, t_trial_cols = 0;

void set_single_trial(int N, int rows, int bt, int cols) {
    t_trial_N = rows && (bt || cols) ? N : 0;
    t_trial_rows = rows;
    t_trial_bt = bt;
    t_trial_cols = cols;
}

static int level_of(int N) {
    int l = 0;
    while ((1 << l) + 1 < N) ++l;
    return l;
}

dev::FusedGeom single_geom(int N) {
    int bt = 0, rh = 0, cols = 0;
    if (N == t_trial_N) {
        bt = t_trial_bt;
        rh = t_trial_rows;
        cols = t_trial_cols;
    } else {
        const TileEntry te = tile_table_get(level_of(N), 1);
        bt = te.bt;
        rh = te.rows;
        cols = te.cols;
    }
    if (const int shape = cols ? dev::block_shape(rh, cols) : 0) return dev::block_geom(N, shape);
    if (!bt) bt = fused_bt(N);
    if (!rh) rh = fused_rh(N, bt, 1);
    return dev::fused_geom(N, bt, rh);
}

int64_t fused_tiles(int N) {
    const dev::FusedGeom g = single_geom(N);
    return (int64_t)g.nstrips * g.nchunks;
}

#define MG_FUSED_BT_SWITCH(bt, LAUNCH) \
    switch (bt) {                      \
        case 64: LAUNCH(64); break;    \
        case 128: LAUNCH(128); break;  \
        case 192: LAUNCH(192); break;  \
        default: LAUNCH(256); break;   \
    }

template <typename T>
hipError_t launch_pre(const Level& lv, const T* bands, const T* x, bool x_zero, const T* b,
                      T omega, T* x2out, T* bc, int dmask, hipStream_t st, const double* guard) {
    const dev::FusedGeom g = single_geom(lv.N);
    const dim3 grid(grid8((int64_t)g.nstrips * g.nchunks)), block(g.bt);
#define PRE(BT)                                                                               \
    if (x_zero)                                                                               \
        hipLaunchKernelGGL((k_pre<T, true, BT>), grid, block, 0, st, bands, lv.bs, lv.N, x, b, \
                           omega, x2out, bc, dmask, g, guard);                                \
    else                                                                                      \
        hipLaunchKernelGGL((k_pre<T, false, BT>), grid, block, 0, st, bands, lv.bs, lv.N, x,   \
                           b, omega, x2out, bc, dmask, g, guard);
#define PRE_BLK(BR, BC)                                                                        \
    if (x_zero)                                                                                \
        hipLaunchKernelGGL((k_pre_blk<T, true, BR, BC>), grid, block, 0, st, bands, lv.bs,     \
                           lv.N, x, b, omega, x2out, bc, dmask, g, guard);                     \
    else                                                                                       \
        hipLaunchKernelGGL((k_pre_blk<T, false, BR, BC>), grid, block, 0, st, bands, lv.bs,    \
                           lv.N, x, b, omega, x2out, bc, dmask, g, guard);
    if (g.blk == 1) {
        PRE_BLK(8, 32)
    } else if (g.blk == 2) {
        PRE_BLK(16, 32)
    } else if (g.blk == 3) {
        PRE_BLK(32, 32)
    } else {
        MG_FUSED_BT_SWITCH(g.bt, PRE)
    }
#undef PRE_BLK
#undef PRE
    return hipGetLastError();
}

template <typename T>
hipError_t launch_post(const Level& lv, const T* bands, const T* x, const T* xc, const T* b,
                       T omega, T* xout, double* partials, double* scal, int slot, double* host,
                       hipStream_t st, const double* guard, RedCtl ctl) {
    const dev::FusedGeom g = single_geom(lv.N);
    const dim3 grid(grid8((int64_t)g.nstrips * g.nchunks)), block(g.bt);
#define POST(BT)                                                                             \
    if (partials)                                                                            \
        hipLaunchKernelGGL((k_post<T, true, BT>), grid, block, 0, st, bands, lv.bs, lv.N, x, \
                           xc, b, omega, xout, partials, g, guard);                          \
    else                                                                                     \
        hipLaunchKernelGGL((k_post<T, false, BT>), grid, block, 0, st, bands, lv.bs, lv.N,   \
                           x, xc, b, omega, xout, (double*)nullptr, g, guard);
#define POST_BLK(BR, BC)                                                                      \
    if (partials)                                                                             \
        hipLaunchKernelGGL((k_post_blk<T, true, BR, BC>), grid, block, 0, st, bands, lv.bs,   \
                           lv.N, x, xc, b, omega, xout, partials, g, guard);                  \
    else                                                                                      \
        hipLaunchKernelGGL((k_post_blk<T, false, BR, BC>), grid, block, 0, st, bands, lv.bs,  \
                           lv.N, x, xc, b, omega, xout, (double*)nullptr, g, guard);
    if (g.blk == 1) {
        POST_BLK(8, 32)
    } else if (g.blk == 2) {
        POST_BLK(16, 32)
    } else if (g.blk == 3) {
        POST_BLK(32, 32)
    } else {
        MG_FUSED_BT_SWITCH(g.bt, POST)
    }
#undef POST_BLK
#undef POST
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !partials) return e;
    return launch_reduce(partials, dev::fused_norm_parts(lv.N), scal, slot, host, st, guard, ctl);
}

template <typename T>
hipError_t launch_tail(const Level* lv, int top, int Lc, const dev::CoarseSolver& cs, T omega,
                       hipStream_t st, const double* guard) {
    dev::TailLevels<T> tl{};
    for (int l = Lc; l <= top; ++l) {
        dev::TailLevel<T>& d = tl.lv[l];
        const Level& v = lv[l];
        d.bands = std::is_same<T, float>::value ? (const T*)v.bands32 : (const T*)v.bands64;
        d.x = std::is_same<T, float>::value ? (T*)v.x32 : (T*)v.x64;
        d.b = std::is_same<T, float>::value ? (T*)v.b32 : (T*)v.b64;
        d.t = std::is_same<T, float>::value ? (T*)v.t32 : (T*)v.t64;
        d.bs = v.bs;
        d.n = v.n;
        d.N = v.N;
    }
    tl.cs = cs;
    tl.top = top;
    tl.Lc = Lc;
    hipLaunchKernelGGL(k_tail<T>, dim3(1), dim3(dev::TAIL_THREADS), 0, st, tl, omega, guard);
    return hipGetLastError();
}

int tail_max_level() { return dev::TAIL_MAX; }

template <typename T>
hipError_t launch_restrict(int Nf, const T* d_f, T* b_c, int dmask, hipStream_t st) {
    const int Nc = (Nf >> 1) + 1;
    hipLaunchKernelGGL(k_restrict<T>, dim3(blocks1d(Nc), Nc), dim3(BLOCK), 0, st, Nf, d_f, b_c,
                       dmask);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(int Nf, const T* x_c, T* x_f, hipStream_t st) {
    hipLaunchKernelGGL(k_prolong<T>, dim3(blocks1d(Nf), Nf), dim3(BLOCK), 0, st, Nf, x_c, x_f);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse(const dev::CoarseSolver& cs, int Nc, const T* b, T* x, hipStream_t st) {
    hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(64), 0, st, cs, Nc, b, x);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(const T* src, T* dst, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_copy<T>, dim3(blocks1d(n)), dim3(BLOCK), 0, st, src, dst, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_norm(const T* v, int64_t n, double* partials, double* scal, int slot,
                       double* host, hipStream_t st) {
    const int64_t nb = norm_blocks(n);
    hipLaunchKernelGGL(k_sumsq<T>, dim3(grid8(nb)), dim3(BLOCK), 0, st, v, n, partials, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(partials, nb, scal, slot, host, st);
}

hipError_t launch_count_nonzero(const double* v, int64_t n, double* partials, double* scal,
                                int slot, double* host, hipStream_t st, RedCtl ctl) {
    const int64_t nb = norm_blocks(n);
    hipLaunchKernelGGL(k_count_nonzero, dim3(grid8(nb)), dim3(BLOCK), 0, st, v, n, partials, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(partials, nb, scal, slot, host, st, nullptr, ctl);
}

hipError_t launch_defect_zero_x(const Level& lv, const double* b, double* d, double* partials,
                                double* scal, int slot, double* host, hipStream_t st,
                                const double* guard, RedCtl ctl) {
    const int64_t nb = stencil_blocks(lv.n, sizeof(double));
    const dim3 g(grid8(nb)), blk(BLOCK);
    if (d)
        hipLaunchKernelGGL((k_defect_zero_x<double, true, true>), g, blk, 0, st, lv.n, b, d,
                           partials, nb, guard);
    else
        hipLaunchKernelGGL((k_defect_zero_x<double, true, false>), g, blk, 0, st, lv.n, b,
                           (double*)nullptr, partials, nb, guard);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(partials, nb, scal, slot, host, st, guard, ctl);
}

template <typename T>
hipError_t launch_fill(T* v, int64_t n, T value, hipStream_t st) {
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks1d(n)), dim3(BLOCK), 0, st, v, n, value);
    return hipGetLastError();
}

hipError_t launch_cast_scaled(const double* d64, float* d32, int64_t n, const double* scal,
                              int slot, hipStream_t st) {
    hipLaunchKernelGGL(k_cast_scaled, dim3(blocks1d(n)), dim3(BLOCK), 0, st, d64, d32, n, scal,
                       slot);
    return hipGetLastError();
}

hipError_t launch_update(double* x, const float* c32, int64_t n, const double* scal,
                         hipStream_t st, const double* guard, bool x_zero) {
    if (x_zero)
        hipLaunchKernelGGL(k_update<true>, dim3(blocks1d(n)), dim3(BLOCK), 0, st, x, c32, n, scal,
                           guard);
    else
        hipLaunchKernelGGL(k_update<false>, dim3(blocks1d(n)), dim3(BLOCK), 0, st, x, c32, n,
                           scal, guard);
    return hipGetLastError();
}

hipError_t launch_defect_cast(const Level& lv, const double* bands, const double* b,
                              const double* x, float* d32, double* partials, double* scal,
                              int slot, double* host, hipStream_t st, const double* guard,
                              RedCtl ctl) {
    const int64_t nb = stencil_blocks(lv.n, sizeof(double));
    hipLaunchKernelGGL(k_defect_cast, dim3(grid8(nb)), dim3(BLOCK), 0, st, bands, lv.bs, lv.N,
                       lv.n, x, b, d32, scal, partials, nb, guard);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(partials, nb, scal, slot, host, st, guard, ctl);
}

hipError_t launch_defect_zero_x_cast(const Level& lv, const double* b, float* d32,
                                     double* partials, double* scal, int slot, double* host,
                                     hipStream_t st, const double* guard, RedCtl ctl) {
    const int64_t nb = stencil_blocks(lv.n, sizeof(double));
    hipLaunchKernelGGL(k_defect_zero_x_cast, dim3(grid8(nb)), dim3(BLOCK), 0, st, lv.n, b, d32,
                       scal, partials, nb, guard);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(partials, nb, scal, slot, host, st, guard, ctl);
}


template <typename TZ>
hipError_t launch_dot(const double* u, const TZ* z, int64_t n, const double* zscal, int zslot,
                      double* partials, double* scal, int slot, hipStream_t st) {
    const int64_t nb = norm_blocks(n);
    hipLaunchKernelGGL(k_dot<TZ>, dim3(grid8(nb)), dim3(BLOCK), 0, st, u, z, n, zscal, zslot,
                       partials, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(partials, nb, scal, slot, nullptr, st);
}
template hipError_t launch_dot<double>(const double*, const double*, int64_t, const double*, int,
                                       double*, double*, int, hipStream_t);
template hipError_t launch_dot<float>(const double*, const float*, int64_t, const double*, int,
                                      double*, double*, int, hipStream_t);

template <typename TZ>
hipError_t launch_pcg_dir(double* p, const TZ* z, int64_t n, const double* scal, int zslot,
                          int s_new, int s_old, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_dir<TZ>, dim3(blocks1d(n)), dim3(BLOCK), 0, st, p, z, n, scal, zslot,
                       s_new, s_old);
    return hipGetLastError();
}
template hipError_t launch_pcg_dir<double>(double*, const double*, int64_t, const double*, int,
                                           int, int, hipStream_t);
template hipError_t launch_pcg_dir<float>(double*, const float*, int64_t, const double*, int,
                                          int, int, hipStream_t);

hipError_t launch_pcg_step(double* x, double* r, const double* p, const double* q, int64_t n,
                           double* scal, int s_num, int s_den, double* partials, int slot,
                           double* host, hipStream_t st) {
    const int64_t nb = norm_blocks(n);
    hipLaunchKernelGGL(k_pcg_step, dim3(grid8(nb)), dim3(BLOCK), 0, st, x, r, p, q, n, scal,
                       s_num, s_den, partials, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(partials, nb, scal, slot, host, st);
}

hipError_t launch_scalar_copy(double* scal, int from, int to, hipStream_t st) {
    hipLaunchKernelGGL(k_scalar_copy, dim3(1), dim3(64), 0, st, scal, from, to);
    return hipGetLastError();
}

#define MG_INSTANTIATE(T)                                                                     \
    template hipError_t launch_spmv<T>(const Level&, const T*, const T*, T*, hipStream_t, bool); \
    template hipError_t launch_defect<T>(const Level&, const T*, const T*, const T*, T*,      \
                                         double*, double*, int, double*, hipStream_t,         \
                                         const double*, RedCtl);                              \
    template hipError_t launch_jacobi<T>(const Level&, const T*, const T*, const T*, T*, T,   \
                                         hipStream_t);                                        \
    template hipError_t launch_jacobi_zero<T>(const Level&, const T*, const T*, T*, T,        \
                                              hipStream_t);                                   \
    template hipError_t launch_restrict<T>(int, const T*, T*, int, hipStream_t);              \
    template hipError_t launch_prolong<T>(int, const T*, T*, hipStream_t);                    \
    template hipError_t launch_coarse<T>(const dev::CoarseSolver&, int, const T*, T*,         \
                                         hipStream_t);                                        \
    template hipError_t launch_copy<T>(const T*, T*, int64_t, hipStream_t);                   \
    template hipError_t launch_norm<T>(const T*, int64_t, double*, double*, int, double*,     \
                                       hipStream_t);                                          \
    template hipError_t launch_fill<T>(T*, int64_t, T, hipStream_t);                          \
    template hipError_t launch_pre<T>(const Level&, const T*, const T*, bool, const T*, T, T*,  \
                                      T*, int, hipStream_t, const double*);                     \
    template hipError_t launch_post<T>(const Level&, const T*, const T*, const T*, const T*, T, \
                                       T*, double*, double*, int, double*, hipStream_t,       \
                                       const double*, RedCtl);                                \
    template hipError_t launch_tail<T>(const Level*, int, int, const dev::CoarseSolver&, T,    \
                                       hipStream_t, const double*);

MG_INSTANTIATE(float)
MG_INSTANTIATE(double)

}  // namespace mg
