// Batched mixed-precision multigrid: many independent problems of different
// levels advance together.  Every V-cycle stage (a sweep, a defect, a
// transfer at one level) is one persistent launch over a work list of
// (problem, tile) items covering every problem that has that level; the
// problems are aligned at the coarse end, so one coarse-solve launch serves
// them all.  Per-problem control (outer defect with the scaled FP32 cast,
// inner cycles, update,
// stop tests of Sec. 6.2's mixed scheme) is a state machine advanced on the
// device by tiny controller kernels, so one iteration is a fixed sequence of
// launches: it is captured once into a HIP graph and replayed.  A problem's
// arithmetic uses the same per-tile device functions and the same
// reduction order as the single-problem solver, so its result does not
// depend on the other problems in the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <unordered_set>

#include "batch.h"
#include "device_ops.h"
#include "fused_ops.h"

namespace mg {

namespace {

using dev::BLOCK;

constexpr int NLISTS = 52;
constexpr int WL_FINEST = 32;
constexpr int WL_ALL = 33;
constexpr int WL_FINEST_COARSE = 50;  // finest tiles of problems with L = Lc
constexpr int WL_SEGS32 = 51;         // segments of the fused passes' residual partials
inline int wl_level(int l) { return l; }
inline int wl_restrict(int l) { return 16 + l; }
inline int wl_fused(int l) { return 34 + l; }

constexpr int STAGE_GRID = 2048;
constexpr int TILE = 1024;  // elements per work item (one FP32 stencil tile)

enum { K_NORM = 0, K_S32 = 1, K_S64 = 2 };
enum { F_BN = 0, F_S = 1, F_R32 = 3 };
enum { PH_INIT = 0, PH_OUTER = 2, PH_INNER = 4 };

// Work list: wl[0] = count, wl[1] = cap, prob[cap] at wl+2, tile prefix
// start[cap+1] at wl+2+cap.  Item t belongs to the last k with start[k] <= t.
__device__ __forceinline__ int wl_total(const int* wl) { return wl[2 + wl[1] + wl[0]]; }

//
// Found by a 64-way search: each round the wavefront's lanes test 64 evenly
// spaced entries of the range at once and keep the segment after the last
// one that is <= t (the entries are non-decreasing and start[0] = 0), so a
// list of up to 4096 problems takes two rounds of loads, not twelve
// dependent ones.  Every lane of the wavefront must call it with the same t.
__device__ __forceinline__ int find_last_le(const int* a, int count, int t) {
    const int lane = (int)(threadIdx.x & 63);
    int lo = 0, len = count;
    while (len > 1) {
        const int step = (len + 63) >> 6;
        const int off = lane * step;
        const bool ok = off < len && a[lo + off] <= t;
        const int last = 63 - __clzll(__ballot(ok));  // lane 0 always holds
        lo += last * step;
        len = min(step, len - last * step);
    }
    return lo;
}

__device__ __forceinline__ void wl_item(const int* wl, int t, int* p, int* tile) {
    const int cap = wl[1];
    const int* start = wl + 2 + cap;
    const int k = find_last_le(start, wl[0], t);
    *p = wl[2 + k];
    *tile = t - start[k];
}

// Compacted items: the items of the listed problems whose flags meet mask,
// in list order.  Every workgroup reads the flags of all listed problems
// (entries split in runs over its BLOCK threads) and writes cum[k] = active
// items of the entries before k; item t of the compacted list belongs to
// the last entry k with cum[k] <= t.  Returns the number of active items.
// Lists of up to ACTIVE_MAX problems; every thread of the workgroup calls it.
constexpr int ACTIVE_MAX = 4096;

__device__ int active_prefix(const int* wl, const BState* __restrict__ state, int mask,
                             int* cum) {
    __shared__ int wsum[BLOCK / 64];
    const int count = wl[0], cap = wl[1];
    const int* prob = wl + 2;
    const int* start = wl + 2 + cap;
    const int per = (count + BLOCK - 1) / BLOCK;
    const int k0 = min((int)threadIdx.x * per, count), k1 = min(k0 + per, count);
    int mine = 0;
    for (int k = k0; k < k1; ++k)
        mine += (state[prob[k]].flags & mask) ? start[k + 1] - start[k] : 0;
    // exclusive scan of the threads' sums: within each wavefront, then
    // across the wavefronts
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    int inc = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(inc, o, 64);
        if (lane >= o) inc += v;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / 64; ++i) {
        base += i < w ? wsum[i] : 0;
        total += wsum[i];
    }
    int run = base + inc - mine;
    for (int k = k0; k < k1; ++k) {
        cum[k] = run;
        run += (state[prob[k]].flags & mask) ? start[k + 1] - start[k] : 0;
    }
    __syncthreads();
    return total;
}

__device__ __forceinline__ float* role32(const BLevel& lv, int r) { return r ? lv.t32 : lv.x32; }

// Work items of list wl for the problems whose flags meet `mask`.  The
// whole launch returns at once when no problem has any of those flags:
// state[cap] holds the union of every live problem's flags, written by the
// control kernel after each phase (and set to all bits when new problems
// are uploaded).
#define FOR_ITEMS(wl)                                              \
    if (!(state[wl[1]].flags & mask)) return;                      \
    const int total_ = wl_total(wl);                               \
    for (int t_ = blockIdx.x; t_ < total_; t_ += gridDim.x) {      \
        int p, tile;                                               \
        wl_item(wl, t_, &p, &tile);                                \
        const BProb& P = probs[p];                                 \
        const int flags = state[p].flags;

// The same for the listed problems whose flags meet `mask` only: the items
// of the others are never visited (see active_prefix).
#define FOR_ACTIVE_ITEMS(wl)                                                           \
    if (!(state[wl[1]].flags & mask)) return;                                          \
    __shared__ int cum_[ACTIVE_MAX];                                                   \
    const bool compact_ = wl[0] <= ACTIVE_MAX;                                         \
    const int total_ = compact_ ? active_prefix(wl, state, mask, cum_) : wl_total(wl); \
    for (int t_ = blockIdx.x; t_ < total_; t_ += gridDim.x) {                          \
        int p, tile;                                                                   \
        if (compact_) {                                                                \
            const int k_ = find_last_le(cum_, wl[0], t_);                              \
            p = wl[2 + k_];                                                            \
            tile = t_ - cum_[k_];                                                      \
        } else {                                                                       \
            wl_item(wl, t_, &p, &tile);                                                \
        }                                                                              \
        const BProb& P = probs[p];                                                     \
        const int flags = state[p].flags;

#define END_ITEMS }

// First pre-smoothing sweep at level l: from a zero iterate on every level
// below the problem's finest and on the finest level at the first inner
// cycle of an outer step; otherwise a full sweep src -> dst.
__global__ __launch_bounds__(BLOCK) void kb_pre1(const BProb* __restrict__ probs,
                                                 const BState* __restrict__ state,
                                                 const int* __restrict__ wl, int l, int src,
                                                 int dst, int mask) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& lv = P.lv[l];
    const float om = (float)P.omega;
    const int64_t base = (int64_t)tile * TILE;
    if (l < P.L || state[p].first) {
        const float* diag = lv.bands32 + 4 * lv.bs;
        float* xo = role32(lv, dst);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t q = base + (int64_t)e * BLOCK + threadIdx.x;
            if (q < lv.n) dev::jacobi_zero_elem(diag, (const float*)lv.b32, xo, q, om);
        }
    } else {
        dev::stencil_tile<float, dev::OP_JACOBI, false, true>(lv.bands32, lv.bs, lv.N, lv.n,
                                                              role32(lv, src), lv.b32,
                                                              role32(lv, dst), om, base);
    }
    END_ITEMS
}

// Zero the iterate where the first sweep would start from zero (only used
// when there is no pre-smoothing).
__global__ __launch_bounds__(BLOCK) void kb_fill_cond(const BProb* __restrict__ probs,
                                                      const BState* __restrict__ state,
                                                      const int* __restrict__ wl, int l, int dst,
                                                      int mask) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    if (!(l < P.L || state[p].first)) continue;
    const BLevel& lv = P.lv[l];
    float* xo = role32(lv, dst);
    const int64_t base = (int64_t)tile * TILE;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t q = base + (int64_t)e * BLOCK + threadIdx.x;
        if (q < lv.n) xo[q] = 0.0f;
    }
    END_ITEMS
}

template <int OP>
__global__ __launch_bounds__(BLOCK) void kb_band(const BProb* __restrict__ probs,
                                                 const BState* __restrict__ state,
                                                 const int* __restrict__ wl, int l, int src,
                                                 int dst, int mask) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& lv = P.lv[l];
    dev::stencil_tile<float, OP, false, true>(lv.bands32, lv.bs, lv.N, lv.n, role32(lv, src),
                                              lv.b32, role32(lv, dst), (float)P.omega,
                                              (int64_t)tile * TILE);
    END_ITEMS
}

__global__ __launch_bounds__(BLOCK) void kb_restrict(const BProb* __restrict__ probs,
                                                     const BState* __restrict__ state,
                                                     const int* __restrict__ wl, int l, int src,
                                                     int mask) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& f = P.lv[l];
    const BLevel& c = P.lv[l - 1];
    const int64_t base = (int64_t)tile * TILE;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t q = base + (int64_t)e * BLOCK + threadIdx.x;
        if (q < c.n)
            dev::restrict_elem<float>(f.N, role32(f, src), c.b32, (int)(q % c.N), (int)(q / c.N),
                                      P.dmask);
    }
    END_ITEMS
}

__global__ __launch_bounds__(BLOCK) void kb_prolong(const BProb* __restrict__ probs,
                                                    const BState* __restrict__ state,
                                                    const int* __restrict__ wl, int l, int dst,
                                                    int mask) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& f = P.lv[l];
    const BLevel& c = P.lv[l - 1];
    const int64_t base = (int64_t)tile * TILE;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t q = base + (int64_t)e * BLOCK + threadIdx.x;
        if (q < f.n)
            dev::prolong_elem<float>(f.N, c.x32, role32(f, dst), (int)(q % f.N), (int)(q / f.N));
    }
    END_ITEMS
}

__global__ __launch_bounds__(BLOCK) void kb_copy(const BProb* __restrict__ probs,
                                                 const BState* __restrict__ state,
                                                 const int* __restrict__ wl, int l, int src,
                                                 int dst, int mask) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& lv = P.lv[l];
    const float* s = role32(lv, src);
    float* d = role32(lv, dst);
    const int64_t base = (int64_t)tile * TILE;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t q = base + (int64_t)e * BLOCK + threadIdx.x;
        if (q < lv.n) d[q] = s[q];
    }
    END_ITEMS
}

// Coarse tail of every problem above the coarse level (one block each): the
// sub-cycle over levels min(L - 1, TAIL_MAX) .. Lc.  The levels' descriptors
// are staged in LDS: the cycle indexes them by a run-time level, which in
// registers would put them in per-lane scratch memory.
__global__ __launch_bounds__(dev::TAIL_THREADS) void kb_tail(const BProb* __restrict__ probs,
                                                 const BState* __restrict__ state,
                                                 const int* __restrict__ wl, int Lc, int mask) {
    __shared__ dev::TailLevels<float> tl;
    FOR_ITEMS(wl)
    if (!(flags & mask) || P.L <= Lc) continue;
    __syncthreads();  // the previous item's cycle has read tl
    if (threadIdx.x == 0) {
        const int top = min(P.L - 1, dev::TAIL_MAX);
        for (int l = Lc; l <= top; ++l) {
            const BLevel& v = P.lv[l];
            tl.lv[l] = dev::TailLevel<float>{v.bands32, v.x32, v.b32, v.t32, v.bs, v.n, v.N, 0};
        }
        tl.cs = P.cs;
        tl.top = top;
        tl.Lc = Lc;
    }
    __syncthreads();
    dev::tail_cycle<float>(tl, (float)P.omega);
    END_ITEMS
}

// Coarsest level (one block per problem); with only_level >= 0 only for the
// problems whose finest level is only_level.
__global__ __launch_bounds__(BLOCK) void kb_coarse(const BProb* __restrict__ probs,
                                                   const BState* __restrict__ state,
                                                   const int* __restrict__ wl, int Lc, int mask,
                                                   int only_level) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    if (only_level >= 0 && P.L != only_level) continue;
    const BLevel& lv = P.lv[Lc];
    dev::coarse_block<float>(P.cs, lv.N, lv.b32, lv.x32);
    END_ITEMS
}

// Fused pre-smoothing pass at level l (two sweeps, defect, restriction) for
// the problems in their inner loop; iterate x -> t, coarse rhs at l-1.
template <int BT>
__global__ __launch_bounds__(BT) void kb_fpre(const BProb* __restrict__ probs,
                                              const BState* __restrict__ state,
                                              const int* __restrict__ wl, int l, int mask) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& lv = P.lv[l];
    const int strip = tile % lv.nstrips, chunk = tile / lv.nstrips;
    const float om = (float)P.omega;
    if (l < P.L || state[p].first)
        dev::pre_tile<float, true, BT>(lv.bands32, lv.bs, lv.N, lv.x32, lv.b32, om, lv.t32,
                                       P.lv[l - 1].b32, P.dmask, strip, chunk, lv.rh, lv.cw);
    else
        dev::pre_tile<float, false, BT>(lv.bands32, lv.bs, lv.N, lv.x32, lv.b32, om, lv.t32,
                                        P.lv[l - 1].b32, P.dmask, strip, chunk, lv.rh, lv.cw);
    END_ITEMS
}

// Fused post-smoothing pass at level l (prolongation, two sweeps: t -> x);
// on the problem's finest level also the residual-norm partials.
template <int BT>
__global__ __launch_bounds__(BT) void kb_fpost(const BProb* __restrict__ probs,
                                               const BState* __restrict__ state,
                                               const int* __restrict__ wl, int l, int mask) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& lv = P.lv[l];
    const int strip = tile % lv.nstrips, chunk = tile / lv.nstrips;
    const float om = (float)P.omega;
    if (l == P.L)
        dev::post_tile<float, true, BT>(lv.bands32, lv.bs, lv.N, lv.t32, P.lv[l - 1].x32, lv.b32,
                                        om, lv.x32, P.partials, strip, chunk, lv.rh, lv.cw);
    else
        dev::post_tile<float, false, BT>(lv.bands32, lv.bs, lv.N, lv.t32, P.lv[l - 1].x32,
                                         lv.b32, om, lv.x32, nullptr, strip, chunk, lv.rh, lv.cw);
    END_ITEMS
}

// The same passes in block tiles of BR x BC owned nodes.
template <int BR, int BC>
__global__ __launch_bounds__(dev::BLK_THREADS) void kb_fpre_blk(const BProb* __restrict__ probs,
                                                               const BState* __restrict__ state,
                                                               const int* __restrict__ wl, int l,
                                                               int mask) {
    __shared__ dev::BlockLds<float, BR, BC> s;
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& lv = P.lv[l];
    const int strip = tile % lv.nstrips, chunk = tile / lv.nstrips;
    const float om = (float)P.omega;
    if (l < P.L || state[p].first)
        dev::pre_block<float, true, BR, BC>(s, lv.bands32, lv.bs, lv.N, lv.x32, lv.b32, om,
                                            lv.t32, P.lv[l - 1].b32, P.dmask, strip, chunk);
    else
        dev::pre_block<float, false, BR, BC>(s, lv.bands32, lv.bs, lv.N, lv.x32, lv.b32, om,
                                             lv.t32, P.lv[l - 1].b32, P.dmask, strip, chunk);
    END_ITEMS
}

template <int BR, int BC>
__global__ __launch_bounds__(dev::BLK_THREADS) void kb_fpost_blk(const BProb* __restrict__ probs,
                                                                const BState* __restrict__ state,
                                                                const int* __restrict__ wl, int l,
                                                                int mask) {
    __shared__ dev::BlockLds<float, BR, BC> s;
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& lv = P.lv[l];
    const int strip = tile % lv.nstrips, chunk = tile / lv.nstrips;
    const float om = (float)P.omega;
    if (l == P.L)
        dev::post_block<float, true, BR, BC>(s, lv.bands32, lv.bs, lv.N, lv.t32,
                                             P.lv[l - 1].x32, lv.b32, om, lv.x32, P.partials,
                                             strip, chunk);
    else
        dev::post_block<float, false, BR, BC>(s, lv.bands32, lv.bs, lv.N, lv.t32,
                                              P.lv[l - 1].x32, lv.b32, om, lv.x32, nullptr, strip,
                                              chunk);
    END_ITEMS
}

// FP32 residual norm of the inner iterate on the finest level (partials);
// with only_level >= 0 only for problems whose finest level is only_level.
__global__ __launch_bounds__(BLOCK) void kb_inner_norm(const BProb* __restrict__ probs,
                                                       const BState* __restrict__ state,
                                                       const int* __restrict__ wl, int mask,
                                                       int only_level) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    if (only_level >= 0 && P.L != only_level) continue;
    const BLevel& lv = P.lv[P.L];
    const double sq = dev::stencil_tile<float, dev::OP_DEFECT, true, false, true>(
        lv.bands32, lv.bs, lv.N, lv.n, lv.x32, lv.b32, nullptr, 0.0f, (int64_t)tile * TILE);
    const double s = dev::block_sum(sq);
    if (threadIdx.x == 0) P.partials[tile] = s;
    END_ITEMS
}

// FP64 defect d = b - A x on the finest level with norm partials, written
// as float(d sc) into the finest FP32 right-hand side (sc = pow2_scale of
// ||b||, as the single-problem mixed solve writes it): two FP64 stencil
// tiles (512 rows each) per work item.
__global__ __launch_bounds__(BLOCK) void kb_outer_defect(const BProb* __restrict__ probs,
                                                         const BState* __restrict__ state,
                                                         const int* __restrict__ wl, int mask) {
    FOR_ACTIVE_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& lv = P.lv[P.L];
    // the first defect of a zero initial iterate is b (b - A 0 gives the
    // same bits): b is copied and its squares summed in the tile's order
    const bool zero_x = state[p].outer == 0 && !(flags & BF_UPDATE) && state[p].xnz == 0;
    const dev::Cast32 cast{lv.b32, dev::pow2_scale(state[p].bn)};
    for (int sub = 0; sub < 2; ++sub) {
        const int64_t blo = (int64_t)(2 * tile + sub) * dev::tile_rows<double>();
        const double sq =
            zero_x ? dev::copy_tile_sumsq<double, true>(lv.b64, nullptr, lv.n, blo, cast)
                   : dev::stencil_tile<double, dev::OP_DEFECT, true, true, true, true>(
                         lv.bands64, lv.bs, lv.N, lv.n, lv.x64, lv.b64, nullptr, 0.0, blo, cast);
        const double s = dev::block_sum(sq);
        if (threadIdx.x == 0) P.partials[2 * tile + sub] = s;
    }
    END_ITEMS
}

// Sum-of-squares partials of b64 (which = 0) or of the scaled FP32 defect
// (which = 1) on the finest level.  With which = 0 (a new problem) also
// whether the initial iterate x64 has a nonzero entry (state.xnz, an
// integer OR over the tiles), so that its first defect can be b itself; a
// zero guess is known to be zero (x64 is not read).
__global__ __launch_bounds__(BLOCK) void kb_sumsq(const BProb* __restrict__ probs,
                                                  BState* __restrict__ state,
                                                  const int* __restrict__ wl, int which,
                                                  int mask) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& lv = P.lv[P.L];
    const int64_t base = (int64_t)tile * dev::NORM_TILE;
    const double sq = which == 0 ? dev::sumsq_tile<double>(lv.b64, lv.n, base)
                                 : dev::sumsq_tile<float>(lv.b32, lv.n, base);
    if (which == 0 && !P.zero_guess) {
        int nz = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t q = base + (int64_t)e * BLOCK + threadIdx.x;
            nz |= q < lv.n && lv.x64[q] != 0.0;
        }
        if (__syncthreads_or(nz) && threadIdx.x == 0) atomicOr(&state[p].xnz, 1);
    }
    const double s = dev::block_sum(sq);
    if (threadIdx.x == 0) P.partials[tile] = s;
    END_ITEMS
}

// x64 += u double(c32), u = pow2_unscale(||b||) (the single solve's
// update); a zero guess's first update takes x64 as zero without reading
// it (0.0 + u c, as the single solve's).
__global__ __launch_bounds__(BLOCK) void kb_update(const BProb* __restrict__ probs,
                                                   const BState* __restrict__ state,
                                                   const int* __restrict__ wl, int mask) {
    FOR_ACTIVE_ITEMS(wl)
    if (!(flags & mask)) continue;
    const BLevel& lv = P.lv[P.L];
    const double s = dev::pow2_unscale(state[p].bn);
    const bool x_zero = P.zero_guess && state[p].outer == 0;
    const int64_t base = (int64_t)tile * TILE;
    double xv[4];  // loads first; lanes past n read element 0 and store nothing
    float cv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t q = base + (int64_t)e * BLOCK + threadIdx.x;
        const int64_t r = q < lv.n ? q : 0;
        xv[e] = x_zero ? 0.0 : lv.x64[r];
        cv[e] = lv.x32[r];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t q = base + (int64_t)e * BLOCK + threadIdx.x;
        if (q < lv.n) lv.x64[q] = xv[e] + s * (double)cv[e];
    }
    END_ITEMS
}

// x64 = 0 on every listed problem whose solution is zero but whose x64 no
// update wrote: a zero right-hand side (solved at once), or a zero guess
// (x64 not read) that stopped before its first update.
__global__ __launch_bounds__(BLOCK) void kb_zero_unwritten(const BProb* __restrict__ probs,
                                                           const BState* __restrict__ state,
                                                           const int* __restrict__ wl) {
    const int total = wl_total(wl);
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        int p, tile;
        wl_item(wl, t, &p, &tile);
        const BProb& P = probs[p];
        const BState& S = state[p];
        const bool zero = (S.bn == 0.0 && S.status == MG_OK) || (P.zero_guess && S.outer == 0);
        if (!zero) continue;
        const BLevel& lv = P.lv[P.L];
        const int64_t base = (int64_t)tile * TILE;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t q = base + (int64_t)e * BLOCK + threadIdx.x;
            if (q < lv.n) lv.x64[q] = 0.0;
        }
    }
}

// Residual partials of problem P's finest level: the fused post pass's
// above the coarse level, the defect tiles' on it.
__device__ __forceinline__ int64_t s32_parts(const BProb& P, int fused_above) {
    const BLevel& F = P.lv[P.L];
    if (fused_above >= 0 && P.L > fused_above) return dev::fused_norm_parts(F.N);
    return (F.n + TILE - 1) / TILE;
}

// First stage of the inner residual's fixed-order sum for problems with more
// than dev::RED_SEG partials: one work item per segment of RED_SEG partials,
// its sum right after the partials (padded to 64), as k_reduce_segs does.
__global__ __launch_bounds__(BLOCK) void kb_segsum(const BProb* __restrict__ probs,
                                                   const BState* __restrict__ state,
                                                   const int* __restrict__ wl, int mask,
                                                   int fused_above) {
    FOR_ITEMS(wl)
    if (!(flags & mask)) continue;
    const int64_t np = s32_parts(P, fused_above);
    const int64_t lo = (int64_t)tile * dev::RED_SEG;
    const double v = dev::strided_sum(P.partials, lo, min(np, lo + dev::RED_SEG));
    if (threadIdx.x == 0) P.partials[(np + 63) / 64 * 64 + tile] = v;
    END_ITEMS
}

// Per-problem transition of the mixed scheme at the end of a phase:
// INIT -> OUTER (or DONE), OUTER -> CAST or DONE (a problem whose inner
// loop ended in this iteration's update counts its outer step first), CAST
// -> INNER, INNER -> INNER or UPDATE.
__device__ void transition(const BProb& P, BState& S, int phase) {
    const int f = S.flags;
    if (phase == PH_INIT && (f & BF_INIT)) {
        if (!isfinite(S.bn)) {
            S.status = MG_ERR_NUMERIC;
            S.flags = BF_DONE;
        } else if (S.bn == 0.0) {
            S.status = MG_OK;
            S.flags = BF_DONE;
        } else {
            S.flags = BF_OUTER;
        }
    } else if (phase == PH_OUTER && (f & (BF_OUTER | BF_UPDATE))) {
        if (f & BF_UPDATE) S.outer += 1;  // its update ran in this iteration
        const int k = S.outer + 1;
        const double rel = S.s / S.bn;
        if (k > 1 && S.n_hist < MG_HIST) S.hist[S.n_hist++] = rel;
        int done = 0;
        if (!isfinite(S.s) || S.s > 1e3 * S.bn) {
            S.status = MG_ERR_NUMERIC;
            done = 1;
        } else if (P.fixed > 0) {
            done = k > P.fixed;
        } else if (S.s <= P.rel_tol * S.bn) {
            done = 1;
        } else if (k > P.max_outer) {
            S.status = MG_ERR_NOCONV;
            done = 1;
        }
        if (!done && S.s == 0.0) done = 1;
        if (done) {
            S.flags = BF_DONE;
        } else {
            // the defect kernel wrote the scaled FP32 right-hand side: the
            // inner loop starts, relative to the scaled defect's norm
            S.dn = dev::pow2_scale(S.bn) * S.s;
            S.first = 1;
            S.it = 0;
            S.flags = BF_INNER;
        }
    } else if (phase == PH_INNER && (f & BF_INNER)) {
        S.it += 1;
        S.cycles += 1;
        S.first = 0;
        if (!isfinite(S.r32) || S.r32 <= P.inner_reduction * S.dn || S.it >= P.inner_max)
            S.flags = BF_UPDATE;
    }
}

// Norm of each problem in the phase from its partials (fixed order), into a
// state field, and the problem's transition.  The inner residual (K_S32)
// of a problem with more than dev::RED_SEG partials adds the segment sums of
// kb_segsum (the same order as summing the partials here).
__device__ void finalize_items(const BProb* __restrict__ probs, BState* __restrict__ state,
                               const int* __restrict__ wl, int kind, int field, int mask,
                               int fused_above, int phase) {
    const int total = wl_total(wl);
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        int p, tile;
        wl_item(wl, t, &p, &tile);
        const BProb& P = probs[p];
        if (!(state[p].flags & mask)) continue;
        const BLevel& F = P.lv[P.L];
        const int64_t n = F.n;
        int64_t np = kind == K_S64
                         ? (n + dev::tile_rows<double>() - 1) / dev::tile_rows<double>()
                         : (n + TILE - 1) / TILE;
        if (kind == K_S32) np = s32_parts(P, fused_above);
        const double s =
            (kind == K_S32 && np > dev::RED_SEG)
                ? dev::strided_sum(P.partials + (np + 63) / 64 * 64, 0,
                                   (np + dev::RED_SEG - 1) / dev::RED_SEG)
                : dev::reduce_partials(P.partials, np);
        if (threadIdx.x == 0) {
            const double r = sqrt(s);
            BState& S = state[p];
            if (field == F_BN)
                S.bn = r;
            else if (field == F_S)
                S.s = r;
            else
                S.r32 = r;
            transition(P, S, phase);
        }
    }
}

// After a phase's transitions (one block; thread per slot): the union of
// every live problem's flags into state[cap] (the early exit of the stage
// kernels), and at the end of an iteration (PH_INNER) the report to the
// host, in entry k mod ITER_RING of the pinned ring (k = iterations so far;
// entries of 2 + cap ints): the problems not done, those still in their
// inner loop, which cannot finish in the next iteration (a problem finishes
// only at an outer step), and every slot's flags (0 for an empty slot).
__device__ void report_all(const BProb* __restrict__ probs, BState* __restrict__ state, int cap,
                           int phase, int* __restrict__ iter, int* __restrict__ ring) {
    int live = 0, sure = 0, present = 0;
    int* entry = nullptr;
    if (phase == PH_INNER) entry = ring + (int64_t)(*iter % ITER_RING) * (2 + cap);
    for (int p = threadIdx.x; p < cap; p += BLOCK) {
        if (probs[p].L == 0) {
            if (entry) entry[2 + p] = 0;
            continue;
        }
        const int f = state[p].flags;
        if (!(f & BF_DONE)) ++live;
        if (f == BF_INNER) ++sure;
        present |= f;
        if (entry) entry[2 + p] = f;
    }
    {
        __shared__ int wor[BLOCK / 64];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) present |= __shfl_xor(present, o, 64);
        if ((threadIdx.x & 63) == 0) wor[threadIdx.x >> 6] = present;
        __syncthreads();
        if (threadIdx.x == 0) {
            int v = 0;
#pragma unroll
            for (int w = 0; w < BLOCK / 64; ++w) v |= wor[w];
            state[cap].flags = v;
        }
    }
    if (phase == PH_INNER) {
        __threadfence_system();
        const double tot = dev::block_sum((double)live);
        const double tsure = dev::block_sum((double)sure);
        if (threadIdx.x == 0) {
            *iter = *iter + 1;
            entry[0] = (int)tot;
            entry[1] = (int)tsure;
            __threadfence_system();
        }
    }
}

// The norms of a phase and each problem's transition (finalize_items),
// then, in the block that finishes last (an integer ticket counts the
// finished blocks; fences order every block's writes before its ticket and
// the last block's reads after it), the flags' union and the report
// (report_all).  The ticket is back to zero after.
__global__ __launch_bounds__(BLOCK) void kb_finctl(const BProb* __restrict__ probs,
                                                   BState* __restrict__ state,
                                                   const int* __restrict__ wl, int kind,
                                                   int field, int mask, int fused_above,
                                                   int phase, int* __restrict__ iter,
                                                   int* __restrict__ ring,
                                                   unsigned* __restrict__ ticket) {
    if (state[wl[1]].flags & mask)
        finalize_items(probs, state, wl, kind, field, mask, fused_above, phase);
    __shared__ unsigned last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    report_all(probs, state, wl[1], phase, iter, ring);
    if (threadIdx.x == 0) *ticket = 0u;
}

}  // namespace

BatchEngine::~BatchEngine() {
    for (hipGraphExec_t g : graph_)
        if (g) (void)hipGraphExecDestroy(g);
    if (st_) (void)hipStreamDestroy(st_);
    if (d_probs_) (void)hipFree(d_probs_);
    if (d_state_) (void)hipFree(d_state_);
    if (d_wl_) (void)hipFree(d_wl_);
    if (setup_st_) (void)hipStreamDestroy(setup_st_);
    if (read_st_) (void)hipStreamDestroy(read_st_);
    for (hipEvent_t e : ev_)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev_upload_)
        if (e) (void)hipEventDestroy(e);
    if (ev_setup_) (void)hipEventDestroy(ev_setup_);
    if (d_iter_) (void)hipFree(d_iter_);
    if (h_state_) (void)hipHostFree(h_state_);
    if (h_ring_) (void)hipHostFree(h_ring_);
    for (int b = 0; b < 2; ++b) {
        if (h_probs_stage_[b]) (void)hipHostFree(h_probs_stage_[b]);
        if (h_wl_stage_[b]) (void)hipHostFree(h_wl_stage_[b]);
        if (h_start_stage_[b]) (void)hipHostFree(h_start_stage_[b]);
    }
    if (h_fetch_) (void)hipHostFree(h_fetch_);
}

mg_status BatchEngine::init(int device, int capacity, int Lmax, int Lc, int nu_pre,
                            int nu_post) {
    if (capacity < 1 || capacity > 65536) return fail(MG_ERR_INVALID, "batch capacity out of range");
    device_ = device;
    cap_ = capacity;
    Lmax_ = Lmax;
    Lc_ = Lc;
    nu_pre_ = nu_pre;
    nu_post_ = nu_post;
    MG_HIP(hipSetDevice(device));
    MG_HIP(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
    MG_HIP(hipStreamCreateWithFlags(&setup_st_, hipStreamNonBlocking));
    MG_HIP(hipStreamCreateWithFlags(&read_st_, hipStreamNonBlocking));
    MG_HIP(hipEventCreateWithFlags(&ev_setup_, hipEventDisableTiming));
    for (hipEvent_t& e : ev_upload_) MG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const size_t wl_ints = (size_t)NLISTS * (3 + 2 * cap_);
    for (int b = 0; b < 2; ++b) {
        MG_HIP(hipHostMalloc((void**)&h_probs_stage_[b], sizeof(BProb) * cap_,
                             hipHostMallocDefault));
        MG_HIP(hipHostMalloc((void**)&h_wl_stage_[b], sizeof(int) * wl_ints, hipHostMallocDefault));
        MG_HIP(hipHostMalloc((void**)&h_start_stage_[b], sizeof(BState) * (cap_ + 1),
                             hipHostMallocDefault));
    }
    MG_HIP(hipHostMalloc((void**)&h_fetch_, sizeof(BState), hipHostMallocDefault));
    MG_HIP(hipMalloc(&d_probs_, sizeof(BProb) * cap_));
    MG_HIP(hipMalloc(&d_state_, sizeof(BState) * (cap_ + 1)));  // + flags union
    MG_HIP(hipMalloc(&d_wl_, sizeof(int) * NLISTS * (3 + 2 * cap_)));
    MG_HIP(hipMalloc(&d_iter_, 64));
    MG_HIP(hipMemset(d_iter_, 0, 64));
    launched_ = 0;
    for (hipEvent_t& e : ev_) MG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    MG_HIP(hipHostMalloc((void**)&h_state_, sizeof(BState) * cap_, hipHostMallocDefault));
    const size_t ring_ints = (size_t)ITER_RING * (2 + cap_);
    MG_HIP(hipHostMalloc((void**)&h_ring_, sizeof(int) * ring_ints, hipHostMallocDefault));
    std::memset(h_ring_, 0, sizeof(int) * ring_ints);
    hp_.assign(cap_, BProb{});
    started_.assign(cap_, 0);
    for (int l = 1; l <= MG_MAX_LEVEL; ++l) bt_[l] = graph_bt_[l] = fused_bt((1 << l) + 1);
    std::memset(h_state_, 0, sizeof(BState) * cap_);
    for (int s = 0; s < cap_; ++s) h_state_[s].flags = BF_DONE;
    MG_HIP(hipMemcpy(d_state_, h_state_, sizeof(BState) * cap_, hipMemcpyHostToDevice));
    {
        BState all{};
        all.flags = -1;
        MG_HIP(hipMemcpy(d_state_ + cap_, &all, sizeof(BState), hipMemcpyHostToDevice));
    }
    probs_dirty_ = true;
    return MG_OK;
}

void BatchEngine::set_slot(int s, mg_hierarchy* h, const mg_solve_opts& o, const double* b,
                           double* x) {
    BProb P{};
    for (int l = h->Lc; l <= h->L; ++l) {
        const Level& v = h->lv[l];
        BLevel& b = P.lv[l];
        b.bands64 = v.bands64;
        b.bands32 = v.bands32;
        b.x64 = v.x64;
        b.b64 = v.b64;
        b.x32 = v.x32;
        b.b32 = v.b32;
        b.t32 = v.t32;
        b.bs = v.bs;
        b.n = v.n;
        b.N = v.N;
        // chunk height: set by build_lists from the composition
        const dev::FusedGeom g = dev::fused_geom(v.N, fused_bt(v.N), 4);
        b.rh = g.rh;
        b.cw = g.cw;
        b.bt = g.bt;
        b.nstrips = g.nstrips;
        b.nchunks = g.nchunks;
        b.blk = 0;
    }
    P.partials = h->partials;
    P.cs = coarse_solver(h);
    P.dmask = h->dmask;
    P.L = h->L;
    P.omega = o.omega;
    P.rel_tol = o.rel_tol;
    P.inner_reduction = o.inner_reduction;
    P.inner_max = o.inner_max_cycles;
    P.max_outer = o.max_cycles;
    P.fixed = o.fixed_cycles;
    P.zero_guess = o.zero_guess;
    if (b) {
        P.lv[P.L].b64 = const_cast<double*>(b);
        P.lv[P.L].x64 = x;
    }
    hp_[s] = P;
    probs_dirty_ = true;
}

void BatchEngine::clear_slot(int s) {
    hp_[s] = BProb{};
    started_[s] = 0;
    probs_dirty_ = true;
}

void BatchEngine::start_slot(int s) { started_[s] = 1; }

namespace {
struct TileTable {
    std::mutex mu;
    std::map<std::pair<int, int>, TileEntry> rows;  // (level, log2 problems) -> tile
    std::atomic<uint64_t> epoch{1};
};
TileTable& tile_table() {
    static TileTable* t = new TileTable();
    return *t;
}
int log2_floor(int64_t v) {
    int k = 0;
    while (v > 1) {
        v >>= 1;
        ++k;
    }
    return k;
}
}  // namespace

TileEntry tile_table_get(int level, int64_t problems) {
    TileTable& t = tile_table();
    std::lock_guard<std::mutex> g(t.mu);
    auto it = t.rows.find({level, log2_floor(problems)});
    return it == t.rows.end() ? TileEntry{0, 0, 0} : it->second;
}

void tile_table_set(int level, int64_t problems, int rows, int bt, int cols) {
    TileTable& t = tile_table();
    std::lock_guard<std::mutex> g(t.mu);
    t.rows[{level, log2_floor(problems)}] = {rows, bt, cols};
    ++t.epoch;
}

void tile_table_clear() {
    TileTable& t = tile_table();
    std::lock_guard<std::mutex> g(t.mu);
    t.rows.clear();
    ++t.epoch;
}

uint64_t tile_table_epoch() { return tile_table().epoch.load(); }

int BatchEngine::problems_at(int l) const {
    int count = 0;
    for (int s = 0; s < cap_; ++s)
        if (hp_[s].L >= l && (l > dev::TAIL_MAX || l == hp_[s].L)) ++count;
    return count;
}

// Work lists of the current composition.
void BatchEngine::build_lists() {
    const int stride = 3 + 2 * cap_;
    h_wl_.assign((size_t)NLISTS * stride, 0);
    auto fill = [&](int id, auto eligible, auto tiles) {
        int* w = h_wl_.data() + (size_t)id * stride;
        int count = 0, acc = 0;
        int* prob = w + 2;
        int* start = w + 2 + cap_;
        for (int s = 0; s < cap_; ++s) {
            if (hp_[s].L == 0 || !eligible(hp_[s])) continue;
            prob[count] = s;
            start[count] = acc;
            acc += tiles(hp_[s]);
            ++count;
        }
        start[count] = acc;
        w[0] = count;
        w[1] = cap_;
    };
    auto ntiles = [](int64_t n) { return (int)((n + TILE - 1) / TILE); };
    auto fused_here = [](const BProb& P, int l) {
        return P.L >= l && (l > dev::TAIL_MAX || l == P.L);
    };
    // tiles of the fused passes for this composition: every problem at a
    // level shares one chunk height and one workgroup width (no result bit
    // depends on either): a choice under trial by the autotuner, else the
    // tuned one, else the rules (fewest threads per row; ~3500 wavefronts)
    for (int l = Lc_ + 1; l <= Lmax_; ++l) {
        int64_t count = 0;
        for (int s = 0; s < cap_; ++s)
            if (hp_[s].L > 0 && fused_here(hp_[s], l)) ++count;
        if (count == 0) continue;
        const int N = (1 << l) + 1;
        const TileEntry te = tile_table_get(l, count);
        int bt = bt_override_[l] ? bt_override_[l] : (tuned_widths_ ? te.bt : 0);
        if (!bt) bt = fused_bt(N);
        int rh = rh_override_[l] ? rh_override_[l] : te.rows;
        if (!rh) rh = fused_rh(N, bt, count);
        const int cols = rh_override_[l] ? cols_override_[l] : (tuned_widths_ ? te.cols : 0);
        const int shape = cols ? dev::block_shape(rh, cols) : 0;
        const dev::FusedGeom g = shape ? dev::block_geom(N, shape) : dev::fused_geom(N, bt, rh);
        bt_[l] = g.bt;
        blk_[l] = g.blk;
        for (int s = 0; s < cap_; ++s) {
            if (hp_[s].L == 0 || !fused_here(hp_[s], l)) continue;
            BLevel& v = hp_[s].lv[l];
            v.rh = g.rh;
            v.nchunks = g.nchunks;
            v.bt = g.bt;
            v.cw = g.cw;
            v.nstrips = g.nstrips;
            v.blk = g.blk;
        }
    }
    for (int l = Lc_ + 1; l <= Lmax_; ++l) {
        fill(wl_level(l), [&](const BProb& P) { return P.L >= l; },
             [&](const BProb& P) { return ntiles(P.lv[l].n); });
        fill(wl_restrict(l), [&](const BProb& P) { return P.L >= l; },
             [&](const BProb& P) { return ntiles(P.lv[l - 1].n); });
        // fused passes run above the coarse tail: on levels > TAIL_MAX and on
        // the problem's finest level
        fill(wl_fused(l), [&](const BProb& P) { return fused_here(P, l); },
             [&](const BProb& P) { return P.lv[l].nstrips * P.lv[l].nchunks; });
    }
    fill(WL_FINEST, [](const BProb&) { return true; },
         [&](const BProb& P) { return ntiles(P.lv[P.L].n); });
    fill(WL_FINEST_COARSE, [&](const BProb& P) { return P.L == Lc_; },
         [&](const BProb& P) { return ntiles(P.lv[P.L].n); });
    fill(WL_ALL, [](const BProb&) { return true; }, [](const BProb&) { return 1; });
    {
        // inner-residual partials per problem (as kb_finalize counts them)
        const bool fused = nu_pre_ == 2 && nu_post_ == 2;
        auto parts = [&](const BProb& P) -> int64_t {
            const BLevel& F = P.lv[P.L];
            if (fused && P.L > Lc_) return dev::fused_norm_parts(F.N);
            return (F.n + TILE - 1) / TILE;
        };
        fill(WL_SEGS32, [&](const BProb& P) { return parts(P) > dev::RED_SEG; },
             [&](const BProb& P) {
                 return (int)((parts(P) + dev::RED_SEG - 1) / dev::RED_SEG);
             });
    }
    // optional launches this composition needs; a new one invalidates the graph
    uint32_t need = 0;
    for (int l = Lc_ + 1; l <= Lmax_; ++l)
        if (h_wl_[(size_t)wl_fused(l) * stride] > 0) need |= 1u << l;
    if (h_wl_[(size_t)WL_FINEST_COARSE * stride] > 0) need |= 1u;
    if (h_wl_[(size_t)WL_SEGS32 * stride] > 0) need |= 1u << 31;
    bool widths_changed = false;
    for (int l = Lc_ + 1; l <= Lmax_; ++l)
        if (bt_[l] != graph_bt_[l] || blk_[l] != graph_blk_[l]) widths_changed = true;
    if ((need & ~launch_mask_) || widths_changed) {
        launch_mask_ |= need;
        for (hipGraphExec_t& g : graph_) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    }
}

// Stream-ordered: launches after this call see the new descriptors, lists
// and started states, and wait for the work enqueued on setup_stream() so
// far.  Host data goes through one of two pinned staging areas, each reused
// only after its previous copies have completed.
mg_status BatchEngine::upload_async() {
    MG_HIP(hipSetDevice(device_));
    MG_HIP(hipEventRecord(ev_setup_, setup_st_));
    MG_HIP(hipStreamWaitEvent(st_, ev_setup_, 0));
    const int b = ubuf_;
    ubuf_ ^= 1;
    MG_HIP(hipEventSynchronize(ev_upload_[b]));
    if (probs_dirty_) {
        build_lists();
        std::memcpy(h_probs_stage_[b], hp_.data(), sizeof(BProb) * cap_);
        std::memcpy(h_wl_stage_[b], h_wl_.data(), sizeof(int) * h_wl_.size());
        MG_HIP(hipMemcpyAsync(d_probs_, h_probs_stage_[b], sizeof(BProb) * cap_,
                              hipMemcpyHostToDevice, st_));
        MG_HIP(hipMemcpyAsync(d_wl_, h_wl_stage_[b], sizeof(int) * h_wl_.size(),
                              hipMemcpyHostToDevice, st_));
        probs_dirty_ = false;
    }
    // initial states of the started slots, one copy per run of consecutive
    // started slots (the others' states are live on the device)
    bool any_started = false;
    for (int s = 0; s < cap_;) {
        if (!started_[s]) {
            ++s;
            continue;
        }
        int e = s;
        for (; e < cap_ && started_[e]; ++e) {
            BState& S = h_start_stage_[b][e];
            std::memset(&S, 0, sizeof(BState));
            S.flags = BF_INIT;
            started_[e] = 0;
        }
        MG_HIP(hipMemcpyAsync(d_state_ + s, &h_start_stage_[b][s], sizeof(BState) * (e - s),
                              hipMemcpyHostToDevice, st_));
        any_started = true;
        s = e;
    }
    if (any_started) {
        // the union of flags now includes BF_INIT: mark every flag present
        BState& A = h_start_stage_[b][cap_];
        std::memset(&A, 0, sizeof(BState));
        A.flags = -1;
        MG_HIP(hipMemcpyAsync(d_state_ + cap_, &A, sizeof(BState), hipMemcpyHostToDevice, st_));
        init_pending_ = true;
    }
    MG_HIP(hipEventRecord(ev_upload_[b], st_));
    return MG_OK;
}

mg_status BatchEngine::upload() {
    if (mg_status s = upload_async()) return s;
    MG_HIP(hipStreamSynchronize(st_));
    return MG_OK;
}

mg_status BatchEngine::launch_iteration() {
    MG_HIP(hipSetDevice(device_));
    if (mg_status s = ensure_graph()) return s;
    return launch();
}

mg_status BatchEngine::wait_iteration(int64_t k, int* live, int* sure, const int** flags) {
    if (mg_status s = wait(k, live, sure)) return s;
    if (flags) *flags = h_ring_ + (k % ITER_RING) * (2 + cap_) + 2;
    return MG_OK;
}

// Device-to-host copy on the read stream, unordered with the iterations:
// only for data no queued iteration writes (the state and iterate of a
// finished problem).
mg_status BatchEngine::fetch(const void* dev, void* host, size_t bytes) {
    MG_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, read_st_));
    MG_HIP(hipStreamSynchronize(read_st_));
    return MG_OK;
}

mg_status BatchEngine::fetch_state(int s, BState* out) {
    if (mg_status e = fetch(d_state_ + s, h_fetch_, sizeof(BState))) return e;
    *out = *h_fetch_;
    return MG_OK;
}

// One fused pass (pre or post) at level l over the problems whose flags meet
// mask, as in an iteration.
hipError_t BatchEngine::launch_fused(int l, bool pre, int mask) {
    const int stride = 3 + 2 * cap_;
    const int* wl = d_wl_ + (size_t)wl_fused(l) * stride;
    const int bt = bt_[l];
    if (blk_[l]) {
        const dim3 GB(STAGE_GRID), BB(dev::BLK_THREADS);
#define BLK(BR)                                                                                 \
    if (pre)                                                                                    \
        hipLaunchKernelGGL((kb_fpre_blk<BR, dev::BLK_COLS>), GB, BB, 0, st_, d_probs_, d_state_, \
                           wl, l, mask);                                                        \
    else                                                                                        \
        hipLaunchKernelGGL((kb_fpost_blk<BR, dev::BLK_COLS>), GB, BB, 0, st_, d_probs_,          \
                           d_state_, wl, l, mask);
        switch (blk_[l]) {
            case 1: BLK(8) break;
            case 2: BLK(16) break;
            default: BLK(32) break;
        }
#undef BLK
        return hipGetLastError();
    }
    const dim3 GF(STAGE_GRID * (dev::F_MAX_THREADS / bt)), BF(bt);
#define ONE(BT)                                                                              \
    if (pre)                                                                                 \
        hipLaunchKernelGGL(kb_fpre<BT>, GF, BF, 0, st_, d_probs_, d_state_, wl, l, mask);   \
    else                                                                                     \
        hipLaunchKernelGGL(kb_fpost<BT>, GF, BF, 0, st_, d_probs_, d_state_, wl, l, mask);
    switch (bt) {
        case 64: ONE(64) break;
        case 128: ONE(128) break;
        case 192: ONE(192) break;
        default: ONE(256) break;
    }
#undef ONE
    return hipGetLastError();
}

mg_status BatchEngine::tune(int reps, std::vector<mg_tile_choice>* out) {
    static const int kRows[] = {4, 8, 12, 16, 24, 32, 48, 64, 96};
    static const int kWidths[] = {64, 128, 192, 256};
    MG_HIP(hipSetDevice(device_));
    if (mg_status s = upload()) return s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MG_HIP(hipEventCreate(&e0));
    MG_HIP(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    if (!(nu_pre_ == 2 && nu_post_ == 2)) return MG_OK;  // only the fused cycle has tiles
    for (int l = Lc_ + 1; l <= Lmax_; ++l) {
        const int count = problems_at(l);
        if (count == 0) continue;
        int best = 0, best_bt = 0, best_cols = 0;
        float best_ms = 0.0f;
        // marching tiles (width x rows), then block tiles on levels of at
        // most BLK_MAX_N nodes per side
        std::vector<std::array<int, 3>> cand;
        for (int bt : kWidths)
            for (int rh : kRows) cand.push_back({bt, rh, 0});
        if ((1 << l) + 1 <= dev::BLK_MAX_N)
            for (int s = 1; s <= dev::BLK_SHAPES; ++s)
                cand.push_back({dev::BLK_THREADS, dev::block_rows(s), dev::BLK_COLS});
        for (const auto& c : cand) {
            {
                const int bt = c[0], rh = c[1];
                rh_override_[l] = rh;
                bt_override_[l] = bt;
                cols_override_[l] = c[2];
                probs_dirty_ = true;
                if (mg_status s = upload()) {
                    rh_override_[l] = bt_override_[l] = cols_override_[l] = 0;
                    return s;
                }
                for (int w = 0; w < 2; ++w) {  // warm-up
                    MG_HIP(launch_fused(l, true, BF_INIT));
                    MG_HIP(launch_fused(l, false, BF_INIT));
                }
                MG_HIP(hipEventRecord(e0, st_));
                for (int r = 0; r < reps; ++r) {
                    MG_HIP(launch_fused(l, true, BF_INIT));
                    MG_HIP(launch_fused(l, false, BF_INIT));
                }
                MG_HIP(hipEventRecord(e1, st_));
                MG_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                MG_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (!best || ms < best_ms) {
                    best = rh;
                    best_bt = bt;
                    best_cols = c[2];
                    best_ms = ms;
                }
            }
        }
        rh_override_[l] = bt_override_[l] = cols_override_[l] = 0;
        tile_table_set(l, count, best, best_bt, best_cols);
        if (out) out->push_back({l, count, best, best_bt / 64, best_cols, 1e3 * best_ms / reps});
    }
    probs_dirty_ = true;
    return upload();
}

hipError_t BatchEngine::enqueue_iteration(bool with_init) {
    const int stride = 3 + 2 * cap_;
    auto W = [&](int id) { return (const int*)(d_wl_ + (size_t)id * stride); };
    const dim3 G(STAGE_GRID), B(BLOCK);
    const dim3 GA(std::min(cap_, 1024));
    BProb* P = d_probs_;
    BState* S = d_state_;
    // the ticket of kb_finctl: the word after the iteration counter
    unsigned* ticket = reinterpret_cast<unsigned*>(d_iter_ + 1);
#define LAUNCH(...)                                        \
    do {                                                   \
        hipLaunchKernelGGL(__VA_ARGS__);                   \
        hipError_t e_ = hipGetLastError();                 \
        if (e_ != hipSuccess) return e_;                   \
    } while (0)
    // new problems: ||b||
    if (with_init) {
        LAUNCH(kb_sumsq, G, B, 0, st_, P, S, W(WL_FINEST), 0, (int)BF_INIT);
        LAUNCH(kb_finctl, GA, B, 0, st_, P, S, W(WL_ALL), (int)K_NORM, (int)F_BN, (int)BF_INIT,
               -1, (int)PH_INIT, d_iter_, h_ring_, ticket);
    }
    // finished inner loops: x += s c; then, for them and the new problems,
    // the FP64 defect, its norm and the stop test
    const int om = BF_OUTER | BF_UPDATE;
    LAUNCH(kb_update, G, B, 0, st_, P, S, W(WL_FINEST), (int)BF_UPDATE);
    LAUNCH(kb_outer_defect, G, B, 0, st_, P, S, W(WL_FINEST), om);
    LAUNCH(kb_finctl, GA, B, 0, st_, P, S, W(WL_ALL), (int)K_S64, (int)F_S, om, -1,
           (int)PH_OUTER, d_iter_, h_ring_, ticket);
    // one FP32 V-cycle for every problem in its inner loop
    const int m = BF_INNER;
    const bool fused = nu_pre_ == 2 && nu_post_ == 2;
    if (fused) {
#define FUSED(pre, l)                                   \
    {                                                   \
        const hipError_t e_ = launch_fused(l, pre, m);  \
        if (e_ != hipSuccess) return e_;                \
    }
        for (int l = Lmax_; l > Lc_; --l)
            if (launch_mask_ & (1u << l)) FUSED(true, l)
        LAUNCH(kb_tail, GA, dim3(dev::TAIL_THREADS), 0, st_, P, S, W(WL_ALL), Lc_, m);
        LAUNCH(kb_coarse, GA, B, 0, st_, P, S, W(WL_ALL), Lc_, m, Lc_);
        for (int l = Lc_ + 1; l <= Lmax_; ++l)
            if (launch_mask_ & (1u << l)) FUSED(false, l)
#undef FUSED
        // problems without a level above the coarse one: residual from a defect pass
        if (launch_mask_ & 1u)
            LAUNCH(kb_inner_norm, G, B, 0, st_, P, S, W(WL_FINEST_COARSE), m, Lc_);
        if (launch_mask_ & (1u << 31))
            LAUNCH(kb_segsum, G, B, 0, st_, P, S, W(WL_SEGS32), m, Lc_);
        LAUNCH(kb_finctl, GA, B, 0, st_, P, S, W(WL_ALL), (int)K_S32, (int)F_R32, m, Lc_,
               (int)PH_INNER, d_iter_, h_ring_, ticket);
        return hipSuccess;
    }
    // roles of the unfused cycle: 0 = x, 1 = t
    int cur = 0, oth = 1;
    for (int l = Lmax_; l > Lc_; --l) {
        cur = 0;
        oth = 1;
        if (nu_pre_ == 0) LAUNCH(kb_fill_cond, G, B, 0, st_, P, S, W(wl_level(l)), l, cur, m);
        for (int k = 0; k < nu_pre_; ++k) {
            if (k == 0)
                LAUNCH(kb_pre1, G, B, 0, st_, P, S, W(wl_level(l)), l, cur, oth, m);
            else
                LAUNCH(kb_band<dev::OP_JACOBI>, G, B, 0, st_, P, S, W(wl_level(l)), l, cur, oth, m);
            std::swap(cur, oth);
        }
        LAUNCH(kb_band<dev::OP_DEFECT>, G, B, 0, st_, P, S, W(wl_level(l)), l, cur, oth, m);
        LAUNCH(kb_restrict, G, B, 0, st_, P, S, W(wl_restrict(l)), l, oth, m);
    }
    LAUNCH(kb_coarse, GA, B, 0, st_, P, S, W(WL_ALL), Lc_, m, -1);
    const int after_pre = nu_pre_ % 2;  // role holding the iterate after pre-smoothing
    for (int l = Lc_ + 1; l <= Lmax_; ++l) {
        cur = after_pre;
        oth = 1 - cur;
        LAUNCH(kb_prolong, G, B, 0, st_, P, S, W(wl_level(l)), l, cur, m);
        for (int k = 0; k < nu_post_; ++k) {
            LAUNCH(kb_band<dev::OP_JACOBI>, G, B, 0, st_, P, S, W(wl_level(l)), l, cur, oth, m);
            std::swap(cur, oth);
        }
        if (cur != 0) LAUNCH(kb_copy, G, B, 0, st_, P, S, W(wl_level(l)), l, cur, 0, m);
    }
    // inner residual and stop test
    LAUNCH(kb_inner_norm, G, B, 0, st_, P, S, W(WL_FINEST), m, -1);
    if (launch_mask_ & (1u << 31))
        LAUNCH(kb_segsum, G, B, 0, st_, P, S, W(WL_SEGS32), m, -1);
    LAUNCH(kb_finctl, GA, B, 0, st_, P, S, W(WL_ALL), (int)K_S32, (int)F_R32, m, -1,
           (int)PH_INNER, d_iter_, h_ring_, ticket);
#undef LAUNCH
    return hipSuccess;
}

mg_status BatchEngine::ensure_graph() {
    for (int w = 0; w < 2; ++w) {
        if (graph_[w]) continue;
        hipGraph_t g = nullptr;
        MG_HIP(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_iteration(w == 1);
        hipError_t e2 = hipStreamEndCapture(st_, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&graph_[w], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            graph_[w] = nullptr;
            return fail(MG_ERR_DEVICE, std::string("batch graph capture: ") + hipGetErrorString(e));
        }
    }
    for (int l = 0; l <= MG_MAX_LEVEL; ++l) {
        graph_bt_[l] = bt_[l];
        graph_blk_[l] = blk_[l];
    }
    return MG_OK;
}

// One iteration; the first after an upload that started problems also runs
// the start phase.
mg_status BatchEngine::launch() {
    MG_HIP(hipGraphLaunch(graph_[init_pending_ ? 1 : 0], st_));
    init_pending_ = false;
    MG_HIP(hipEventRecord(ev_[launched_ % ITER_RING], st_));
    ++launched_;
    return MG_OK;
}

// Wait for iteration k; its counts of live and of certainly-continuing problems.
mg_status BatchEngine::wait(int64_t k, int* live, int* sure) {
    MG_HIP(hipEventSynchronize(ev_[k % ITER_RING]));
    const volatile int* r = h_ring_ + (k % ITER_RING) * (2 + cap_);
    *live = r[0];
    *sure = r[1];
    return MG_OK;
}

mg_status BatchEngine::step(int* active_left) {
    MG_HIP(hipSetDevice(device_));
    if (mg_status s = ensure_graph()) return s;
    const int64_t k = launched_;
    if (mg_status s = launch()) return s;
    int live = 0, sure = 0;
    if (mg_status s = wait(k, &live, &sure)) return s;
    if (active_left) *active_left = live;
    return MG_OK;
}

// Iterations until no problem is live (at most iter_cap).  While the last
// finished iteration shows a problem still in its inner loop, the next but
// one iteration is certainly needed and is queued before the host waits, so
// the device does not idle between iterations; at outer steps the host
// waits for the decision.  No iteration is queued that is not needed.
mg_status BatchEngine::run(int64_t iter_cap, int64_t* iterations) {
    const TraceRange trace("batch iterations");
    MG_HIP(hipSetDevice(device_));
    if (mg_status s = ensure_graph()) return s;
    const int64_t first = launched_;
    int64_t next = first;  // next iteration to wait for
    if (iter_cap > 0)
        if (mg_status s = launch()) return s;
    while (next < launched_) {
        int live = 0, sure = 0;
        if (mg_status s = wait(next, &live, &sure)) return s;
        ++next;
        if (live == 0) break;
        const bool room = launched_ - first < iter_cap;
        if (room && launched_ == next)
            if (mg_status s = launch()) return s;  // nothing queued: go on
        if (room && launched_ == next + 1 && sure > 0)
            if (mg_status s = launch()) return s;  // needed after the queued one
    }
    if (iterations) *iterations = next - first;
    return MG_OK;
}

mg_status BatchEngine::zero_unwritten() {
    MG_HIP(hipSetDevice(device_));
    const int stride = 3 + 2 * cap_;
    hipLaunchKernelGGL(kb_zero_unwritten, dim3(STAGE_GRID), dim3(BLOCK), 0, st_, d_probs_,
                       d_state_, (const int*)(d_wl_ + (size_t)WL_FINEST * stride));
    MG_HIP(hipGetLastError());
    return MG_OK;
}

mg_status BatchEngine::read_states() {
    MG_HIP(hipSetDevice(device_));
    MG_HIP(hipMemcpyAsync(h_state_, d_state_, sizeof(BState) * cap_, hipMemcpyDeviceToHost, st_));
    MG_HIP(hipStreamSynchronize(st_));
    return MG_OK;
}

}  // namespace mg

// ---------------------------------------------------------------- C ABI

namespace mg {

// Algorithmic bytes of one FP32 V-cycle of a level-L problem (same byte
// model as the single-problem driver; the finest first sweep counted full).
double vcycle_bytes32(int L, int Lc, int nu_pre, int nu_post) {
    auto n = [](int l) { return (double)(((int64_t(1) << l) + 1) * ((int64_t(1) << l) + 1)); };
    double b = 8.0 * n(Lc);
    if (nu_pre == 2 && nu_post == 2) {
        for (int l = Lc + 1; l <= L; ++l)
            b += (l < L ? 11.0 : 12.0) * 4.0 * n(l) + 12.0 * 4.0 * n(l) + 8.0 * n(l - 1);
        return b;
    }
    for (int l = Lc + 1; l <= L; ++l) {
        const double sweeps = (double)(nu_pre + nu_post) * 48.0 * n(l);
        const double zero_saving = (l < L && nu_pre > 0) ? 36.0 * n(l) : 0.0;
        b += sweeps - zero_saving + 48.0 * n(l) + 4.0 * (n(l) + n(l - 1)) +
             4.0 * (n(l - 1) + 2.0 * n(l));
    }
    return b;
}

double mixed_solve_bytes(int L, int Lc, int nu_pre, int nu_post, const BState& S) {
    const double n = (double)(((int64_t(1) << L) + 1) * ((int64_t(1) << L) + 1));
    const int outer_defects = S.outer + 1;
    const double norm_pass = (nu_pre == 2 && nu_post == 2 && L > Lc) ? 0.0 : 44.0 * n;
    return 8.0 * n + outer_defects * 96.0 * n + S.outer * (12.0 + 4.0 + 20.0) * n +
           S.cycles * (vcycle_bytes32(L, Lc, nu_pre, nu_post) + norm_pass);
}

void fill_stats(const BState& S, int L, int Lc, int nu_pre, int nu_post, mg_stats* st) {
    mg_stats o{};
    o.status = (mg_status)S.status;
    o.cycles = S.cycles;
    o.outer_steps = S.outer;
    o.bnorm = S.bn;
    o.rel_res = S.bn > 0.0 ? S.s / S.bn : 0.0;
    o.n_hist = S.n_hist;
    for (int k = 0; k < S.n_hist && k < MG_HIST; ++k) o.res_hist[k] = S.hist[k];
    o.alg_bytes = mixed_solve_bytes(L, Lc, nu_pre, nu_post, S);
    *st = o;
}

}  // namespace mg

using namespace mg;

namespace {

// Idle batch engines kept between mg_solve_batch calls, so that repeated
// batches reuse the device descriptors, work-list buffers and the captured
// iteration graph.  An engine serves one call at a time; it is taken out of
// the pool for the call.  The pool lives until the process ends (device
// memory of a few MB per engine; never destroyed during static teardown).
struct EnginePool {
    struct Entry {
        int device, Lmax, Lc, nu_pre, nu_post;
        BatchEngine* eng;
    };
    std::mutex mu;
    std::vector<Entry> idle;  // oldest first
    static constexpr size_t MAX_IDLE = 4;

    BatchEngine* take(int device, int count, int Lmax, int Lc, int nu_pre, int nu_post) {
        std::lock_guard<std::mutex> g(mu);
        int best = -1;
        for (int i = 0; i < (int)idle.size(); ++i) {
            const Entry& e = idle[i];
            if (e.device == device && e.Lmax == Lmax && e.Lc == Lc && e.nu_pre == nu_pre &&
                e.nu_post == nu_post && e.eng->capacity() >= count &&
                (best < 0 || e.eng->capacity() < idle[best].eng->capacity()))
                best = i;
        }
        if (best < 0) return nullptr;
        BatchEngine* eng = idle[best].eng;
        idle.erase(idle.begin() + best);
        return eng;
    }
    void give(int device, int Lmax, int Lc, int nu_pre, int nu_post, BatchEngine* eng) {
        std::lock_guard<std::mutex> g(mu);
        idle.push_back({device, Lmax, Lc, nu_pre, nu_post, eng});
        if (idle.size() > MAX_IDLE) {
            delete idle.front().eng;
            idle.erase(idle.begin());
        }
    }
};

EnginePool& engine_pool() {
    static EnginePool* pool = new EnginePool();
    return *pool;
}

}  // namespace

extern "C" mg_status mg_solve_batch(mg_hierarchy* const* hs, const double* const* b,
                                    double* const* x, int count, const mg_solve_opts* opts,
                                    void* stream, mg_stats* stats) {
    const TraceRange trace("mg_solve_batch");
    if (!hs || !b || !x || count < 1) return fail(MG_ERR_INVALID, "empty or null batch");
    mg_solve_opts def;
    mg_default_opts(&def);
    def.precision = MG_PREC_MIXED;
    const mg_solve_opts& o0 = opts ? opts[0] : def;
    int Lmax = 0;
    for (int p = 0; p < count; ++p) {
        const mg_hierarchy* h = hs[p];
        const mg_solve_opts& o = opts ? opts[p] : def;
        if (!h || !h->assembled) return fail(MG_ERR_INVALID, "null or unassembled hierarchy");
        if (h->ctx->device != hs[0]->ctx->device || h->Lc != hs[0]->Lc)
            return fail(MG_ERR_INVALID, "batch problems must share device and coarse level");
        for (int q = 0; q < p; ++q)
            if (hs[q] == h) return fail(MG_ERR_INVALID, "a hierarchy appears twice in the batch");
        if (!b[p] || !x[p] || b[p] == x[p] || ((uintptr_t)b[p] & 15) || ((uintptr_t)x[p] & 15))
            return fail(MG_ERR_INVALID, "b, x must be distinct 16-byte aligned device pointers");
        if (o.precision != MG_PREC_MIXED)
            return fail(MG_ERR_INVALID, "the batched solver runs the mixed-precision scheme");
        if (o.krylov)
            return fail(MG_ERR_INVALID, "the batched solver runs multigrid defect correction");
        if (o.nu_pre != o0.nu_pre || o.nu_post != o0.nu_post)
            return fail(MG_ERR_INVALID, "smoothing counts must agree across the batch");
        if (o.nu_pre < 0 || o.nu_post < 0 || o.nu_pre + o.nu_post == 0 || o.nu_pre > 16 ||
            o.nu_post > 16 || !(o.omega > 0.0 && o.omega < 2.0) || !(o.rel_tol >= 0.0) ||
            o.max_cycles < 1 || o.inner_max_cycles < 1 ||
            !(o.inner_reduction >= 0.0 && o.inner_reduction < 1.0) || o.fixed_cycles < 0 ||
            (o.zero_guess != 0 && o.zero_guess != 1))
            return fail(MG_ERR_INVALID, "invalid solver options");
        Lmax = std::max(Lmax, h->L);
    }
    {
        // the problems work in place on the callers' vectors: no x may be
        // another problem's x or any problem's b
        std::unordered_set<const void*> xs;
        for (int p = 0; p < count; ++p)
            if (!xs.insert(x[p]).second)
                return fail(MG_ERR_INVALID, "two problems of the batch share an x vector");
        for (int p = 0; p < count; ++p)
            if (xs.count(b[p]))
                return fail(MG_ERR_INVALID, "a problem's b is another problem's x");
    }
    const int device = hs[0]->ctx->device, Lc = hs[0]->Lc;
    MG_HIP(hipSetDevice(device));
    MG_HIP(hipStreamSynchronize((hipStream_t)stream));
    EnginePool& pool = engine_pool();
    BatchEngine* taken = pool.take(device, count, Lmax, Lc, o0.nu_pre, o0.nu_post);
    if (!taken) {
        taken = new (std::nothrow) BatchEngine();
        if (!taken) return fail(MG_ERR_NOMEM, "host allocation failed");
        if (mg_status s = taken->init(device, count, Lmax, Lc, o0.nu_pre, o0.nu_post)) {
            delete taken;
            return s;
        }
    }
    // back to the pool on every exit path, unless the device failed under it
    struct Return {
        EnginePool& pool;
        BatchEngine* eng;
        int device, Lmax, Lc, nu_pre, nu_post;
        bool ok = false;
        ~Return() {
            if (ok)
                pool.give(device, Lmax, Lc, nu_pre, nu_post, eng);
            else
                delete eng;
        }
    } ret{pool, taken, device, Lmax, Lc, o0.nu_pre, o0.nu_post};
    BatchEngine& eng = *taken;
    for (int s = count; s < eng.capacity(); ++s) eng.clear_slot(s);
    int64_t iter_cap = 8;
    for (int p = 0; p < count; ++p) {
        mg_hierarchy* h = hs[p];
        const mg_solve_opts& o = opts ? opts[p] : def;
        eng.set_slot(p, h, o, b[p], x[p]);
        eng.start_slot(p);
        const int outer = o.fixed_cycles > 0 ? o.fixed_cycles : o.max_cycles;
        iter_cap = std::max<int64_t>(iter_cap, (int64_t)(outer + 1) * (o.inner_max_cycles + 1) + 4);
    }
    if (mg_status s = eng.upload()) return s;
    if (mg_status s = eng.run(iter_cap, nullptr)) return s;
    if (mg_status s = eng.zero_unwritten()) return s;
    if (mg_status s = eng.read_states()) return s;
    mg_status worst = MG_OK;
    for (int p = 0; p < count; ++p) {
        mg_hierarchy* h = hs[p];
        const BState& S = eng.state(p);
        if (stats) fill_stats(S, h->L, h->Lc, o0.nu_pre, o0.nu_post, &stats[p]);
        if (!(S.flags & BF_DONE)) {
            if (stats) stats[p].status = MG_ERR_NOCONV;
            worst = MG_ERR_NOCONV;
        } else if (S.status != MG_OK && worst == MG_OK) {
            worst = (mg_status)S.status;
        }
    }
    MG_HIP(hipStreamSynchronize(eng.stream()));
    ret.ok = true;
    if (worst != MG_OK) return fail(worst, "at least one problem of the batch did not converge");
    return MG_OK;
}

extern "C" mg_status mg_batch_autotune(mg_hierarchy* const* hs, int count,
                                       const mg_solve_opts* opts, int reps, mg_tile_choice* out,
                                       int out_cap, int* n_out) {
    if (n_out) *n_out = 0;
    if (!hs || count < 1) return fail(MG_ERR_INVALID, "empty or null batch");
    if (reps < 1 || reps > 1000) return fail(MG_ERR_INVALID, "reps must lie in [1, 1000]");
    if (out_cap < 0 || (out_cap > 0 && !out)) return fail(MG_ERR_INVALID, "bad output array");
    mg_solve_opts o;
    mg_default_opts(&o);
    o.precision = MG_PREC_MIXED;
    if (opts) o = *opts;
    int Lmax = 0;
    for (int p = 0; p < count; ++p) {
        const mg_hierarchy* h = hs[p];
        if (!h || !h->assembled) return fail(MG_ERR_INVALID, "null or unassembled hierarchy");
        if (h->ctx->device != hs[0]->ctx->device || h->Lc != hs[0]->Lc)
            return fail(MG_ERR_INVALID, "batch problems must share device and coarse level");
        for (int q = 0; q < p; ++q)
            if (hs[q] == h) return fail(MG_ERR_INVALID, "a hierarchy appears twice in the batch");
        Lmax = std::max(Lmax, h->L);
    }
    if (o.nu_pre < 0 || o.nu_post < 0 || o.nu_pre + o.nu_post == 0 || o.nu_pre > 16 ||
        o.nu_post > 16 || !(o.omega > 0.0 && o.omega < 2.0))
        return fail(MG_ERR_INVALID, "invalid solver options");
    const int device = hs[0]->ctx->device, Lc = hs[0]->Lc;
    MG_HIP(hipSetDevice(device));
    EnginePool& pool = engine_pool();
    BatchEngine* eng = pool.take(device, count, Lmax, Lc, o.nu_pre, o.nu_post);
    if (!eng) {
        eng = new (std::nothrow) BatchEngine();
        if (!eng) return fail(MG_ERR_NOMEM, "host allocation failed");
        if (mg_status s = eng->init(device, count, Lmax, Lc, o.nu_pre, o.nu_post)) {
            delete eng;
            return s;
        }
    }
    for (int s = count; s < eng->capacity(); ++s) eng->clear_slot(s);
    for (int p = 0; p < count; ++p) {
        eng->set_slot(p, hs[p], o);
        eng->start_slot(p);
    }
    std::vector<mg_tile_choice> rows;
    const mg_status st = eng->tune(reps, &rows);
    if (st != MG_OK) {
        delete eng;
        return st;
    }
    pool.give(device, Lmax, Lc, o.nu_pre, o.nu_post, eng);
    const int n = std::min<int>(out_cap, (int)rows.size());
    for (int i = 0; i < n; ++i) out[i] = rows[i];
    if (n_out) *n_out = (int)rows.size();
    return MG_OK;
}

extern "C" mg_status mg_batch_set_tile(int level, int problems, int tile_rows, int row_waves,
                                       int tile_cols) {
    if (level < 2 || level > MG_MAX_LEVEL) return fail(MG_ERR_INVALID, "level outside [2, 14]");
    if (problems < 1) return fail(MG_ERR_INVALID, "problems must be >= 1");
    if (tile_cols) {
        if (!dev::block_shape(tile_rows, tile_cols))
            return fail(MG_ERR_INVALID, "a block tile is 8, 16 or 32 rows by 32 columns");
        if (row_waves != 0 && row_waves != dev::BLK_THREADS / 64)
            return fail(MG_ERR_INVALID, "a block tile has 4 wavefronts (row_waves 0 or 4)");
        tile_table_set(level, problems, tile_rows, dev::BLK_THREADS, tile_cols);
        return MG_OK;
    }
    if (tile_rows < 4 || tile_rows > 256 || tile_rows % 4)
        return fail(MG_ERR_INVALID, "tile_rows must be a multiple of 4 in [4, 256]");
    if (row_waves < 0 || row_waves > dev::F_MAX_THREADS / 64)
        return fail(MG_ERR_INVALID, "row_waves must lie in [0, 4]");
    tile_table_set(level, problems, tile_rows, 64 * row_waves);
    return MG_OK;
}

extern "C" mg_status mg_batch_clear_tiles(void) {
    tile_table_clear();
    return MG_OK;
}
