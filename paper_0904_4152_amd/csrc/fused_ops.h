// Fused smoothing passes of the V(2,2) cycle.  One workgroup owns a strip
// of grid columns and a chunk of grid rows and marches down the rows; each
// row of bands, x and b is read from HBM once and kept (bands in a register
// ring of six rows, iterates in LDS rings of three rows) while every
// fused step that needs it runs:
//   pre  : two damped Jacobi sweeps (the first possibly from a zero
//          iterate), the defect of the result and its restriction P^T d to
//          the next coarser level;
//   post : prolongation and correction x + P x_c, two damped Jacobi sweeps,
//          and optionally the sum of squares of the final defect.
// Each node's arithmetic is the one of the unfused kernels (same operands,
// same operation order), so fused and unfused cycles give identical bits.
// Strips overlap by F_HALO columns and chunks by F_HALO rows; the overlap is
// recomputed and only owned nodes are written.
//
// Rows of x and of bands are loaded two to three steps ahead of their use,
// so that enough bytes are in flight per wavefront to cover HBM latency.
// Row bookkeeping of one step of the pre pass: the x row jx enters; after a
// first barrier the first sweep runs at row jx-1 and the defect at jx-4,
// after a second barrier the second sweep at jx-2 and the restriction at
// jx-5.  The post pass runs the first sweep at jx-1, the second at jx-2 and
// the norm at jx-3, a barrier before each.  With j0 the first row of the
// march, an iterate row j lives
// in LDS slot (j - j0) mod 3 and a band row in register slot (j - j0) mod 6;
// the loop is unrolled by six so every slot index is a compile-time
// constant.  The march starts at the first row that is needed and runs
// whole blocks of six steps past the last one (the extra steps compute
// nothing that is kept).
#pragma once

#include "device_ops.h"
#include "mgfem.h"

namespace mg {
namespace dev {

constexpr int F_HALO = 4;           // columns / rows recomputed per side
constexpr int F_MIN_THREADS = 64;   // workgroup widths: 64, 128, 192 or 256 threads,
constexpr int F_MAX_THREADS = 256;  // one grid column per thread

// Columns of one segment of the residual-norm partials (see post_tile);
// strips own whole segments.
constexpr int F_NORM_COLS = 8;

struct FusedGeom {
    int bt;       // threads per workgroup
    int cw;       // owned columns per strip (a multiple of F_NORM_COLS, at most bt - 2 F_HALO)
    int nstrips;  // strips of cw columns (the last one may be narrower)
    int nchunks;  // chunks of rh rows
    int rh;       // owned rows per chunk (even)
    int blk;      // 0: marching tiles; else a block tile shape (block_geom)
};

// Strips of equal width (rounded up to a multiple of F_NORM_COLS) as few as
// bt threads allow.
__host__ __device__ inline FusedGeom fused_geom(int N, int bt, int rh) {
    FusedGeom g;
    g.bt = bt;
    g.rh = rh;
    const int cmax = bt - 2 * F_HALO;  // a multiple of F_NORM_COLS
    g.nstrips = (N + cmax - 1) / cmax;
    g.cw = (N + g.nstrips - 1) / g.nstrips;
    g.cw = (g.cw + F_NORM_COLS - 1) / F_NORM_COLS * F_NORM_COLS;
    g.nchunks = (N + rh - 1) / rh;
    g.blk = 0;
    return g;
}

// Block tiles (see pre_block): shape s in 1..BLK_SHAPES owns 4 << s rows
// (8, 16 or 32) by BLK_COLS columns; 0 is no block shape.
constexpr int BLK_SHAPES = 3;
constexpr int BLK_COLS = 32;
// Largest level side the autotuners try block tiles on: above it the halo
// (at least 0.9 x the owned nodes recomputed) outweighs the shorter chain.
constexpr int BLK_MAX_N = 1025;
__host__ __device__ constexpr int block_rows(int shape) { return 4 << shape; }
__host__ __device__ inline int block_shape(int rows, int cols) {
    if (cols != BLK_COLS) return 0;
    for (int s = 1; s <= BLK_SHAPES; ++s)
        if (rows == block_rows(s)) return s;
    return 0;
}
__host__ __device__ inline FusedGeom block_geom(int N, int shape) {
    FusedGeom g;
    g.bt = 256;
    g.rh = block_rows(shape);
    g.cw = BLK_COLS;
    g.nstrips = (N + g.cw - 1) / g.cw;
    g.nchunks = (N + g.rh - 1) / g.rh;
    g.blk = shape;
    return g;
}

__device__ __forceinline__ bool in_range(int v, int lo, int hi) { return v >= lo && v < hi; }

// v in [lo, hi) for lo <= hi, with one compare.
__device__ __forceinline__ bool in_win(int v, int lo, int hi) {
    return (unsigned)(v - lo) < (unsigned)(hi - lo);
}

// The 9-term band product at one node from the rows j-1, j, j+1 of an
// iterate held in LDS, around LDS column t: the fma chain of stencil_tile.
template <typename T>
__device__ __forceinline__ T band_row_product(const T (&bk)[9], const T* __restrict__ rm,
                                              const T* __restrict__ rc,
                                              const T* __restrict__ rp, int t) {
    const T* rows[3] = {rm, rc, rp};
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) acc = fma(bk[k], rows[k / 3][t + k % 3 - 1], acc);
    return acc;
}

// Raw buffer resources: one per band array, for b and for x.  A load
// whose byte offset falls outside [0, bytes) returns zero, so rows above and
// below the grid need no checks (negative offsets wrap to huge unsigned ones).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int RSRC_WORD3 = 0x00020000;  // raw (untyped) buffer access on CDNA
constexpr int AUX_NT = 2;               // non-temporal: bands are read once

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0,
                                             (int)(uint32_t)bytes, RSRC_WORD3);
}

template <typename T, int AUX>
struct BufLoad;
template <int AUX>
struct BufLoad<float, AUX> {
    static __device__ __forceinline__ float get(rsrc_t r, uint32_t off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, AUX));
    }
};
template <int AUX>
struct BufLoad<double, AUX> {
    static __device__ __forceinline__ double get(rsrc_t r, uint32_t off) {
        return __builtin_bit_cast(double,
                                  __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, AUX));
    }
};
template <typename T, int AUX = 0>
__device__ __forceinline__ T bload(rsrc_t r, uint32_t off) {
    return BufLoad<T, AUX>::get(r, off);
}

template <typename T>
struct RowRsrc {
    rsrc_t band[9];
    rsrc_t b;
    __device__ RowRsrc(const T* bands, int64_t bs, const T* bb, int64_t n) {
#pragma unroll
        for (int k = 0; k < 9; ++k) band[k] = make_rsrc(bands + k * bs, n * (int64_t)sizeof(T));
        b = make_rsrc(bb, n * (int64_t)sizeof(T));
    }
};

// Byte offset past every buffer: a load from it returns zero.  The largest
// buffer (an FP64 vector at the finest admitted level, 16385^2 x 8 B) is
// just over 2 GiB, so the offset sits at 3 GiB, with room below 2^32 for the
// small strides added to it.
constexpr uint32_t OFF_NONE = 0xC0000000u;
static_assert((uint64_t)((1 << MG_MAX_LEVEL) + 1) * ((1 << MG_MAX_LEVEL) + 1) * sizeof(double) <
                  (uint64_t)OFF_NONE,
              "out-of-range offset inside a buffer");

// Bands and b of one node at byte offset off; zeros when !need.  The loads
// are issued on every lane (an unneeded lane reads past the buffer), so no
// branch separates a load from its later use and the compiler's wait
// counting stays exact across the loop.
template <typename T>
__device__ __forceinline__ void load_row(const RowRsrc<T>& R, uint32_t off, bool need,
                                         T (&bk)[9], T& bb) {
    const uint32_t o = need ? off : OFF_NONE;
#pragma unroll
    for (int k = 0; k < 9; ++k) bk[k] = bload<T, AUX_NT>(R.band[k], o);
    bb = bload<T>(R.b, o);
}

// The diagonal and upper bands (4..8) and b of one node; the lower bands
// are rebuilt from the neighbours' upper bands (see LowerBands).
template <typename T>
__device__ __forceinline__ void load_upper(const RowRsrc<T>& R, uint32_t off, bool need,
                                           T (&bk)[9], T& bb) {
    const uint32_t o = need ? off : OFF_NONE;
#pragma unroll
    for (int k = 4; k < 9; ++k) bk[k] = bload<T, AUX_NT>(R.band[k], o);
    bb = bload<T>(R.b, o);
}

// The assembled matrix is symmetric bit for bit (each entry and its mirror
// sum the same element terms in the same order), so the lower bands of a
// row are upper bands of its neighbours:
//   A[p][p-1]   = band 5 at p-1      (same row, left column)
//   A[p][p-N-1] = band 8 at p-N-1    (previous row, left column)
//   A[p][p-N]   = band 7 at p-N      (previous row, same column)
//   A[p][p-N+1] = band 6 at p-N+1    (previous row, right column).
// A tile reads 5 of the 9 band streams; bands 5, 6 and 8 of each row pass
// through LDS to the neighbouring columns (6 and 8 kept for two rows), band
// 7 of the previous row is still in the thread's register ring.  Columns
// and rows outside the grid read as zero, as the stored lower bands are.
template <typename T, int BT>
struct LowerBands {
    T* u5;  // band 5 of the row being completed
    T* u6;  // band 6 of two consecutive rows (slot = relative row parity)
    T* u8;  // band 8, likewise
    __device__ void init() {
        if (threadIdx.x < 2) {
            const int g = threadIdx.x ? BT + 1 : 0;
            u5[g] = u6[g] = u6[(BT + 2) + g] = u8[g] = u8[(BT + 2) + g] = T(0);
        }
    }
    // Before a barrier: publish the upper bands of row r (slot par).
    __device__ __forceinline__ void publish(const T (&bk)[9], int par, int t) {
        u5[t] = bk[5];
        u6[par * (BT + 2) + t] = bk[6];
        u8[par * (BT + 2) + t] = bk[8];
    }
    // After it: complete row r from its own and row r-1's published bands
    // (row r-1 in slot prev, its band 7 in bkp).
    __device__ __forceinline__ void complete(T (&bk)[9], const T (&bkp)[9], int prev, int t) {
        bk[0] = u8[prev * (BT + 2) + t - 1];
        bk[1] = bkp[7];
        bk[2] = u6[prev * (BT + 2) + t + 1];
        bk[3] = u5[t - 1];
    }
};

__device__ __forceinline__ uint32_t node_off(int j, int N, int col, int size) {
    return (uint32_t)(j * N + col) * (uint32_t)size;
}

// Pre-smoothing tile (strip, chunk) on a level with N nodes per side:
// x2 = J(J(x)) on owned nodes and bc = P^T (b - A x2) on the owned coarse
// nodes (0 at coarse nodes on the Dirichlet sides of dmask).  With XZERO the
// first sweep starts from a zero iterate and x is not read.  Band rows live
// in a ring of six register slots (the loop is unrolled by six): the load of
// row jx+2 goes out in step jx as soon as the defect has freed its slot, two
// and a half steps before the row is first used; x rows go out three steps
// ahead.
//
// One step (x row jx entering) runs in two barrier-separated phases: phase A
// takes the first sweep at row jx-1 (from the x rows written before the
// first barrier) and the defect at row jx-4 (from second-sweep rows of
// earlier steps); phase B takes the second sweep at row jx-2 (from the
// first-sweep row of phase A) and the restriction at row jx-5 (from the
// defect row of phase A).  Every LDS row ring has three slots: a slot is
// rewritten only in a window that no reader of its old row shares.
template <typename T, bool XZERO, int BT>
__device__ void pre_tile(const T* __restrict__ bands, int64_t bs, int N, const T* __restrict__ x,
                         const T* __restrict__ b, T omega, T* __restrict__ x2out,
                         T* __restrict__ bc, int dmask, int strip, int chunk, int rh, int cw) {
    __shared__ T X[3][BT + 2], A[3][BT + 2], B[3][BT + 2], D[3][BT + 2];
    __shared__ T U5[BT + 2], U6[2][BT + 2], U8[2][BT + 2];
    LowerBands<T, BT> lower{U5, &U6[0][0], &U8[0][0]};
    const int t = threadIdx.x + 1;  // LDS column; 0 and BT+1 are guards
    const int c0 = strip * cw, c1 = min(c0 + cw, N);
    const int r0 = chunk * rh, r1 = min(r0 + rh, N);
    const int col = c0 - F_HALO + (int)threadIdx.x;
    const bool cval = col >= 0 && col < N;
    // column / row ranges where each step is needed (rows clipped to the
    // grid: rows outside it hold zeros)
    const bool c_op1 = cval && in_range(col, c0 - 3, c1 + 3);
    const bool c_op2 = cval && in_range(col, c0 - 2, c1 + 2);
    const bool c_op3 = cval && in_range(col, c0 - 1, c1 + 1);
    const bool c_own = in_range(col, c0, c1);
    const bool c_coarse = c_own && !(col & 1);
    const int lo1 = max(r0 - 3, 0), hi1 = min(r1 + 3, N);
    const int lo2 = max(r0 - 2, 0), hi2 = min(r1 + 2, N);
    const int lo3 = max(r0 - 1, 0), hi3 = min(r1 + 1, N);
    const int Nc = (N >> 1) + 1;
    const int64_t n = (int64_t)N * N;
    const RowRsrc<T> R(bands, bs, b, n);
    const rsrc_t Rx = make_rsrc(x, n * (int64_t)sizeof(T));
    if (threadIdx.x < 2) {
        const int g = threadIdx.x ? BT + 1 : 0;
#pragma unroll
        for (int s = 0; s < 3; ++s) X[s][g] = A[s][g] = B[s][g] = D[s][g] = T(0);
    }
    lower.init();
    T bk[6][9], bb[6];  // band rows, slot (r - js) mod 6
    T pfx[3];           // x rows, slot (r - js) mod 3 (LDS rows likewise)
    // The first x row any sweep needs (r0 - F_HALO) enters LDS before the
    // loop, whose first step brings in the next; the last restriction row
    // leaves last.
    const int js = r0 - F_HALO + 1;
    const int jend = r1 + 5;
    auto xload = [&](int j) -> T {
        if (XZERO) return T(0);
        return bload<T>(Rx, cval && j < r1 + 4 ? node_off(j, N, col, sizeof(T)) : OFF_NONE);
    };
    // upper bands and b: the rows the first sweep needs and the one above
    // (its lower bands come from there), on every column of the tile (the
    // halo columns' bands complete their neighbours' rows)
    auto needb = [&](int j) { return cval && in_range(j, r0 - 4, r1 + 3); };
    if (!XZERO) X[2][t] = xload(js - 1);  // slot of row js - 1
    pfx[0] = xload(js);
    pfx[1] = xload(js + 1);
    pfx[2] = xload(js + 2);
    load_upper(R, node_off(js - 1, N, col, sizeof(T)), needb(js - 1), bk[5], bb[5]);
    load_upper(R, node_off(js, N, col, sizeof(T)), needb(js), bk[0], bb[0]);
    load_upper(R, node_off(js + 1, N, col, sizeof(T)), needb(js + 1), bk[1], bb[1]);
#pragma unroll 1
    for (int jb = js; jb < jend; jb += 6) {
#pragma unroll
        for (int ph = 0; ph < 6; ++ph) {
            const int jx = jb + ph;  // x row entering: LDS slot x3
            const int x3 = ph % 3;
            const int j1 = jx - 1, j2 = jx - 2, jd = jx - 4, jr = jx - 5;
            const int b1 = (ph + 5) % 6, b2 = (ph + 4) % 6, bd = (ph + 2) % 6;
            // LDS slots: x3 holds rows jx, jx-3, jx-6; l1 rows jx-1, jx-4;
            // l2 rows jx-2, jx-5
            const int l1 = (x3 + 2) % 3, l2 = (x3 + 1) % 3;
            // x row jx and the upper bands of row jx-1 into LDS; prefetch x
            // row jx+3 into the register just freed
            if (!XZERO) X[x3][t] = pfx[x3];
            lower.publish(bk[b1], (ph + 1) & 1, t);
            pfx[x3] = xload(jx + 3);
            __syncthreads();
            // ---- phase A
            lower.complete(bk[b1], bk[b2], ph & 1, t);
            // Every lane computes each step (lanes and rows outside a step's
            // window select zero), so the steps run without divergent
            // branches.
            // first sweep at row j1
            {
                T v;
                if (XZERO) {
                    v = jacobi_div(omega * bb[b1], bk[b1][4]);
                } else {
                    const T acc = band_row_product(bk[b1], X[l2], X[l1], X[x3], t);
                    v = X[l1][t] + jacobi_div(omega * (bb[b1] - acc), bk[b1][4]);
                }
                A[l1][t] = (c_op1 & in_win(j1, lo1, hi1)) ? v : T(0);
            }
            // defect at row jd from second-sweep rows jd-1, jd, jd+1
            {
                const T acc = band_row_product(bk[bd], B[l2], B[l1], B[x3], t);
                D[l1][t] = (c_op3 & in_win(jd, lo3, hi3)) ? bb[bd] - acc : T(0);
            }
            // the bands of row jx+2 into the slot row jd no longer needs
            load_upper(R, node_off(jx + 2, N, col, sizeof(T)), needb(jx + 2), bk[bd], bb[bd]);
            __syncthreads();
            // ---- phase B
            // second sweep at row j2 (written on owned nodes)
            {
                const T acc = band_row_product(bk[b2], A[x3], A[l2], A[l1], t);
                T v = A[l2][t] + jacobi_div(omega * (bb[b2] - acc), bk[b2][4]);
                v = (c_op2 & in_win(j2, lo2, hi2)) ? v : T(0);
                if (in_win(j2, r0, r1) && c_own) x2out[(int64_t)j2 * N + col] = v;
                B[l2][t] = v;
            }
            // restriction of defect rows jr-1, jr, jr+1 to coarse row jr/2
            if (in_win(jr, r0, r1) && !(jr & 1)) {
                const int I = col >> 1, J = jr >> 1;
                // defect columns and rows outside the grid are zero in LDS
                const T* u = D[x3];  // row jr - 1
                const T* c = D[l2];  // row jr
                const T* o = D[l1];  // row jr + 1
                const T corner = (u[t - 1] + u[t + 1]) + (o[t - 1] + o[t + 1]);
                const T edge = (u[t] + o[t]) + (c[t - 1] + c[t + 1]);
                const T s = c[t] + T(0.5) * edge + T(0.25) * corner;
                if (c_coarse) bc[(int64_t)J * Nc + I] = is_dirichlet(Nc, I, J, dmask) ? T(0) : s;
            }
        }
    }
}

// Grid rows per residual partial of a fused post pass; chunk heights are
// multiples of it, so no group of rows straddles two tiles.
constexpr int F_NORM_ROWS = 4;

// Partial sums of squares a fused post pass with NORM writes on a level of
// N nodes per side: one per (group of F_NORM_ROWS grid rows, segment of
// F_NORM_COLS grid columns), row groups outer.  The layout depends on N
// alone, not on the tiling.
__host__ __device__ inline int64_t fused_norm_parts(int N) {
    return (int64_t)((N + F_NORM_ROWS - 1) / F_NORM_ROWS) * ((N + F_NORM_COLS - 1) / F_NORM_COLS);
}

// Post-smoothing tile: x_out = J(J(x + P x_c)) on owned nodes.  With NORM
// also rowpart[G * NSEG + m] = the sum of (b - A x_out)^2 over rows 4G ..
// 4G+3 and columns 8m .. 8m+7 (NSEG segments per row), in one fixed order:
// each column's rows in increasing order, then the eight column sums as
// ((c0 + c1) + (c2 + c3)) + ((c4 + c5) + (c6 + c7)).  Neither the chunk
// heights nor the strip widths change a bit of it.  Same register ring as
// pre_tile; a barrier before each of the first sweep (row jx-1), the second
// (row jx-2) and the norm (row jx-3).
template <typename T, bool NORM, int BT>
__device__ void post_tile(const T* __restrict__ bands, int64_t bs, int N, const T* __restrict__ x,
                          const T* __restrict__ xc, const T* __restrict__ b, T omega,
                          T* __restrict__ xout, double* __restrict__ rowpart, int strip, int chunk,
                          int rh, int cw) {
    __shared__ T X[3][BT + 2], A[3][BT + 2], B[3][BT + 2];
    __shared__ T U5[BT + 2], U6[2][BT + 2], U8[2][BT + 2];
    LowerBands<T, BT> lower{U5, &U6[0][0], &U8[0][0]};
    constexpr int H = NORM ? 3 : 2;  // halo the last step needs
    const int t = threadIdx.x + 1;
    const int c0 = strip * cw, c1 = min(c0 + cw, N);
    const int r0 = chunk * rh, r1 = min(r0 + rh, N);
    const int col = c0 - F_HALO + (int)threadIdx.x;
    const bool cval = col >= 0 && col < N;
    const bool c_x = cval && in_range(col, c0 - H, c1 + H);
    const bool c_op1 = cval && in_range(col, c0 - (H - 1), c1 + (H - 1));
    const bool c_op2 = cval && in_range(col, c0 - (H - 2), c1 + (H - 2));
    const bool c_own = in_range(col, c0, c1);
    const int lo1 = max(r0 - (H - 1), 0), hi1 = min(r1 + (H - 1), N);
    const int lo2 = max(r0 - (H - 2), 0), hi2 = min(r1 + (H - 2), N);
    const int64_t n = (int64_t)N * N;
    const RowRsrc<T> R(bands, bs, b, n);
    const rsrc_t Rx = make_rsrc(x, n * (int64_t)sizeof(T));
    if (threadIdx.x < 2) {
        const int g = threadIdx.x ? BT + 1 : 0;
#pragma unroll
        for (int s = 0; s < 3; ++s) X[s][g] = A[s][g] = B[s][g] = T(0);
    }
    lower.init();
    T bk[6][9], bb[6];
    // x and the four coarse values around each x row in flight (slot r mod 3)
    T pfx[3], pc0[3], pc1[3], pc2[3], pc3[3];
    // Norm partials: at the end of a row group every lane leaves its
    // column's sum in NS; after the next barrier the lane at the first
    // column of each owned segment adds the segment's eight sums.
    __shared__ double NS[BT];
    double nacc = 0.0;  // this lane's column sum over the current row group
    int pend = -1;      // row group whose sums wait in NS (uniform), or -1
    const int nseg = (N + F_NORM_COLS - 1) / F_NORM_COLS;
    const bool lead = c_own && ((col - c0) % F_NORM_COLS) == 0;
    auto flush = [&]() {
        if (lead) {
            const double* v = NS + threadIdx.x;
            const double s8 = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
            rowpart[(int64_t)pend * nseg + col / F_NORM_COLS] = s8;
        }
    };
    // first x row needed .. last row of the last step (the norm, or the
    // second sweep)
    const int jstart = r0 - H;
    const int jend = r1 + (NORM ? 3 : 2);
    // x row j plus its coarse correction P x_c (the arithmetic of
    // prolong_elem): the x value and the four coarse values around the node
    // are loaded ahead and combined when the row enters
    const int Nc = (N >> 1) + 1;
    const rsrc_t Rc = make_rsrc(xc, (int64_t)Nc * Nc * (int64_t)sizeof(T));
    auto x_use = [&](int j) { return c_x && in_range(j, r0 - H, r1 + H) && in_range(j, 0, N); };
    auto xrow_load = [&](int j, T& xv, T& c0, T& c1, T& c2, T& c3) {
        const bool use = x_use(j);
        const uint32_t ox = use ? node_off(j, N, col, sizeof(T)) : OFF_NONE;
        const uint32_t oc =
            use ? (uint32_t)((j >> 1) * Nc + (col >> 1)) * (uint32_t)sizeof(T) : OFF_NONE;
        xv = bload<T>(Rx, ox);
        c0 = bload<T>(Rc, oc);
        c1 = bload<T>(Rc, oc + (uint32_t)sizeof(T));
        c2 = bload<T>(Rc, oc + (uint32_t)(Nc * sizeof(T)));
        c3 = bload<T>(Rc, oc + (uint32_t)((Nc + 1) * sizeof(T)));
    };
    const bool c_even = !(col & 1);
    auto xrow_value = [&](int j, T xv, T c0, T c1, T c2, T c3) -> T {
        // every case is evaluated and one selected (no divergent branch)
        const T v_row = c_even ? c0 : T(0.5) * (c0 + c1);  // even grid row
        const T v_odd = c_even ? T(0.5) * (c0 + c2) : T(0.25) * ((c0 + c1) + (c2 + c3));
        const T v = (j & 1) ? v_odd : v_row;
        return x_use(j) ? xv + v : T(0);
    };
    // upper bands and b: the first sweep's rows and the one above, on every
    // column of the tile (see pre_tile)
    auto needb = [&](int j) { return cval && in_range(j, r0 - H, r1 + (H - 1)); };
    // Without NORM no step reads row jx-3 and the register ring has room to
    // load bands and x one row further ahead (three rows in flight).
    constexpr int AHEAD = NORM ? 2 : 3;
    xrow_load(jstart, pfx[0], pc0[0], pc1[0], pc2[0], pc3[0]);
    xrow_load(jstart + 1, pfx[1], pc0[1], pc1[1], pc2[1], pc3[1]);
    if (AHEAD == 3) xrow_load(jstart + 2, pfx[2], pc0[2], pc1[2], pc2[2], pc3[2]);
    load_upper(R, node_off(jstart - 1, N, col, sizeof(T)), needb(jstart - 1), bk[5], bb[5]);
    load_upper(R, node_off(jstart, N, col, sizeof(T)), needb(jstart), bk[0], bb[0]);
    if (AHEAD == 3)
        load_upper(R, node_off(jstart + 1, N, col, sizeof(T)), needb(jstart + 1), bk[1], bb[1]);
#pragma unroll 1
    for (int jb = jstart; jb < jend; jb += 6) {
#pragma unroll
        for (int ph = 0; ph < 6; ++ph) {
            const int jx = jb + ph;
            const int x3 = ph % 3;
            const int j1 = jx - 1, j2 = jx - 2, j3 = jx - 3;
            const int b1 = (ph + 5) % 6, b2 = (ph + 4) % 6, b3 = (ph + 3) % 6;
            const int l1 = (x3 + 2) % 3, l2 = (x3 + 1) % 3;
            X[x3][t] = xrow_value(jx, pfx[x3], pc0[x3], pc1[x3], pc2[x3], pc3[x3]);
            lower.publish(bk[b1], (ph + 1) & 1, t);
            {
                // x row jx+AHEAD into its slot (the one just written to LDS
                // when three rows are in flight)
                const int xs = (x3 + AHEAD) % 3;
                xrow_load(jx + AHEAD, pfx[xs], pc0[xs], pc1[xs], pc2[xs], pc3[xs]);
            }
            load_upper(R, node_off(jx + AHEAD - 1, N, col, sizeof(T)), needb(jx + AHEAD - 1),
                       bk[(ph + AHEAD - 1) % 6], bb[(ph + AHEAD - 1) % 6]);
            __syncthreads();
            if (NORM && pend >= 0) {
                flush();
                pend = -1;
            }
            lower.complete(bk[b1], bk[b2], ph & 1, t);
            // every lane computes each sweep (lanes and rows outside the
            // sweep's window select zero): no divergent branches
            {
                const T acc = band_row_product(bk[b1], X[l2], X[l1], X[x3], t);
                const T v = X[l1][t] + jacobi_div(omega * (bb[b1] - acc), bk[b1][4]);
                A[l1][t] = (c_op1 & in_win(j1, lo1, hi1)) ? v : T(0);
            }
            __syncthreads();
            {
                const T acc = band_row_product(bk[b2], A[x3], A[l2], A[l1], t);
                T v = A[l2][t] + jacobi_div(omega * (bb[b2] - acc), bk[b2][4]);
                v = (c_op2 & in_win(j2, lo2, hi2)) ? v : T(0);
                if (in_win(j2, r0, r1) && c_own) xout[(int64_t)j2 * N + col] = v;
                if (NORM) B[l2][t] = v;
            }
            if (NORM) __syncthreads();
            if (NORM && in_win(j3, r0, r1)) {
                {
                    const T acc = band_row_product(bk[b3], B[l1], B[x3], B[l2], t);
                    const T d = bb[b3] - acc;
                    nacc += c_own ? (double)d * (double)d : 0.0;
                }
                if ((j3 % F_NORM_ROWS) == F_NORM_ROWS - 1 || j3 == r1 - 1) {
                    NS[threadIdx.x] = nacc;
                    nacc = 0.0;
                    pend = j3 / F_NORM_ROWS;
                }
            }
        }
    }
    if (NORM && pend >= 0) {
        __syncthreads();
        flush();
    }
}

// ---------------------------------------------------------------- block tiles
// On small levels a marching tile is bound by the latency of its chain of
// row steps (each step waits on loads issued a few steps earlier), not by
// bytes.  A block tile of BR x BC owned nodes instead loads its whole region
// (the owned nodes and F_HALO rows and columns on every side) into LDS at
// once and runs each fused step over the region, a workgroup barrier
// between steps: one memory latency per pass plus a few steps at LDS
// latency.  The steps, their windows, the per-node arithmetic and the
// layout and summation order of the norm partials are those of pre_tile
// and post_tile, so both kinds of tile give the same bits.
constexpr int BLK_THREADS = 256;

template <int BR, int BC>
struct BlockRegion {
    static constexpr int W = BC + 2 * F_HALO;  // LDS row length
    static constexpr int H = BR + 2 * F_HALO;
    static constexpr int E = W * H;
};

// LDS image of a block region: five band streams, b and two work arrays
// (each holds two iterates whose lives do not overlap); nodes outside the
// grid hold zeros.  The post pass also keeps the coarse values around the
// region (coarse rows r0/2 - 2 .. r0/2 + BR/2 + 2, likewise columns) and,
// with the norm, each column's sum over a group of rows.  A kernel declares
// one image and passes it to whichever pass it runs.
template <typename T, int BR, int BC>
struct BlockLds {
    static constexpr int E = BlockRegion<BR, BC>::E;
    static constexpr int CR = BR / 2 + 5, CC = BC / 2 + 5;
    T dg[E], u5[E], u6[E], u7[E], u8[E], b[E], p[E], q[E];
    T sc[CR * CC];
    double ns[(BR / F_NORM_ROWS) * BC];
};

// Band product at LDS node e from an LDS iterate: the fma chain of
// band_row_product, the lower bands taken from the neighbours' upper ones.
template <typename T, int BR, int BC>
__device__ __forceinline__ T block_product(const BlockLds<T, BR, BC>& s, const T* __restrict__ x,
                                           int e) {
    constexpr int W = BlockRegion<BR, BC>::W;
    const T bk[9] = {s.u8[e - W - 1], s.u7[e - W], s.u6[e - W + 1], s.u5[e - 1], s.dg[e],
                     s.u5[e],         s.u6[e],     s.u7[e],         s.u8[e]};
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) acc = fma(bk[k], x[e + (k / 3 - 1) * W + (k % 3 - 1)], acc);
    return acc;
}

// The thread's index, opaque to the compiler: everything derived from it is
// computed where it is used.  (Inside the batched engine's loop over tiles
// the compiler would otherwise hoist every per-thread index of every step
// out of the loop and hold them all in registers.)
__device__ __forceinline__ int block_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Runs f(e, j, col) for every node of the owned block widened by h on each
// side (rows r0-h .. r0+BR+h-1, columns c0-h .. c0+BC+h-1, grid or not),
// spread over the workgroup's threads (tid: this thread).
template <int BR, int BC, int h, typename F>
__device__ __forceinline__ void block_window(int tid, int r0, int c0, F&& f) {
    constexpr int W = BlockRegion<BR, BC>::W;
    constexpr int ww = BC + 2 * h, cnt = (BR + 2 * h) * ww;
#pragma unroll
    for (int u = 0; u < (cnt + BLK_THREADS - 1) / BLK_THREADS; ++u) {
        const int i = tid + u * BLK_THREADS;
        if (cnt % BLK_THREADS == 0 || i < cnt) {
            const int lr = F_HALO - h + i / ww, lc = F_HALO - h + i % ww;
            f(lr * W + lc, r0 - F_HALO + lr, c0 - F_HALO + lc);
        }
    }
}

// The region's bands, b and (unless XZERO) iterate into LDS: every load is
// issued before the first store.
template <typename T, int BR, int BC, bool WITH_X>
__device__ __forceinline__ void block_load(BlockLds<T, BR, BC>& s, int tid,
                                           const T* __restrict__ bands, int64_t bs, int N,
                                           const T* __restrict__ b, const T* __restrict__ x,
                                           int r0, int c0) {
    constexpr int W = BlockRegion<BR, BC>::W, E = BlockRegion<BR, BC>::E;
    constexpr int U = (E + BLK_THREADS - 1) / BLK_THREADS;
    const int64_t n = (int64_t)N * N;
    const RowRsrc<T> R(bands, bs, b, n);
    const rsrc_t Rx = make_rsrc(x, n * (int64_t)sizeof(T));
    T r[U][7];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = tid + u * BLK_THREADS;
        const int j = r0 - F_HALO + e / W, col = c0 - F_HALO + e % W;
        const bool in = e < E && in_range(j, 0, N) && in_range(col, 0, N);
        const uint32_t o = in ? node_off(j, N, col, sizeof(T)) : OFF_NONE;
#pragma unroll
        for (int k = 4; k < 9; ++k) r[u][k - 4] = bload<T>(R.band[k], o);
        r[u][5] = bload<T>(R.b, o);
        r[u][6] = WITH_X ? bload<T>(Rx, o) : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = tid + u * BLK_THREADS;
        if (E % BLK_THREADS == 0 || e < E) {
            s.dg[e] = r[u][0];
            s.u5[e] = r[u][1];
            s.u6[e] = r[u][2];
            s.u7[e] = r[u][3];
            s.u8[e] = r[u][4];
            s.b[e] = r[u][5];
            s.p[e] = r[u][6];
        }
    }
}

// Pre-smoothing block (tile row chunk, column strip): what pre_tile computes
// for the same owned nodes.
template <typename T, bool XZERO, int BR, int BC>
__device__ void pre_block(BlockLds<T, BR, BC>& s, const T* __restrict__ bands, int64_t bs, int N,
                          const T* __restrict__ x, const T* __restrict__ b, T omega,
                          T* __restrict__ x2out, T* __restrict__ bc, int dmask, int strip,
                          int chunk) {
    constexpr int W = BlockRegion<BR, BC>::W;
    __syncthreads();  // a workgroup may run several tiles in turn
    const int tid = block_tid();
    const int c0 = strip * BC, c1 = min(c0 + BC, N);
    const int r0 = chunk * BR, r1 = min(r0 + BR, N);
    block_load<T, BR, BC, !XZERO>(s, tid, bands, bs, N, b, x, r0, c0);
    __syncthreads();
    // first sweep (x in p) on the owned nodes widened by 3 -> q
    block_window<BR, BC, 3>(tid, r0, c0, [&](int e, int j, int col) {
        const bool w = in_range(j, max(r0 - 3, 0), min(r1 + 3, N)) &&
                       in_range(col, max(c0 - 3, 0), min(c1 + 3, N));
        T v;
        if (XZERO) {
            v = jacobi_div(omega * s.b[e], s.dg[e]);
        } else {
            const T acc = block_product(s, s.p, e);
            v = s.p[e] + jacobi_div(omega * (s.b[e] - acc), s.dg[e]);
        }
        s.q[e] = w ? v : T(0);
    });
    __syncthreads();
    // second sweep (q) widened by 2 -> p, owned nodes to x2out
    block_window<BR, BC, 2>(tid, r0, c0, [&](int e, int j, int col) {
        const bool w = in_range(j, max(r0 - 2, 0), min(r1 + 2, N)) &&
                       in_range(col, max(c0 - 2, 0), min(c1 + 2, N));
        const T acc = block_product(s, s.q, e);
        T v = s.q[e] + jacobi_div(omega * (s.b[e] - acc), s.dg[e]);
        v = w ? v : T(0);
        if (in_range(j, r0, r1) && in_range(col, c0, c1)) x2out[(int64_t)j * N + col] = v;
        s.p[e] = v;
    });
    __syncthreads();
    // defect (p) widened by 1 -> q
    block_window<BR, BC, 1>(tid, r0, c0, [&](int e, int j, int col) {
        const bool w = in_range(j, max(r0 - 1, 0), min(r1 + 1, N)) &&
                       in_range(col, max(c0 - 1, 0), min(c1 + 1, N));
        const T acc = block_product(s, s.p, e);
        s.q[e] = w ? s.b[e] - acc : T(0);
    });
    __syncthreads();
    // restriction to the owned coarse nodes
    const int Nc = (N >> 1) + 1;
    constexpr int CW = BC / 2, CN = (BR / 2) * (BC / 2);
#pragma unroll
    for (int u = 0; u < (CN + BLK_THREADS - 1) / BLK_THREADS; ++u) {
        const int i = tid + u * BLK_THREADS;
        const int j = r0 + 2 * (i / CW), col = c0 + 2 * (i % CW);
        if ((CN % BLK_THREADS == 0 || i < CN) && j < r1 && col < c1) {
            const int e = (j - r0 + F_HALO) * W + (col - c0 + F_HALO);
            const T* u = s.q + e - W;  // row j - 1
            const T* c = s.q + e;      // row j
            const T* o = s.q + e + W;  // row j + 1
            const T corner = (u[-1] + u[1]) + (o[-1] + o[1]);
            const T edge = (u[0] + o[0]) + (c[-1] + c[1]);
            const T sres = c[0] + T(0.5) * edge + T(0.25) * corner;
            const int I = col >> 1, J = j >> 1;
            bc[(int64_t)J * Nc + I] = is_dirichlet(Nc, I, J, dmask) ? T(0) : sres;
        }
    }
}

// Post-smoothing block: what post_tile computes for the same owned nodes,
// with NORM the same partial sums of squares.
template <typename T, bool NORM, int BR, int BC>
__device__ void post_block(BlockLds<T, BR, BC>& s, const T* __restrict__ bands, int64_t bs, int N,
                           const T* __restrict__ x, const T* __restrict__ xc,
                           const T* __restrict__ b, T omega, T* __restrict__ xout,
                           double* __restrict__ rowpart, int strip, int chunk) {
    constexpr int CR = BlockLds<T, BR, BC>::CR, CC = BlockLds<T, BR, BC>::CC;
    T* const sc = s.sc;
    double* const ns = s.ns;
    constexpr int H = NORM ? 3 : 2;  // halo the last step needs
    const int c0 = strip * BC, c1 = min(c0 + BC, N);
    const int r0 = chunk * BR, r1 = min(r0 + BR, N);
    const int Nc = (N >> 1) + 1;
    __syncthreads();  // a workgroup may run several tiles in turn
    const int tid = block_tid();
    {
        const int J0 = r0 / 2 - 2, I0 = c0 / 2 - 2;
        const rsrc_t Rc = make_rsrc(xc, (int64_t)Nc * Nc * (int64_t)sizeof(T));
        constexpr int U = (CR * CC + BLK_THREADS - 1) / BLK_THREADS;
        T r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = tid + u * BLK_THREADS;
            const int J = J0 + i / CC, I = I0 + i % CC;
            const bool in = i < CR * CC && in_range(J, 0, Nc) && in_range(I, 0, Nc);
            r[u] = bload<T>(Rc, in ? (uint32_t)(J * Nc + I) * (uint32_t)sizeof(T) : OFF_NONE);
        }
        block_load<T, BR, BC, true>(s, tid, bands, bs, N, b, x, r0, c0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = tid + u * BLK_THREADS;
            if ((CR * CC) % BLK_THREADS == 0 || i < CR * CC) sc[i] = r[u];
        }
    }
    __syncthreads();
    // x + P x_c on the owned nodes widened by H (the arithmetic of
    // prolong_elem), in place in p
    block_window<BR, BC, H>(tid, r0, c0, [&](int e, int j, int col) {
        const bool use = in_range(j, max(r0 - H, 0), min(r1 + H, N)) &&
                         in_range(col, max(c0 - H, 0), min(c1 + H, N));
        const int ci = ((j >> 1) - (r0 / 2 - 2)) * CC + ((col >> 1) - (c0 / 2 - 2));
        const int cs = use ? ci : 0;
        const T k0 = sc[cs], k1 = sc[cs + 1], k2 = sc[cs + CC], k3 = sc[cs + CC + 1];
        const bool c_even = !(col & 1);
        const T v_row = c_even ? k0 : T(0.5) * (k0 + k1);
        const T v_odd = c_even ? T(0.5) * (k0 + k2) : T(0.25) * ((k0 + k1) + (k2 + k3));
        const T v = (j & 1) ? v_odd : v_row;
        s.p[e] = use ? s.p[e] + v : T(0);
    });
    __syncthreads();
    // first sweep (p) widened by H-1 -> q
    block_window<BR, BC, H - 1>(tid, r0, c0, [&](int e, int j, int col) {
        const bool w = in_range(j, max(r0 - (H - 1), 0), min(r1 + (H - 1), N)) &&
                       in_range(col, max(c0 - (H - 1), 0), min(c1 + (H - 1), N));
        const T acc = block_product(s, s.p, e);
        const T v = s.p[e] + jacobi_div(omega * (s.b[e] - acc), s.dg[e]);
        s.q[e] = w ? v : T(0);
    });
    __syncthreads();
    // second sweep (q) widened by H-2 -> p, owned nodes to xout
    block_window<BR, BC, H - 2>(tid, r0, c0, [&](int e, int j, int col) {
        const bool w = in_range(j, max(r0 - (H - 2), 0), min(r1 + (H - 2), N)) &&
                       in_range(col, max(c0 - (H - 2), 0), min(c1 + (H - 2), N));
        const T acc = block_product(s, s.q, e);
        T v = s.q[e] + jacobi_div(omega * (s.b[e] - acc), s.dg[e]);
        v = w ? v : T(0);
        if (in_range(j, r0, r1) && in_range(col, c0, c1)) xout[(int64_t)j * N + col] = v;
        s.p[e] = v;
    });
    if (!NORM) return;
    __syncthreads();
    // each column's sum of squares over a group of F_NORM_ROWS rows, rows in
    // increasing order, then the segments' eight column sums
    constexpr int W = BlockRegion<BR, BC>::W;
    constexpr int NG = BR / F_NORM_ROWS, NC = NG * BC;
#pragma unroll
    for (int u = 0; u < (NC + BLK_THREADS - 1) / BLK_THREADS; ++u) {
        const int i = tid + u * BLK_THREADS;
        if (NC % BLK_THREADS == 0 || i < NC) {
            const int g = i / BC, c = i % BC;
            const bool own = c0 + c < c1;
            double acc2 = 0.0;
#pragma unroll
            for (int k = 0; k < F_NORM_ROWS; ++k) {
                const int j = r0 + g * F_NORM_ROWS + k;
                const int e = (j - r0 + F_HALO) * W + c + F_HALO;
                const T d = s.b[e] - block_product(s, s.p, e);
                if (j < r1) acc2 += own ? (double)d * (double)d : 0.0;
            }
            ns[i] = acc2;
        }
    }
    __syncthreads();
    constexpr int NSG = BC / F_NORM_COLS, NP = NG * NSG;
    const int nseg = (N + F_NORM_COLS - 1) / F_NORM_COLS;
    if (tid < NP) {
        const int g = tid / NSG, m = tid % NSG;
        if (r0 + g * F_NORM_ROWS < r1 && c0 + m * F_NORM_COLS < c1) {
            const double* v = ns + g * BC + m * F_NORM_COLS;
            const double s8 =
                ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
            rowpart[(int64_t)(r0 / F_NORM_ROWS + g) * nseg + c0 / F_NORM_COLS + m] = s8;
        }
    }
}

// ---------------------------------------------------------------- coarse tail
// Levels at and below TAIL_MAX hold at most 33 x 33 nodes: one workgroup
// runs the whole V(2,2) sub-cycle over them, with workgroup barriers
// between the steps instead of kernel launches.  The bands of these levels
// and every work vector live in LDS for the whole sub-cycle (one load of the
// bands and of b at the top level, one store of x at the top level), so the
// chain of dependent steps runs at LDS latency.  Per-node arithmetic is the
// one of the separate kernels: same results, bit for bit.
constexpr int TAIL_MAX = 5;
constexpr int TAIL_THREADS = 1024;  // about one node of the 33 x 33 level per thread

template <typename T>
struct TailLevel {
    const T* bands;
    T* x;
    T* b;
    T* t;
    int64_t bs;
    int64_t n;
    int N;
    int pad;
};

template <typename T>
struct TailLevels {
    TailLevel<T> lv[TAIL_MAX + 1];  // index = level
    CoarseSolver cs;                // coarsest solve; cs.dmask: the Dirichlet sides
    int top;  // highest level of the tail; entered with a zero iterate
    int Lc;
};

// LDS image of level l: 9 bands (band-major, stride n), then x with N+1
// zeros on either side, b, and t with N+1 zeros on either side (the zeros
// stand for the neighbours outside the grid of the band products).
__host__ __device__ constexpr int tail_level_elems(int l) {
    return 12 * ((1 << l) + 1) * ((1 << l) + 1) + 4 * ((1 << l) + 2);
}
__host__ __device__ constexpr int tail_lds_elems() {
    int e = 0;
    for (int l = 1; l <= TAIL_MAX; ++l) e += tail_level_elems(l);
    return e;
}

template <typename T>
struct TailLds {
    T* bands;
    T* x;
    T* b;
    T* t;
    int N, n;
    __device__ TailLds(T* lds, int Lc, int l) {
        int off = 0;
        for (int m = Lc; m < l; ++m) off += tail_level_elems(m);
        N = (1 << l) + 1;
        n = N * N;
        const int pad = N + 1;
        bands = lds + off;
        x = bands + 9 * n + pad;
        b = x + n + pad;
        t = b + n + pad;
    }
};

// Band product at node p of an LDS level: the fma chain of stencil_tile.
template <typename T>
__device__ __forceinline__ T tail_product(const TailLds<T>& v, const T* __restrict__ x, int p) {
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < 9; ++k)
        acc = fma(v.bands[k * v.n + p], x[p + (k / 3 - 1) * v.N + (k % 3 - 1)], acc);
    return acc;
}

// Damped Jacobi sweep xo = x + omega (b - A x) / a_pp on an LDS level.
template <typename T>
__device__ __forceinline__ void tail_jacobi(const TailLds<T>& v, const T* x, T* xo, T omega) {
    for (int p = threadIdx.x; p < v.n; p += TAIL_THREADS) {
        const T acc = tail_product(v, x, p);
        xo[p] = x[p] + jacobi_div(omega * (v.b[p] - acc), v.bands[4 * v.n + p]);
    }
}

// x_top = V(top, 0, b_top) over levels top..Lc (one workgroup of TAIL_THREADS
// threads).
// Elements per thread of one level's nine bands, and of the top level's b.
__host__ __device__ constexpr int tail_band_loads(int l) {
    return (9 * ((1 << l) + 1) * ((1 << l) + 1) + TAIL_THREADS - 1) / TAIL_THREADS;
}
__host__ __device__ constexpr int tail_all_loads() {
    int c = ((1 << TAIL_MAX) + 1) * ((1 << TAIL_MAX) + 1) / TAIL_THREADS + 1;
    for (int l = 1; l <= TAIL_MAX; ++l) c += tail_band_loads(l);
    return c;
}

// The bands of levels Lc..top and b of level top from global memory into
// LDS.  Every load is issued, unconditionally, before the first store (the
// levels and the elements per thread are unrolled to constants; a load that
// is not needed reads a valid element of the top level and is not stored), so
// the copy costs about one memory latency instead of one per element a
// thread moves.
template <typename T>
__device__ __forceinline__ void tail_load(const TailLevels<T>& tl, T* lds) {
    T r[tail_all_loads()];
    const TailLevel<T>& gt = tl.lv[tl.top];
    int o = 0;
#pragma unroll
    for (int l = 1; l <= TAIL_MAX; ++l) {
        const int n = ((1 << l) + 1) * ((1 << l) + 1);
        const bool on = l >= tl.Lc && l <= tl.top;
        const TailLevel<T>& g = tl.lv[l];
#pragma unroll
        for (int u = 0; u < tail_band_loads(l); ++u) {
            const int e = (int)threadIdx.x + u * TAIL_THREADS;
            const int ec = min(e, 9 * n - 1);
            const int k = ec / n, p = ec - k * n;
            r[o + u] = *(on ? g.bands + (int64_t)k * g.bs + p : gt.bands);
        }
        o += tail_band_loads(l);
    }
    constexpr int BL = ((1 << TAIL_MAX) + 1) * ((1 << TAIL_MAX) + 1) / TAIL_THREADS + 1;
#pragma unroll
    for (int u = 0; u < BL; ++u) {
        const int p = (int)threadIdx.x + u * TAIL_THREADS;
        r[o + u] = gt.b[min(p, (int)gt.n - 1)];
    }
    o = 0;
#pragma unroll
    for (int l = 1; l <= TAIL_MAX; ++l) {
        const int n = ((1 << l) + 1) * ((1 << l) + 1);
        if (l >= tl.Lc && l <= tl.top) {
            const TailLds<T> v(lds, tl.Lc, l);
#pragma unroll
            for (int u = 0; u < tail_band_loads(l); ++u) {
                const int e = (int)threadIdx.x + u * TAIL_THREADS;
                if (e < 9 * n) v.bands[e] = r[o + u];
            }
            for (int e = threadIdx.x; e < v.N + 1; e += TAIL_THREADS) {
                v.x[-v.N - 1 + e] = v.x[v.n + e] = T(0);
                v.t[-v.N - 1 + e] = v.t[v.n + e] = T(0);
            }
        }
        o += tail_band_loads(l);
    }
    {
        const TailLds<T> v(lds, tl.Lc, tl.top);
#pragma unroll
        for (int u = 0; u < BL; ++u) {
            const int p = (int)threadIdx.x + u * TAIL_THREADS;
            if (p < v.n) v.b[p] = r[o + u];
        }
    }
}

template <typename T>
__device__ void tail_cycle(const TailLevels<T>& tl, T omega) {
    __shared__ T lds[tail_lds_elems()];
    tail_load(tl, lds);
    __syncthreads();
    for (int l = tl.top; l > tl.Lc; --l) {
        const TailLds<T> v(lds, tl.Lc, l);
        for (int p = threadIdx.x; p < v.n; p += TAIL_THREADS)
            jacobi_zero_elem(v.bands + 4 * v.n, v.b, v.t, p, omega);
        __syncthreads();
        tail_jacobi(v, v.t, v.x, omega);
        __syncthreads();
        for (int p = threadIdx.x; p < v.n; p += TAIL_THREADS) v.t[p] = v.b[p] - tail_product(v, v.x, p);
        __syncthreads();
        const TailLds<T> c(lds, tl.Lc, l - 1);
        for (int q = threadIdx.x; q < c.n; q += TAIL_THREADS)
            restrict_elem<T>(v.N, v.t, c.b, q % c.N, q / c.N, tl.cs.dmask);
        __syncthreads();
    }
    {
        const TailLds<T> c(lds, tl.Lc, tl.Lc);
        coarse_block<T>(tl.cs, c.N, c.b, c.x);
    }
    for (int l = tl.Lc + 1; l <= tl.top; ++l) {
        const TailLds<T> v(lds, tl.Lc, l);
        const TailLds<T> c(lds, tl.Lc, l - 1);
        for (int p = threadIdx.x; p < v.n; p += TAIL_THREADS) prolong_elem<T>(v.N, c.x, v.x, p % v.N, p / v.N);
        __syncthreads();
        tail_jacobi(v, v.x, v.t, omega);
        __syncthreads();
        tail_jacobi(v, v.t, v.x, omega);
        __syncthreads();
    }
    const TailLds<T> v(lds, tl.Lc, tl.top);
    for (int p = threadIdx.x; p < v.n; p += TAIL_THREADS) tl.lv[tl.top].x[p] = v.x[p];
}

}  // namespace dev
}  // namespace mg
