// Internal declarations of the multigrid library: device-resident hierarchy
// layout and the kernel launchers shared by the C ABI, the solvers, the
// batched path and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "device_ops.h"
#include "mgfem.h"

namespace mg {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
mg_status fail(mg_status s, const std::string& msg);

#define MG_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::mg::fail(MG_ERR_DEVICE, std::string(#call) + ": " +              \
                                                 hipGetErrorString(e_));              \
    } while (0)

// ---------------------------------------------------------------- layout
// Band arrays of one level live in one allocation: band k starts at
// k * band_stride elements.  The stride is n rounded up to 1024 elements plus
// 64, so that the nine streams of a band product do not start on the same
// HBM channel.
int64_t band_stride(int64_t n);
// Vectors are padded to a multiple of 64 elements (the tail stays zero).
int64_t vec_len(int64_t n);

struct Level {
    int l = 0;
    int N = 0;
    int64_t n = 0;
    int64_t bs = 0;           // band stride (elements)
    double* bands64 = nullptr;
    float* bands32 = nullptr;
    double *x64 = nullptr, *b64 = nullptr, *t64 = nullptr;
    float *x32 = nullptr, *b32 = nullptr, *t32 = nullptr;
};

}  // namespace mg

struct mg_context {
    int device = 0;
    size_t budget = 0;      // 0: unlimited
    size_t in_use = 0;
    size_t high_water = 0;
    std::mutex mu;
    // reduction scratch of the BLAS level-1 calls (grown on demand, charged)
    std::mutex blas_mu;
    double* blas_scratch = nullptr;
    size_t blas_bytes = 0;
    double* blas_host = nullptr;  // pinned result mirror
    // Charge `bytes` against the budget; false if it does not fit.
    bool reserve(size_t bytes);
    void release(size_t bytes);
};

namespace mg {
// A named host range in profiler traces (rocprofv3 --marker-trace): the
// span of a solve, an outer step, an iteration, a host wait.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};
}  // namespace mg

struct GraphCache;  // defined in solve.hip

struct mg_hierarchy {
    mg_context* ctx = nullptr;
    int L = 0, Lc = 1;
    int dmask = 15;                // Dirichlet sides (bits 1: x=0, 2: x=1, 4: y=0, 8: y=1)
    size_t charged = 0;
    std::vector<void*> allocs;
    mg::Level lv[MG_MAX_LEVEL + 1];
    double* coords = nullptr;      // finest coordinates, 2n
    double* d64 = nullptr;         // finest FP64 defect (mixed solver)
    double* partials = nullptr;    // per-block partial sums of the reductions
    int64_t n_partials = 0;
    double* scal = nullptr;        // device scalars (norms), 64 doubles
    double* host_scal = nullptr;   // pinned mirror of scal
    double* chol = nullptr;        // m x m Cholesky factor of the coarse unknowns' block
    int m = 0;                     // coarse unknowns (nodes off the Dirichlet sides)
    int coarse_cg = 0;             // coarsest solve: 1 conjugate gradients, 0 Cholesky
    double coarse_tol = 1e-10;     // CG stop: ||r|| <= coarse_tol ||b||
    int coarse_max_iter = 200;     // CG step limit
    int* flag = nullptr;           // device status flag of the coarse factorisation
    bool assembled = false;
    GraphCache* graphs = nullptr;
    // FP32 cycles the mixed solve's inner loops took at outer steps 1..8 of
    // the previous solve (the number of cycles queued at once next time)
    int inner_pred[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // outer steps of the previous such solve (0: none yet): later steps are
    // not queued ahead of their defect's norm
    int outer_prev = 0;
};

namespace mg {

// Scalar slots in hierarchy::scal (sum of squares at s, norm at s+1).
enum : int {
    SC_B = 0,
    SC_R64 = 2,
    SC_R32 = 4,
    SC_D32 = 6,   // norm at +1: the scaled FP64 defect the inner loop is relative to
    SC_USER = 8,
    // preconditioned CG: p.q, r.z (current and previous), ||r||
    SC_PQ = 10,
    SC_RZ = 12,
    SC_RZ_OLD = 14,
    SC_RR = 16,
    SC_XNZ = 18,  // nonzero elements of the initial iterate
    // device control of the mixed solve's inner loop (k_inner_ctrl)
    SC_STOP = 20,  // nonzero: the loop is over (its remaining cycles return at once)
    SC_WAIT = 21,  // nonzero: the loop is still running (the update waits)
    SC_ITER = 22,  // cycles run; host mirror: the same, plus ITER_DONE once over
    SC_RED = 23,   // FP32 residual reduction factor of the loop
    SC_CAP = 24,   // cycle cap of the loop
    SC_CONV = 25,  // nonzero: the outer loop is over (the work queued after returns)
    SC_R64B = 26,  // FP64 outer defect norm of even outer steps (odd ones: SC_R64)
    SC_XZ = 28     // 1 if the initial iterate is zero (RED_ZFLAG), else 0
};
constexpr double ITER_DONE = 1000.0;

// What the final kernel of a reduction does besides writing the norm: the
// mixed solve's decisions on the device (see red_control in kernels.hip).
enum : int { RED_NONE = 0, RED_OUTER = 1, RED_STEP = 3, RED_ZFLAG = 4 };
struct RedCtl {
    int mode = RED_NONE;
    double thr = 0.0;  // OUTER: stop at norm <= thr ||b||
    double div = 0.0;  // OUTER: diverged above div ||b||
    int cap = 0;       // OUTER: nonzero stops (step count used up)
    int reset = 0;     // OUTER: a step that goes on also starts its inner loop
    double ithr = 0.0; // OUTER with reset: the inner reduction factor
    int icap = 0;      // OUTER with reset: the inner cycle cap
};

// How the hierarchy's coarsest level is solved.
dev::CoarseSolver coarse_solver(const mg_hierarchy* h);

// ---------------------------------------------------------------- kernels
// All launchers enqueue on `st` and return the HIP launch error.
hipError_t launch_coords(double* xy, int L, double jitter, uint64_t seed, hipStream_t st);
// Coordinates and the seeded uniform right-hand side with x0 = 0 (one launch;
// the same values as launch_coords + launch_rhs_uniform).
hipError_t launch_coords_rhs(double* xy, int L, double jitter, uint64_t geom_seed,
                             uint64_t rhs_seed, int dmask, double* b, double* x0,
                             hipStream_t st);
// dmask below: the Dirichlet sides of the problem (bits as in mg_hierarchy).
// Bands of levels Lc..L (lv indexed by level) from the finest coordinates.
hipError_t launch_assemble(const double* xy_fine, const Level* lv, int Lc, int L, int dmask,
                           hipStream_t st);
hipError_t launch_chol_factor(const Level& lc, int dmask, double* chol, int* flag,
                              hipStream_t st);
hipError_t launch_rhs_sinsin(const double* xy, int N, double* b, hipStream_t st);
// Seeded uniform right-hand side; x0 (nullable) set to zero alongside.
hipError_t launch_rhs_uniform(int N, uint64_t seed, int dmask, double* b, double* x0,
                              hipStream_t st);

// Stencil family on one level.
template <typename T>
// sym: read the lower bands as shifted upper bands (same values for the
// assembled, symmetric matrices; five band streams from HBM instead of nine).
hipError_t launch_spmv(const Level& lv, const T* bands, const T* x, T* y, hipStream_t st,
                       bool sym = false);
// Reductions land in scal[slot] (sum of squares) and scal[slot+1] (norm) in
// device memory and, when host is not null, also in host[slot], host[slot+1]
// (pinned memory, for the host to read once the stream has synchronized).
// d = b - A x (d may be null); if partials != null also writes per-block
// sums of d^2 and reduces them.
// A guard makes every kernel of the launch return at once while *guard != 0;
// the fused passes, the tail, the reductions, the cast and the update take
// one too.  ctl: see RedCtl.
template <typename T>
hipError_t launch_defect(const Level& lv, const T* bands, const T* b, const T* x, T* d,
                         double* partials, double* scal, int slot, double* host, hipStream_t st,
                         const double* guard = nullptr, RedCtl ctl = {});
template <typename T>
hipError_t launch_jacobi(const Level& lv, const T* bands, const T* b, const T* x, T* xo,
                         T omega, hipStream_t st);
// Jacobi sweep from a zero initial guess: xo = omega b / diag.
template <typename T>
hipError_t launch_jacobi_zero(const Level& lv, const T* bands, const T* b, T* xo, T omega,
                              hipStream_t st);
template <typename T>
hipError_t launch_restrict(int Nf, const T* d_f, T* b_c, int dmask, hipStream_t st);
template <typename T>
hipError_t launch_prolong(int Nf, const T* x_c, T* x_f, hipStream_t st);
template <typename T>
hipError_t launch_coarse(const dev::CoarseSolver& cs, int Nc, const T* b, T* x, hipStream_t st);
template <typename T>
hipError_t launch_copy(const T* src, T* dst, int64_t n, hipStream_t st);
// Sum of squares of v (accumulated in FP64) into scal[slot], norm into
// scal[slot+1].
template <typename T>
hipError_t launch_norm(const T* v, int64_t n, double* partials, double* scal, int slot,
                       double* host, hipStream_t st);
template <typename T>
hipError_t launch_fill(T* v, int64_t n, T value, hipStream_t st);
// d32 = float(d64 / s) with s = scal[slot + 1] (0 if s == 0).
hipError_t launch_cast_scaled(const double* d64, float* d32, int64_t n, const double* scal,
                              int slot, hipStream_t st);
// scal[slot] = number of nonzero elements of v (FP64, exact).
hipError_t launch_count_nonzero(const double* v, int64_t n, double* partials, double* scal,
                                int slot, double* host, hipStream_t st, RedCtl ctl = {});
// launch_defect (FP64, with the norm; d may be null) for x = 0: the same
// bits, from b alone.
hipError_t launch_defect_zero_x(const Level& lv, const double* b, double* d, double* partials,
                                double* scal, int slot, double* host, hipStream_t st,
                                const double* guard = nullptr, RedCtl ctl = {});
// The mixed scheme's FP64 defect of an outer step: launch_defect (with
// the norm into scal[slot]) writing float(d sc) into d32 instead of d, sc =
// dev::pow2_scale(||b||) (||b|| = scal[SC_B + 1]); and the same for a zero
// iterate (d = b, launch_defect_zero_x's bits).
hipError_t launch_defect_cast(const Level& lv, const double* bands, const double* b,
                              const double* x, float* d32, double* partials, double* scal,
                              int slot, double* host, hipStream_t st,
                              const double* guard = nullptr, RedCtl ctl = {});
hipError_t launch_defect_zero_x_cast(const Level& lv, const double* b, float* d32,
                                     double* partials, double* scal, int slot, double* host,
                                     hipStream_t st, const double* guard = nullptr,
                                     RedCtl ctl = {});
// x += u double(c32), u = dev::pow2_unscale(||b||) (||b|| = scal[SC_B + 1]):
// the FP32 correction scaled back.  x_zero: x is taken as zero and not read
// (the same bits as with a zeroed x).
hipError_t launch_update(double* x, const float* c32, int64_t n, const double* scal,
                         hipStream_t st, const double* guard = nullptr, bool x_zero = false);

// Deterministic sum of np partials (dev::reduce_partials' order; one
// block, or beyond dev::RED_SEG partials one block per segment whose sums go
// right after the partials, padded to 64, and are summed by the last of
// them): scal[slot] = sum, scal[slot + 1] = sqrt(sum), mirrored into
// host[slot..] when not null.  Every partials buffer is preceded by one
// reserved 8-byte word, zero when allocated: the ticket of the segmented
// form (back to zero after each reduction).
constexpr int64_t PARTIALS_FRONT = 64;  // doubles reserved before a partials buffer
hipError_t launch_reduce(double* partials, int64_t np, double* scal, int slot, double* host,
                         hipStream_t st, const double* guard = nullptr, RedCtl ctl = {});

// Preconditioned CG vector operations.  z is FP64, or FP32 scaled by
// zscal[zslot + 1] (zslot >= 0).  u . z into scal[slot]; p = z + beta p with
// beta = scal[s_new] / scal[s_old]; alpha = scal[s_num] / scal[s_den],
// x += alpha p, r -= alpha q and ||r||^2 into scal[slot] (norm at slot + 1,
// mirrored to host when not null); scal[to..to+1] = scal[from..from+1].
template <typename TZ>
hipError_t launch_dot(const double* u, const TZ* z, int64_t n, const double* zscal, int zslot,
                      double* partials, double* scal, int slot, hipStream_t st);
template <typename TZ>
hipError_t launch_pcg_dir(double* p, const TZ* z, int64_t n, const double* scal, int zslot,
                          int s_new, int s_old, hipStream_t st);
hipError_t launch_pcg_step(double* x, double* r, const double* p, const double* q, int64_t n,
                           double* scal, int s_num, int s_den, double* partials, int slot,
                           double* host, hipStream_t st);
hipError_t launch_scalar_copy(double* scal, int from, int to, hipStream_t st);

// Fused smoothing passes of a V(2,2) level (see fused_ops.h): pre = two
// sweeps (x_zero: the first from a zero iterate) + defect + restriction into
// bc; post = prolongation/correction + two sweeps, and with partials the
// residual norm reduced into scal[slot], scal[slot + 1].
template <typename T>
hipError_t launch_pre(const Level& lv, const T* bands, const T* x, bool x_zero, const T* b,
                      T omega, T* x2out, T* bc, int dmask, hipStream_t st,
                      const double* guard = nullptr);
template <typename T>
hipError_t launch_post(const Level& lv, const T* bands, const T* x, const T* xc, const T* b,
                       T omega, T* xout, double* partials, double* scal, int slot, double* host,
                       hipStream_t st, const double* guard = nullptr, RedCtl ctl = {});
// The V(2,2) sub-cycle over levels top..Lc (top <= tail_max_level(), entered
// with a zero iterate on level top) in one workgroup.  lv is indexed by level.
template <typename T>
hipError_t launch_tail(const Level* lv, int top, int Lc, const dev::CoarseSolver& cs, T omega,
                       hipStream_t st, const double* guard = nullptr);
int tail_max_level();
// Tiling of the fused passes on a level of N nodes per side: workgroup
// width, chunk height for a pass over `count` problems, geometry of a
// single-problem pass, tiles per single-problem pass, and the residual
// partials of a fused post pass (one layout for every width).
namespace dev {
struct FusedGeom;
}  // namespace dev
int fused_bt(int N);
int fused_rh(int N, int bt, int64_t count);
// Tiling of a single-problem fused pass: a choice under trial by the
// autotuner (set_single_trial; 0, 0, 0 ends it), else the tile table's
// entry for one problem at the level, else the rules.
dev::FusedGeom single_geom(int N);
void set_single_trial(int N, int rows, int bt, int cols = 0);

// Process-wide table of tuned tiles of the fused passes, keyed by level and
// by the number of problems at that level (rounded down to a power of two;
// a single-problem solve counts as one): rows per tile and workgroup width
// in threads of a marching tile, or rows and columns of a block tile; zeros
// when the level has no entry.  Every change advances the table's epoch
// (captured cycles of an older epoch are captured again).
struct TileEntry {
    int rows;
    int bt;
    int cols;  // > 0: a block tile of rows x cols owned nodes
};
TileEntry tile_table_get(int level, int64_t problems);
void tile_table_set(int level, int64_t problems, int rows, int bt, int cols = 0);
void tile_table_clear();
uint64_t tile_table_epoch();
int64_t fused_tiles(int N);
int64_t fused_max_norm_parts(int N);

// Workgroups (= tiles) of a band-product launch and of a vector-norm launch.
int64_t stencil_blocks(int64_t n, int elem_bytes);
int64_t norm_blocks(int64_t n);

}  // namespace mg
