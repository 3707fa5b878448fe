/*
 * mgfem.h -- C ABI of the MI355X multigrid Poisson library.
 *
 * The library solves the Poisson problem -Laplace(u) = f on the unit square
 * (HONEI, arXiv 0904.4152, Sec. 2.1, eq. 1) discretised with conforming
 * bilinear Q1 finite elements on a tensor-product grid that may be deformed
 * (jittered), fully assembled into nine bands (Sec. 2.1; Sec. 4.1 banded
 * matrices with fixed band positions), with a geometric V-cycle of two damped
 * Jacobi pre- and post-smoothing steps (Sec. 6.2), in FP64 or as an FP64
 * defect correction around single-precision multigrid cycles (Sec. 6.2,
 * mixed precision).
 *
 * Conventions shared by every call:
 *   - level l has N = 2^l + 1 nodes per side and n = N*N unknowns (Sec. 2.1:
 *     level L gives (2^L+1)^2 unknowns); node (i,j) (i along x) has index
 *     p = j*N + i;
 *   - band k = 0..8 holds A[p][p + off_k] at index p, off_k =
 *     (k/3 - 1)*N + (k%3 - 1), i.e. offsets -N-1, -N, -N+1, -1, 0, 1, N-1,
 *     N, N+1;
 *   - homogeneous boundary conditions, Dirichlet on a chosen set of sides
 *     (every side unless the hierarchy was made by mg_hierarchy_create_bc)
 *     and the natural (free) Neumann condition on the others (Sec. 2.1:
 *     mixed Dirichlet and Neumann conditions): rows and columns of
 *     Dirichlet nodes are zero except a unit diagonal, and their right-hand
 *     side entries must be zero;
 *   - every vector argument named dev_* or documented as "device" is a
 *     contiguous, unpadded device buffer of n elements in index order p,
 *     owned by the caller; the library never keeps such a pointer after the
 *     call returns;
 *   - stream arguments are hipStream_t values passed as void* (NULL is the
 *     default stream); asynchronous calls only enqueue work on it;
 *   - every call returns an mg_status; on a non-OK status the outputs are
 *     unspecified and mg_last_error() describes the failure (thread local).
 *     No C++ exception crosses this boundary.
 */
#ifndef MGFEM_H
#define MGFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MG_OK = 0,
    MG_ERR_INVALID = 1,  /* bad argument (level, pointer, size, option) */
    MG_ERR_NOMEM = 2,    /* device memory budget or device memory exhausted */
    MG_ERR_NOCONV = 3,   /* max_cycles reached before rel_tol */
    MG_ERR_NUMERIC = 4,  /* NaN/Inf or divergence (residual > 1e3 ||b||) */
    MG_ERR_DEVICE = 5,   /* HIP runtime error */
    MG_ERR_BUSY = 6      /* server: ticket still pending */
} mg_status;

typedef enum { MG_PREC_FP64 = 0, MG_PREC_MIXED = 1 } mg_precision;
typedef enum { MG_F64 = 0, MG_F32 = 1 } mg_dtype;

typedef struct mg_context mg_context;
typedef struct mg_hierarchy mg_hierarchy;
typedef struct mg_server mg_server;

#define MG_MAX_LEVEL 14
#define MG_MAX_COARSE_LEVEL 4
/* Side bits of dirichlet_sides: x = 0, x = 1, y = 0, y = 1. */
#define MG_SIDE_X0 1
#define MG_SIDE_X1 2
#define MG_SIDE_Y0 4
#define MG_SIDE_Y1 8
#define MG_ALL_DIRICHLET 15
/* Solvers of the coarsest level (mg_hierarchy_set_coarse_solver). */
#define MG_COARSE_CHOLESKY 0
#define MG_COARSE_CG 1
#define MG_COARSE_CG_MAX_ITER 10000
#define MG_HIST 128

/* Solver options (Sec. 6.2: V cycle, two damped Jacobi pre- and
 * post-smoothing steps; mixed precision defect correction). */
typedef struct {
    int nu_pre;              /* pre-smoothing sweeps (2) */
    int nu_post;             /* post-smoothing sweeps (2) */
    double omega;            /* Jacobi damping (0.7) */
    double rel_tol;          /* stop when ||b - A x||_2 <= rel_tol ||b||_2 (1e-8) */
    int max_cycles;          /* FP64: V-cycles; mixed: outer steps (100) */
    mg_precision precision;  /* MG_PREC_FP64 or MG_PREC_MIXED */
    double inner_reduction;  /* mixed: FP32 residual reduction per outer step (1e-2) */
    int inner_max_cycles;    /* mixed: cap on FP32 cycles per outer step (8) */
    int fixed_cycles;        /* > 0: run exactly this many cycles / outer steps */
    int use_graph;           /* 1: replay captured HIP graphs for the cycles (1) */
    int krylov;              /* 1: CG preconditioned by one V-cycle (0) */
    int zero_guess;          /* 1: start from x = 0 whatever dev_x holds (dev_x is
                                output only, not read); 0: dev_x is the initial
                                guess (0) */
} mg_solve_opts;

typedef struct {
    mg_status status;
    int cycles;              /* FP64 V-cycles, or FP32 V-cycles of the mixed solve */
    int outer_steps;         /* mixed: FP64 defect-correction updates */
    double bnorm;            /* ||b||_2 */
    double rel_res;          /* ||b - A x||_2 / ||b||_2 at exit, evaluated in FP64 */
    double seconds;          /* host wall time of the call; server: submission to result */
    double alg_bytes;        /* algorithmic HBM bytes of the kernels launched */
    int n_hist;
    double res_hist[MG_HIST]; /* relative residual after each cycle / outer step */
    double queue_seconds;     /* server: submission to admission */
} mg_stats;

/* Defaults: 2, 2, 0.7, 1e-8, 100, FP64, 1e-2, 8, 0, 1, 0. */
void mg_default_opts(mg_solve_opts* opts);
const char* mg_last_error(void);
const char* mg_status_string(mg_status s);

/* ---- context -------------------------------------------------------------
 * A context binds one HIP device and a device-memory budget in bytes (0:
 * no limit beyond the device).  Every allocation of the library is charged
 * against it; a request that would exceed it fails with MG_ERR_NOMEM and
 * leaves nothing allocated (Sec. 4.2: device memory is a hard limit and the
 * library fails cleanly when more is requested).  One context per thread. */
mg_status mg_context_create(int device, size_t hbm_budget_bytes, mg_context** out);
mg_status mg_context_destroy(mg_context* ctx);
mg_status mg_context_memory(const mg_context* ctx, size_t* in_use, size_t* high_water);

/* ---- hierarchy -----------------------------------------------------------
 * Device-resident grid hierarchy for levels coarse_level..L (Sec. 2.1,
 * geometric multigrid): node coordinates, nine FP64 bands per level and
 * their round-to-nearest FP32 copies, and the work vectors of both solvers.
 * Geometry: host_xy (nullable, 2n doubles interleaved x,y for the finest
 * level, copied) or, when NULL, the uniform grid moved at interior nodes by
 * dx = (2u-1)*jitter*h, dy = (2u'-1)*jitter*h with u, u' the SplitMix64
 * draws 2p and 2p+1 of geom_seed, generated on the device.  Coarse levels
 * use the finest coordinates sampled every 2^(L-l) nodes.
 * 1 <= coarse_level <= min(L, 4); L <= 14.  Returns MG_ERR_NOMEM without
 * allocating anything when the hierarchy does not fit the budget. */
mg_status mg_hierarchy_create(mg_context* ctx, int L, int coarse_level, double jitter,
                              uint64_t geom_seed, const double* host_xy, mg_hierarchy** out);
/* The same with Dirichlet conditions only on the sides set in
 * dirichlet_sides (MG_SIDE_* bits, 1..15; Sec. 2.1 mixed conditions, Sec.
 * 6.2.2 free Neumann and geometric Dirichlet sides) and the natural Neumann
 * condition on the rest.  A node on a Dirichlet side is a Dirichlet node,
 * corners included.  Every level and the coarse solve use the same sides;
 * the coarse solve factorises the block of the coarsest level's nodes off
 * the Dirichlet sides.  MG_ERR_INVALID for 0 (the pure Neumann problem is
 * singular) or a value above 15.  mg_hierarchy_create(...) is
 * mg_hierarchy_create_bc(..., MG_ALL_DIRICHLET, out). */
mg_status mg_hierarchy_create_bc(mg_context* ctx, int L, int coarse_level, double jitter,
                                 uint64_t geom_seed, const double* host_xy, int dirichlet_sides,
                                 mg_hierarchy** out);
/* Device bytes mg_hierarchy_create would charge for (L, coarse_level). */
size_t mg_hierarchy_bytes(int L, int coarse_level);
/* Assemble all levels (Sec. 2.1: the matrix is assembled fully): 2x2 Gauss
 * element matrices on the isoparametric bilinear map, Dirichlet treatment,
 * FP32 copy, and the Cholesky factor of the coarsest level's block of
 * non-Dirichlet nodes.
 * Synchronous.  MG_ERR_NUMERIC if the coarse block is not positive definite
 * (a tangled grid). */
mg_status mg_hierarchy_assemble(mg_hierarchy* h, void* stream);
/* How every later cycle of h solves its coarsest level, in FP64 (also the
 * coarse solve of the single-precision cycles):
 *   MG_COARSE_CHOLESKY (the default): the Cholesky factor of the block of
 *     the nodes off the Dirichlet sides, made by mg_hierarchy_assemble
 *     (single-threaded substitutions: fast up to coarse level 2 or 3);
 *   MG_COARSE_CG: unpreconditioned conjugate gradients from a zero iterate
 *     (Sec. 6.2 uses CG for the coarse grid problems), stopping before a step
 *     once ||r|| <= tol ||b|| (r by the recurrence) or after max_iter steps
 *     (1..MG_COARSE_CG_MAX_ITER; tol in [0, 1)).  Its dot products have one
 *     fixed summation order, so every path gives the same bits.
 * tol and max_iter are ignored for MG_COARSE_CHOLESKY.  Synchronises the
 * device and drops the hierarchy's captured cycles.  Not thread safe per
 * hierarchy. */
mg_status mg_hierarchy_set_coarse_solver(mg_hierarchy* h, int solver, double tol, int max_iter);
mg_status mg_hierarchy_destroy(mg_hierarchy* h);
mg_status mg_hierarchy_info(const mg_hierarchy* h, int* L, int* coarse_level, int64_t* n_finest);
/* Copy the 9*n band values of one level to host memory, band-major
 * (host_out[k*n + p]); dtype selects the FP64 or FP32 copy.  Synchronous. */
mg_status mg_get_bands(const mg_hierarchy* h, int level, mg_dtype dtype, void* host_out);
/* Copy the 2n coordinates (x,y interleaved) of one level to host memory. */
mg_status mg_get_coords(const mg_hierarchy* h, int level, double* host_out);

/* Right-hand sides on the finest level (asynchronous on stream):
 * mg_rhs_sinsin: load vector of f = 2 pi^2 sin(pi x) sin(pi y) (3x3 Gauss),
 * whose exact solution is u = sin(pi x) sin(pi y) (Sec. 6.2.1 accuracy test
 * with an analytically known solution), boundary entries 0; only for a
 * hierarchy with every side Dirichlet (MG_ERR_INVALID otherwise);
 * mg_rhs_uniform: b_p = 2u - 1 with u the SplitMix64 draw p of seed, at
 * nodes off the Dirichlet sides, 0 on them. */
mg_status mg_rhs_sinsin(const mg_hierarchy* h, double* dev_b, void* stream);
mg_status mg_rhs_uniform(const mg_hierarchy* h, uint64_t seed, double* dev_b, void* stream);

/* ---- solve (Sec. 6.2) -------------------------------------------------------
 * Solve A x = b on the finest level.  dev_x is in/out (initial guess, then
 * the solution; with opts->zero_guess output only).  FP64: V-cycles until ||b - A x|| <= rel_tol ||b||.  Mixed:
 * FP64 defect d = b - A x and norm s, d32 = float(d 2^-e) with e the binary
 * exponent of ||b|| (||b|| = m 2^e, m in [0.5, 1); a power of two scales
 * exactly, it only keeps the FP32 values in range), FP32 V-cycles on
 * A32 c = d32 from c = 0 until the FP32 residual is at most inner_reduction
 * 2^-e s (at most inner_max_cycles), x += 2^e double(c); the coarsest solve
 * is always FP64.
 * krylov = 1: conjugate gradients preconditioned by one V(nu_pre, nu_post)
 * cycle from a zero iterate (Sec. 4.1: a solver plugged into another as its
 * preconditioner), in FP64; the cycle is FP64, or with MG_PREC_MIXED an FP32
 * cycle on r / ||r|| scaled back by ||r||.  Stops once the recurrence
 * residual ||r|| <= rel_tol ||b||; stats.cycles counts CG steps (one cycle
 * each), res_hist the recurrence residuals, rel_res the true residual at
 * exit; inner_reduction and inner_max_cycles are unused.
 * Returns after the result is in dev_x.  The solve runs on an internal
 * stream that waits (on the device, not the host) for the work queued on
 * `stream` before the call, and work queued on `stream` after the call waits
 * for the solve's.  The mixed solver updates dev_x in place as it goes (the
 * others write it at the end), so dev_x holds the last iterate also after
 * an error.  With the V(2,2) cycle on a hierarchy with levels above 5 the
 * mixed solver's inner loop is decided on the device (same decisions and
 * bits as the host loop; the host reads one state per outer step).  Not
 * thread safe per hierarchy.  stats may be NULL. */
mg_status mg_solve(mg_hierarchy* h, const double* dev_b, double* dev_x,
                   const mg_solve_opts* opts, void* stream, mg_stats* stats);

/* ---- batched solve ---------------------------------------------------------
 * Not a passage of the paper: the library's entry point for many small
 * solves at once, each exactly the mixed solve of Sec. 6.2.
 * Solve count independent problems A_p x_p = b_p (each with its own
 * assembled hierarchy; levels may differ, the coarse level must agree) with
 * the mixed-precision scheme of mg_solve, advancing all of them together:
 * each V-cycle stage is one persistent launch over every problem that has
 * that level, and each problem's outer/inner stop decisions are taken on the
 * device.  A problem's arithmetic does not depend on the other problems in
 * the batch (its result equals a batch of one bit for bit).  opts: NULL
 * (defaults, mixed) or an array of count entries; precision must be
 * MG_PREC_MIXED, krylov 0, and nu_pre/nu_post must agree.  b[p], x[p]: device vectors
 * of that problem's finest n; x is in/out (with opts zero_guess output
 * only) and is updated in place as the solve goes, b is read in place: no
 * x may be another problem's x or any problem's b (MG_ERR_INVALID), and
 * neither may change during the call.  stats: NULL or count entries.
 * Synchronous.  Returns the first non-OK per-problem status, if any.
 * The batch machinery (device descriptors of the problems, work lists and
 * the captured iteration graph; a few MB of device memory outside any
 * context budget) is kept after the call and reused by later calls with the
 * same device, largest level, coarse level and smoothing counts; at most
 * four idle sets are kept, until the process ends.  Concurrent calls use
 * separate sets; one hierarchy must not be in two concurrent calls. */
mg_status mg_solve_batch(mg_hierarchy* const* hs, const double* const* b, double* const* x,
                         int count, const mg_solve_opts* opts, void* stream, mg_stats* stats);

/* ---- batched tiles: autotuner ----------------------------------------------
 * Sec. 3: the GPU thread-block partition is a runtime parameter.  The fused
 * passes of the batched solver process each level in marching tiles, a
 * strip of columns by a number of grid rows with a workgroup of 1 to 4
 * wavefronts across a strip's row, or in block tiles of 8, 16 or 32 rows by
 * 32 columns (one 256-thread workgroup, the tile and its halo in LDS).  The
 * choice comes from a process-wide table filled by this autotuner, keyed by
 * level and by the number of problems at that level rounded down to a power
 * of two; levels without an entry use marching tiles with the rules
 * "fewest threads per row" (width) and "largest height in 4..64 that still
 * gives about 3500 wavefronts" (rows).  No result bit depends on the tiles:
 * a batched result equals the single solve bit for bit whatever the table
 * holds.  The server applies tuned rows only (a width or shape change would
 * re-capture its iteration graph while its mix changes).
 * mg_batch_autotune: for the composition of these problems (options as for
 * mg_solve_batch; NULL: defaults), times the fused pre- and post-smoothing
 * passes of every level for each of 4, 8, 12, 16, 24, 32, 48, 64, 96 rows per
 * tile and 1, 2, 3, 4 wavefronts per row, and on levels of at most 1025 nodes per side for
 * each block tile (reps pairs each, on the problems' FP32 work vectors,
 * which no later solve reads before writing), stores the fastest in the
 * table and writes up to out_cap choices to out (*n_out = choices).
 * Synchronous; thread safe with respect to other batches on separate
 * hierarchies.  Only V(2,2) cycles have tiles.
 * mg_batch_set_tile: installs one entry (e.g. read back from a file): with
 * tile_cols = 0 a marching tile, tile_rows a multiple of 4 in [4, 256],
 * row_waves in 1..4 or 0 for the width rule; with tile_cols = 32 a block
 * tile, tile_rows 8, 16 or 32, row_waves 0 or 4.  mg_batch_clear_tiles:
 * empties the table. */
typedef struct {
    int level;
    int problems;     /* problems at this level in the tuned composition */
    int tile_rows;    /* chosen rows per tile */
    int row_waves;    /* chosen wavefronts per workgroup (across a strip's row when marching) */
    int tile_cols;    /* 0: marching tile; else columns of a block tile */
    double us;        /* one pre + post pass pair with that tile, microseconds */
} mg_tile_choice;
mg_status mg_batch_autotune(mg_hierarchy* const* hs, int count, const mg_solve_opts* opts,
                            int reps, mg_tile_choice* out, int out_cap, int* n_out);
mg_status mg_batch_set_tile(int level, int problems, int tile_rows, int row_waves,
                            int tile_cols);
mg_status mg_batch_clear_tiles(void);
/* The same tuning for the single-problem solver (mg_solve, mg_vcycle and
 * the fused-pass entry points read the table's entries for one problem): for
 * every level on which h's V(2,2) cycle runs fused passes, times the FP32
 * pre- and post-smoothing passes as the mixed solve runs them (reps pairs
 * per candidate, on h's FP32 work vectors) for 4, 8, 12, 16, 24, 32, 40, 48,
 * 64, 80, 96, 128, 160, 192 and 256 rows per tile and 1 .. 4 wavefronts per
 * row, and on levels of at most 1025 nodes per side for
 * each block tile, and stores the fastest under problems = 1.  Tiles
 * change no result bit; solves captured before are captured again.
 * Synchronous; not thread safe per hierarchy. */
mg_status mg_hierarchy_autotune(mg_hierarchy* h, int reps, mg_tile_choice* out, int out_cap,
                                int* n_out);

/* ---- serving ---------------------------------------------------------------
 * Not a passage of the paper: the library's continuous-batching service
 * around the batched solve, under the device-memory limit of Sec. 4.2.
 * A server owns a BatchEngine of `slots` slots, a scheduler thread and a pool
 * of device-resident hierarchies of levels coarse_level..max_level charged
 * against hbm_budget_bytes (and the context budget).  Requests are admitted
 * in arrival order when a slot is free and their hierarchy fits the budget
 * (idle hierarchies of other levels are evicted first); their problem is
 * generated on the device (jittered grid from geom_seed, assembly, uniform
 * right-hand side from rhs_seed, x0 = 0) and solved with the mixed scheme to
 * rel_tol, advancing together with every other live request, one
 * graph-replayed iteration at a time (continuous batching).  A request whose
 * hierarchy cannot fit even on an idle server finishes with MG_ERR_NOMEM.
 * opts (nullable): smoothing, omega and inner-loop options shared by all
 * requests (precision and krylov are forced to MG_PREC_MIXED and 0).
 * Thread safe. */
typedef struct {
    uint64_t completed;
    size_t queued;
    int live;
    size_t queue_high_water;
    size_t bytes;             /* hierarchies held (live + idle pool) */
    size_t bytes_high_water;
    double busy_seconds;      /* time with at least one iteration on the device */
} mg_server_info_t;

mg_status mg_server_create(mg_context* ctx, int slots, size_t hbm_budget_bytes, int max_level,
                           int coarse_level, const mg_solve_opts* opts, mg_server** out);
/* Queue a request; never blocks on the device.  keep_x != 0 keeps the
 * solution for collection.  MG_ERR_NOMEM if the level can never fit. */
mg_status mg_server_submit(mg_server* s, int L, double rel_tol, double jitter,
                           uint64_t geom_seed, uint64_t rhs_seed, int keep_x, uint64_t* ticket);
/* MG_ERR_BUSY while the ticket is pending; otherwise the request's status,
 * its stats (seconds = submission to result on the host) and, if kept and
 * host_x is non-NULL, its solution (n doubles).  A ticket is collected once. */
mg_status mg_server_poll(mg_server* s, uint64_t ticket, double* host_x, mg_stats* stats);
/* Collect the oldest finished request, waiting up to timeout_s seconds;
 * MG_ERR_BUSY if none finished in time. */
mg_status mg_server_next(mg_server* s, double timeout_s, uint64_t* ticket, double* host_x,
                         mg_stats* stats);
mg_status mg_server_info(mg_server* s, mg_server_info_t* info);
/* Finish every queued and running request, then free everything. */
mg_status mg_server_destroy(mg_server* s);

/* ---- BLAS level 1 (Sec. 6.1: axpy and the other vector-vector operations,
 * bound by memory bandwidth, as the basic architecture comparison) ----------
 * x, y: device vectors of n elements of dtype on ctx's device, 16-byte
 * aligned (may be NULL when n = 0), 0 <= n <= MG_BLAS_MAX_N.
 * mg_axpy: y = alpha x + y, one fused multiply-add per element (FP32:
 *   alpha rounded to FP32 first); x and y must not alias; asynchronous.
 * mg_dot: x . y, mg_norm2: ||x||_2; products and sums in FP64 in one fixed
 *   order (each thread over its elements in index order, then a fixed tree
 *   over the workgroup, then the tiles in the library's two-stage order), so
 *   a result depends only on the data.  Synchronous: waits for stream and
 *   writes *host_out.  They keep a reduction scratch in the context of about
 *   8 bytes per 1024 FP64 / 2048 FP32 elements plus 8 KiB, grown when a
 *   longer vector needs more and charged to the context budget
 *   (MG_ERR_NOMEM when it does not fit); calls on one context serialise. */
#define MG_BLAS_MAX_N ((int64_t)1 << 33)
mg_status mg_axpy(mg_context* ctx, mg_dtype dtype, int64_t n, double alpha, const void* x, void* y,
                  void* stream);
mg_status mg_dot(mg_context* ctx, mg_dtype dtype, int64_t n, const void* x, const void* y,
                 double* host_out, void* stream);
mg_status mg_norm2(mg_context* ctx, mg_dtype dtype, int64_t n, const void* x, double* host_out,
                   void* stream);
/* mg_dot for callers that cannot allocate device or pinned memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same x . y, the same bits as mg_dot, written to the
 * caller's device scalar dev_out[0] (8-byte aligned, on ctx's device)
 * asynchronously on stream; the call allocates nothing and never waits.
 * The tile partials live in one fixed device array of the library (1 MiB
 * per device that runs the call, held until the process ends), so n is at
 * most 2^27 (MG_F64) or 2^28 (MG_F32) elements: MG_ERR_INVALID above that.
 * Every call on one device shares that array, and the array keeps the last
 * call's partials: calls that may overlap on one device (other streams,
 * other threads) race and must be ordered by the caller.  Other arguments
 * and errors as for mg_dot. */
mg_status mg_dot_noalloc(mg_context* ctx, mg_dtype dtype, int64_t n, const void* x,
                         const void* y, double* dev_out, void* stream);

/* ---- four-band combination (Sec. 2.2: the shallow-water prediction step,
 * u_new = u + M1 v + M2 w + M3 u + M4 u + S(u), with four-band matrices) ----
 * u_new[p] = u[p] + sum_{i<m} sum_{k<4} band_i,k[p] v_i[p + offsets[4i+k]]
 *            (+ s[p] when s is not NULL),  p = 0..n-1,
 * where band k of term i is bands[i][k * band_stride + p] (band_stride >= n)
 * and neighbours outside [0, n) count as zero.  1 <= m <= 4; every offset in
 * (-n, n); v_i may repeat and may be u; u_new must not alias any input.
 * The terms are added after u in (i, k) order, each as one fused
 * multiply-add, the source last.  All pointers are device memory of dtype
 * on ctx's device (bands, offsets and v are host arrays of m pointers / 4m
 * ints).  Asynchronous on stream. */
mg_status mg_band4_combine(mg_context* ctx, mg_dtype dtype, int64_t n, int m,
                           const void* const* bands, int64_t band_stride, const int* offsets,
                           const void* const* v, const void* u, const void* s, void* u_new,
                           void* stream);

/* ---- single operators (asynchronous; for parity tests and benchmarks) -----
 * x, y, b, d: device vectors of the level's n elements in dtype. */
/* y = A x (Sec. 4.1/4.2 banded matrix-vector product). */
mg_status mg_spmv(const mg_hierarchy* h, int level, mg_dtype dtype, const void* x, void* y,
                  void* stream);
/* d = b - A x; if host_norm is non-NULL also ||d||_2 (accumulated in FP64,
 * deterministic order), which makes the call synchronous.  d may be NULL
 * when only the norm is wanted (Sec. 6.3.1: a norm of a residual built
 * from one banded product). */
mg_status mg_defect(const mg_hierarchy* h, int level, mg_dtype dtype, const void* b,
                    const void* x, void* d, double* host_norm, void* stream);
/* sweeps damped Jacobi steps x <- x + omega (b - A x) / diag(A) (Sec. 6.2),
 * out of place internally, result in x. */
mg_status mg_smooth(const mg_hierarchy* h, int level, mg_dtype dtype, const void* b, void* x,
                    int sweeps, double omega, void* stream);
/* One damped Jacobi sweep out of place, a single kernel launch:
 * x_out = x + omega (b - A x) / diag(A) (Sec. 6.2).  x_out must not alias x
 * or b. */
mg_status mg_jacobi(const mg_hierarchy* h, int level, mg_dtype dtype, const void* b,
                    const void* x, void* x_out, double omega, void* stream);
/* Fused pre-smoothing pass of a V(2,2) level (one kernel launch; Sec. 6.2):
 * x2 = two damped Jacobi sweeps starting from x (x_zero != 0: from a zero
 * iterate, x is not read) and b_c = P^T (b - A x2) on level-1 with the
 * coarse boundary set to 0.  level > coarse level; x2 must not alias x or b;
 * b_c has the n of level-1. */
mg_status mg_pre_smooth(const mg_hierarchy* h, int level, mg_dtype dtype, const void* b,
                        const void* x, int x_zero, double omega, void* x2, void* b_c,
                        void* stream);
/* Fused post-smoothing pass (one kernel launch): x_out = two damped Jacobi
 * sweeps starting from x + P x_c; if host_norm is non-NULL also
 * ||b - A x_out||_2 (FP64 accumulation; makes the call synchronous).
 * x_out must not alias x, x_c or b. */
mg_status mg_post_smooth(const mg_hierarchy* h, int level, mg_dtype dtype, const void* b,
                         const void* x, const void* x_c, double omega, void* x_out,
                         double* host_norm, void* stream);
/* b_c = P^T d_f with the coarse nodes on the Dirichlet sides set to 0; P is
 * bilinear interpolation in index space (weights 1, 1/2, 1/4).  The paper
 * names no transfer operators (Sec. 6.2 only says geometric multigrid): this
 * is the library's reading, the exact transpose of mg_prolong, which makes
 * P^T A_f P the coarse operator on uniform grids. */
mg_status mg_restrict(const mg_hierarchy* h, int fine_level, mg_dtype dtype, const void* d_f,
                      void* b_c, void* stream);
/* x_f += P x_c: bilinear interpolation in index space (the library's
 * reading, as for mg_restrict). */
mg_status mg_prolong(const mg_hierarchy* h, int fine_level, mg_dtype dtype, const void* x_c,
                     void* x_f, void* stream);
/* Direct solve on the coarsest level (FP64 Cholesky, cast in/out for F32):
 * interior unknowns from the factor, boundary x = b. */
mg_status mg_coarse_solve(const mg_hierarchy* h, mg_dtype dtype, const void* b, void* x,
                          void* stream);
/* One V(nu_pre, nu_post) cycle at `level` in place on x (levels below use the
 * hierarchy's own work vectors).  fused != 0 (V(2,2) only) runs each level
 * as two fused passes (two sweeps + defect + restriction; prolongation + two
 * sweeps) with bit-identical results to the unfused sequence of kernels. */
mg_status mg_vcycle(mg_hierarchy* h, int level, mg_dtype dtype, const void* b, void* x,
                    int nu_pre, int nu_post, double omega, int fused, void* stream);

#ifdef __cplusplus
}
#endif
#endif
