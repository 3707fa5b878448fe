/*
 * mg_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the Q1 finite
 * element multigrid Poisson solver of HONEI (arXiv 0904.4152): the Poisson
 * problem of Sec. 2.1 (eq. 1) discretised with conforming bilinear Q1
 * elements on a tensor-product grid of the unit square, fully assembled into
 * a 9-band matrix (Sec. 2.1, Sec. 4.1 "banded matrices ... fixed positions"),
 * and solved by a geometric V-cycle with two damped Jacobi pre- and
 * post-smoothing steps (Sec. 6.2), either in FP64 or as an FP64 defect
 * correction around single-precision multigrid cycles (Sec. 6.2).
 *
 * Only tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library.  The GPU product path shares no code with it.
 *
 * Conventions (readings of points the paper leaves open):
 *   N = 2^L + 1 nodes per side, n = N*N, node (i,j) has index p = j*N + i.
 *   Band k (k = 0..8) stores A[p, p + off_k] at index p, with
 *   off_k = (k/3 - 1)*N + (k%3 - 1); band-major storage bands[k*n + p].
 *   Homogeneous Dirichlet on the sides in a mask dmask (bit 1: x = 0,
 *   bit 2: x = 1, bit 4: y = 0, bit 8: y = 1; 15 = the whole boundary, the
 *   default): their rows and columns are zeroed and the diagonal set to 1.
 *   The other sides carry the natural homogeneous Neumann condition (their
 *   rows are the assembled ones).
 *   Coarse levels are rediscretised on the fine coordinates sampled every
 *   2^(L-l) nodes; restriction is the transpose of bilinear index-space
 *   prolongation followed by zeroing the coarse boundary.
 */
#ifndef MG_ORACLE_H
#define MG_ORACLE_H
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element stiffness of one bilinear quadrilateral, 2x2 Gauss.  xq, yq: the
 * four corners counter-clockwise from (i,j); K: 4x4 row-major. */
void or_element_stiffness(const double* xq, const double* yq, double* K);

/* Assemble the 9 bands of the stiffness matrix on an N x N node grid with
 * coordinates xy (2*n, interleaved).  dirichlet != 0 applies the boundary
 * treatment described above.  bands: 9*n doubles. */
void or_assemble(int N, const double* xy, int dirichlet, double* bands);
/* The same with Dirichlet treatment on the sides in dmask only. */
#define OR_ALL_DIRICHLET 15
void or_assemble_bc(int N, const double* xy, int dmask, double* bands);

/* Load vector b_p = sum_e int_e f phi_p (3x3 Gauss).  fn 0: f = 2 pi^2
 * sin(pi x) sin(pi y); fn 1: f = 1.  dirichlet != 0 zeroes boundary nodes. */
void or_load_vector(int N, const double* xy, int fn, int dirichlet, double* b);
/* fn 2: f = 2 pi^2 cos(pi x) sin(pi y) (solution cos(pi x) sin(pi y), Neumann
 * on x = 0, 1); fn 3: f = pi^2/2 sin(pi x/2) sin(pi y/2) (solution
 * sin(pi x/2) sin(pi y/2), Neumann on x = 1 and y = 1).  Zero on the
 * Dirichlet sides in dmask. */
void or_load_vector_bc(int N, const double* xy, int fn, int dmask, double* b);

/* L2 error ||u - u_h|| against u = sin(pi x) sin(pi y), 5x5 Gauss. */
double or_l2_error_sinsin(int N, const double* xy, const double* u);
/* The same against the exact solution of load fn (0, 2 or 3 above). */
double or_l2_error(int N, const double* xy, const double* u, int fn);

/* Band operations (FP64). */
void or_spmv(int N, const double* bands, const double* x, double* y);
void or_defect(int N, const double* bands, const double* b, const double* x, double* d);
void or_jacobi(int N, const double* bands, const double* b, const double* x,
               double* x_out, double omega);
/* Restriction: b_c = P^T d_f, then (filter != 0) zero on the coarse boundary. */
void or_restrict(int Nf, const double* d_f, double* b_c, int filter);
/* The same, zeroing the coarse nodes on the Dirichlet sides in dmask. */
void or_restrict_bc(int Nf, const double* d_f, double* b_c, int dmask);
/* Prolongation with correction: x_f += P x_c. */
void or_prolong_add(int Nf, const double* x_c, double* x_f);
double or_norm2(size_t n, const double* v);
/* Host threads the element-wise loops use: 1 for the plain build, the
 * OpenMP thread count for a -fopenmp build (same results either way). */
int or_threads(void);

/* Dense Cholesky (lower, in place, row-major m x m); returns 0 or -1 if a
 * pivot is not positive. */
int or_cholesky(int m, double* A);
void or_cholesky_solve(int m, const double* Lf, double* b);
double or_dot(size_t n, const double* u, const double* v);
/* BLAS level 1 of Sec. 6.1: y = alpha x + y; u . v and ||v|| sum in index order. */
void or_axpy(size_t n, double alpha, const double* x, double* y);
/* Sec. 2.2 prediction step: out = u + sum_i M_i v_i (+ s), four bands each. */
void or_band4_combine(size_t n, int m, const double* const* bands, size_t bs, const int* off,
                      const double* const* v, const double* u, const double* s, double* out);
/* Unpreconditioned CG on one level's banded system, from the iterate in x,
 * until ||b - A x|| <= tol ||b|| (recurrence residual) or max_iter steps;
 * returns the steps taken. */
int or_cg(int N, const double* bands, const double* b, double* x, double tol, int max_iter);

/* Single-precision band operations used by the emulated mixed solver. */
void or_spmv_f32(int N, const float* bands, const float* x, float* y);
void or_jacobi_f32(int N, const float* bands, const float* b, const float* x,
                   float* x_out, float omega);
void or_restrict_f32(int Nf, const float* d_f, float* b_c);
void or_restrict_f32_bc(int Nf, const float* d_f, float* b_c, int dmask);
void or_prolong_add_f32(int Nf, const float* x_c, float* x_f);

/* ---- hierarchy and solvers ---- */
typedef struct or_hier or_hier;

typedef struct {
    int nu_pre, nu_post;
    double omega;
    double rel_tol;
    int max_cycles;        /* FP64: V-cycles; mixed: outer steps */
    int fixed_cycles;      /* > 0: run exactly this many (no stop test) */
    double inner_reduction;
    int inner_max_cycles;
    int coarse_cg;         /* 1: coarsest level by CG from zero (Sec. 6.2); 0: Cholesky */
    double coarse_tol;     /* CG: stop once ||r|| <= coarse_tol ||b|| */
    int coarse_max_iter;   /* CG: at most this many steps */
} or_opts;

typedef struct {
    int status;            /* 0 ok, 3 no convergence, 4 numeric */
    int cycles;            /* V-cycles (FP64) or total inner cycles (mixed) */
    int outer_steps;
    double bnorm;          /* ||b||_2 */
    double rel_res;        /* ||b - A x||_2 / ||b||_2 at exit */
    int n_hist;
    double res_hist[256];  /* relative residual after each cycle / outer step */
} or_stats;

or_hier* or_hier_create(int L, int Lc, const double* xy_fine);
/* The same with Dirichlet sides dmask (1..15; at least one side, else the
 * operator is singular). */
or_hier* or_hier_create_bc(int L, int Lc, const double* xy_fine, int dmask);
void or_hier_destroy(or_hier* h);
int or_hier_N(const or_hier* h, int l);
const double* or_hier_bands(const or_hier* h, int l);
const double* or_hier_coords(const or_hier* h, int l);
/* One V(nu_pre, nu_post) cycle at level l, in place on x. */
int or_vcycle(or_hier* h, int l, double* x, const double* b, const or_opts* o);
int or_solve_fp64(or_hier* h, const double* b, double* x, const or_opts* o, or_stats* st);
int or_solve_mixed_emulated(or_hier* h, const double* b, double* x, const or_opts* o,
                            or_stats* st);
/* CG preconditioned by one V-cycle from zero (FP64, or FP32 on the scaled
 * residual with precond32). */
int or_solve_pcg(or_hier* h, const double* b, double* x, const or_opts* o, int precond32,
                 or_stats* st);

#ifdef __cplusplus
}
#endif
#endif
