/* Runs every function of the oracle (oracle/mg_oracle.c) on small inputs,
 * boundary masks and degenerate sizes, for builds with
 * -fsanitize=address,undefined (tests/test_scheduler_cpu.py builds and runs
 * it): any out-of-bounds access, leak or undefined operation aborts.  The
 * numerical checks are loose here; the oracle's pins live in the Python
 * tests. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mg_oracle.h"

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);      \
            exit(1);                                                          \
        }                                                                     \
    } while (0)

static double urand(unsigned* s) {
    *s = *s * 1103515245u + 12345u;
    return ((*s >> 8) & 0xFFFF) / 65536.0;
}

static double* grid(int L, double a, unsigned seed) {
    int N = (1 << L) + 1;
    double h = 1.0 / (N - 1);
    double* xy = (double*)malloc(2 * (size_t)N * N * sizeof(double));
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            size_t p = (size_t)j * N + i;
            int in = i > 0 && j > 0 && i < N - 1 && j < N - 1;
            xy[2 * p] = i * h + (in ? (2 * urand(&seed) - 1) * a * h : 0.0);
            xy[2 * p + 1] = j * h + (in ? (2 * urand(&seed) - 1) * a * h : 0.0);
        }
    return xy;
}

static void level_ops(int L, int dmask) {
    int N = (1 << L) + 1;
    size_t n = (size_t)N * N;
    double* xy = grid(L, 0.2, 7u + L);
    double* bands = (double*)calloc(9 * n, sizeof(double));
    or_assemble_bc(N, xy, dmask, bands);
    double* b = (double*)calloc(n, sizeof(double));
    double* x = (double*)calloc(n, sizeof(double));
    double* y = (double*)calloc(n, sizeof(double));
    or_load_vector_bc(N, xy, 0, dmask, b);
    or_spmv(N, bands, b, y);
    or_defect(N, bands, b, x, y);
    or_jacobi(N, bands, b, x, y, 0.7);
    if (L >= 1) {
        int Nc = (N - 1) / 2 + 1;
        double* bc = (double*)calloc((size_t)Nc * Nc, sizeof(double));
        or_restrict_bc(N, y, bc, dmask);
        or_prolong_add(N, bc, x);
        float* bf = (float*)calloc(9 * n, sizeof(float));
        float* xf = (float*)calloc(n, sizeof(float));
        float* yf = (float*)calloc(n, sizeof(float));
        float* cf = (float*)calloc((size_t)Nc * Nc, sizeof(float));
        for (size_t k = 0; k < 9 * n; ++k) bf[k] = (float)bands[k];
        for (size_t p = 0; p < n; ++p) xf[p] = (float)b[p];
        or_spmv_f32(N, bf, xf, yf);
        or_jacobi_f32(N, bf, xf, xf, yf, 0.7f);
        or_restrict_f32_bc(N, yf, cf, dmask);
        or_prolong_add_f32(N, cf, yf);
        free(bc); free(bf); free(xf); free(yf); free(cf);
    }
    memset(x, 0, n * sizeof(double));
    int steps = or_cg(N, bands, b, x, 1e-10, 50);
    CHECK(steps >= 0 && steps <= 50);
    CHECK(isfinite(or_norm2(n, x)) && isfinite(or_dot(n, x, b)));
    if (dmask == OR_ALL_DIRICHLET) {
        CHECK(isfinite(or_l2_error_sinsin(N, xy, x)));
        CHECK(isfinite(or_l2_error(N, xy, x, 0)));
    }
    free(xy); free(bands); free(b); free(x); free(y);
}

static void solvers(int L, int Lc, int dmask, int coarse_cg) {
    int N = (1 << L) + 1;
    size_t n = (size_t)N * N;
    double* xy = grid(L, 0.15, 3u + L + dmask);
    or_hier* h = or_hier_create_bc(L, Lc, xy, dmask);
    CHECK(h != NULL);
    double* b = (double*)calloc(n, sizeof(double));
    double* x = (double*)calloc(n, sizeof(double));
    or_load_vector_bc(N, or_hier_coords(h, L), 1, dmask, b);
    or_opts o = {2, 2, 0.7, 1e-8, 60, 0, 1e-2, 8, coarse_cg, 1e-12, 400};
    or_stats st;
    CHECK(or_solve_fp64(h, b, x, &o, &st) == 0 && st.rel_res <= 1e-8);
    memset(x, 0, n * sizeof(double));
    CHECK(or_solve_mixed_emulated(h, b, x, &o, &st) == 0 && st.rel_res <= 1e-8);
    for (int p32 = 0; p32 < 2; ++p32) {
        memset(x, 0, n * sizeof(double));
        CHECK(or_solve_pcg(h, b, x, &o, p32, &st) == 0 && st.rel_res <= 1e-8);
    }
    or_vcycle(h, L, x, b, &o);
    CHECK(or_hier_N(h, Lc) == (1 << Lc) + 1 && or_hier_bands(h, L) != NULL);
    /* a zero right-hand side returns x = 0 at once */
    memset(b, 0, n * sizeof(double));
    CHECK(or_solve_fp64(h, b, x, &o, &st) == 0 && or_norm2(n, x) == 0.0);
    or_hier_destroy(h);
    free(xy); free(b); free(x);
}

static void blas_and_band4(void) {
    size_t n = 1000;
    double* x = (double*)malloc(n * sizeof(double));
    double* y = (double*)malloc(n * sizeof(double));
    for (size_t i = 0; i < n; ++i) x[i] = y[i] = (double)i;
    or_axpy(n, 2.0, x, y);
    CHECK(y[10] == 30.0);
    CHECK(or_dot(0, x, y) == 0.0 && or_norm2(0, x) == 0.0);
    double* bands[2];
    const double* bc[2];
    const double* v[2] = {x, y};
    int off[8] = {-(int)n + 1, -1, 1, (int)n - 1, -2, 2, -3, 3};
    for (int i = 0; i < 2; ++i) {
        bands[i] = (double*)malloc(4 * n * sizeof(double));
        for (size_t k = 0; k < 4 * n; ++k) bands[i][k] = 0.5;
        bc[i] = bands[i];
    }
    double* out = (double*)malloc(n * sizeof(double));
    or_band4_combine(n, 2, bc, n, off, v, x, NULL, out);
    or_band4_combine(n, 2, bc, n, off, v, x, y, out);
    CHECK(isfinite(out[0]) && isfinite(out[n - 1]));
    free(bands[0]); free(bands[1]); free(out); free(x); free(y);
    double xq[4] = {0, 1, 1.2, -0.1}, yq[4] = {0, 0.1, 1, 0.9}, K[16];
    or_element_stiffness(xq, yq, K);
    double A[9] = {4, 1, 0, 1, 4, 1, 0, 1, 4}, r[3] = {1, 2, 3};
    CHECK(or_cholesky(3, A) == 0);
    or_cholesky_solve(3, A, r);
    double B[4] = {1, 2, 2, 1};
    CHECK(or_cholesky(2, B) == -1);
}

int main(void) {
    for (int L = 1; L <= 5; ++L)
        for (int dmask = 1; dmask <= 15; dmask += 2) level_ops(L, dmask);
    level_ops(4, 4);
    level_ops(4, 8);
    int masks[4] = {15, 1, 5, 12};
    for (int m = 0; m < 4; ++m) {
        solvers(5, 1, masks[m], 0);
        solvers(5, 3, masks[m], 0);
        solvers(5, 2, masks[m], 1);
    }
    solvers(4, 4, 15, 0);
    CHECK(or_hier_create_bc(3, 1, NULL, 0) == NULL);
    CHECK(or_hier_create_bc(3, 4, NULL, 15) == NULL);
    blas_and_band4();
    printf("ALL PASS threads=%d\n", or_threads());
    return 0;
}
