/*
 * mg_oracle.c -- TEST INFRASTRUCTURE ONLY (see mg_oracle.h).
 *
 * Plain FP64 loops, no blocking or fusion: every function follows the
 * definition it cites so that it can be checked against the paper by eye.
 * Built with -O2 -ffp-contract=off so that no multiply-add is fused.  The
 * plain build runs on one thread.  Built with -fopenmp, the loops whose
 * iterations write disjoint outputs (band products, sweeps, transfers, one
 * grid row or one node per iteration) are shared among the host's cores;
 * every sum stays a sequential loop, so each output is the same arithmetic
 * in the same order and the results are bitwise those of the plain build.
 */
#include "mg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int or_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static const double OR_PI = 3.14159265358979323846;

/* Band k <-> (di, dj) neighbour offset; Sec. 2.1: the tensor-product
 * numbering gives a band structure known a priori. */
static int band_di(int k) { return k % 3 - 1; }
static int band_dj(int k) { return k / 3 - 1; }

static int is_boundary(int N, int i, int j) {
    return i == 0 || j == 0 || i == N - 1 || j == N - 1;
}

/* Node (i,j) lies on a Dirichlet side: bit 1 x = 0 (i = 0), bit 2 x = 1
 * (i = N-1), bit 4 y = 0 (j = 0), bit 8 y = 1 (j = N-1).  The rest of the
 * boundary carries the natural homogeneous Neumann condition (Sec. 2.1:
 * Dirichlet and Neumann parts of the boundary): its rows are the assembled
 * ones. */
static int is_dirichlet(int N, int i, int j, int dmask) {
    return (i == 0 && (dmask & 1)) || (i == N - 1 && (dmask & 2)) || (j == 0 && (dmask & 4)) ||
           (j == N - 1 && (dmask & 8));
}

/* Reference square [-1,1]^2, corners counter-clockwise. */
static const double XI_A[4] = {-1.0, 1.0, 1.0, -1.0};
static const double ETA_A[4] = {-1.0, -1.0, 1.0, 1.0};

static double phi_ref(int a, double xi, double eta) {
    return 0.25 * (1.0 + XI_A[a] * xi) * (1.0 + ETA_A[a] * eta);
}
static double dphi_dxi(int a, double eta) { return 0.25 * XI_A[a] * (1.0 + ETA_A[a] * eta); }
static double dphi_deta(int a, double xi) { return 0.25 * ETA_A[a] * (1.0 + XI_A[a] * xi); }

/* Isoparametric bilinear map at (xi, eta): physical point, Jacobian
 * determinant and physical gradients of the four shape functions.  The
 * derivatives of the map are summed over corner coordinates taken relative
 * to the first corner (the shape-function derivatives sum to zero, so this
 * is the same map); it avoids cancelling O(1) coordinates to O(h) results. */
static void map_point(const double* xq, const double* yq, double xi, double eta,
                      double* px, double* py, double* detJ, double* gx, double* gy) {
    double x_xi = 0, x_eta = 0, y_xi = 0, y_eta = 0, x = 0, y = 0;
    for (int a = 0; a < 4; ++a) {
        double p = phi_ref(a, xi, eta);
        double dxi = dphi_dxi(a, eta), deta = dphi_deta(a, xi);
        x += p * xq[a];
        y += p * yq[a];
        x_xi += dxi * (xq[a] - xq[0]);
        x_eta += deta * (xq[a] - xq[0]);
        y_xi += dxi * (yq[a] - yq[0]);
        y_eta += deta * (yq[a] - yq[0]);
    }
    double det = x_xi * y_eta - x_eta * y_xi;
    if (px) *px = x;
    if (py) *py = y;
    *detJ = det;
    if (gx) {
        /* grad phi = J^{-T} (dphi/dxi, dphi/deta), J = [[x_xi, x_eta], [y_xi, y_eta]] */
        for (int a = 0; a < 4; ++a) {
            double dxi = dphi_dxi(a, eta), deta = dphi_deta(a, xi);
            gx[a] = (y_eta * dxi - y_xi * deta) / det;
            gy[a] = (-x_eta * dxi + x_xi * deta) / det;
        }
    }
}

/* Gauss-Legendre rules on [-1,1]. */
static void gauss_rule(int npt, double* pts, double* wts) {
    if (npt == 2) {
        double g = 1.0 / sqrt(3.0);
        pts[0] = -g; pts[1] = g; wts[0] = wts[1] = 1.0;
    } else if (npt == 3) {
        double g = sqrt(0.6);
        pts[0] = -g; pts[1] = 0.0; pts[2] = g;
        wts[0] = 5.0 / 9.0; wts[1] = 8.0 / 9.0; wts[2] = 5.0 / 9.0;
    } else { /* 5 */
        double a = sqrt(5.0 - 2.0 * sqrt(10.0 / 7.0)) / 3.0;
        double b = sqrt(5.0 + 2.0 * sqrt(10.0 / 7.0)) / 3.0;
        double wa = (322.0 + 13.0 * sqrt(70.0)) / 900.0;
        double wb = (322.0 - 13.0 * sqrt(70.0)) / 900.0;
        pts[0] = -b; pts[1] = -a; pts[2] = 0.0; pts[3] = a; pts[4] = b;
        wts[0] = wb; wts[1] = wa; wts[2] = 128.0 / 225.0; wts[3] = wa; wts[4] = wb;
    }
}

/* K_e[a][b] = sum_q w_q detJ_q grad phi_a . grad phi_b  (2x2 Gauss). */
void or_element_stiffness(const double* xq, const double* yq, double* K) {
    double pts[5], wts[5];
    gauss_rule(2, pts, wts);
    for (int a = 0; a < 16; ++a) K[a] = 0.0;
    for (int qj = 0; qj < 2; ++qj) {
        for (int qi = 0; qi < 2; ++qi) {
            double det, gx[4], gy[4];
            map_point(xq, yq, pts[qi], pts[qj], NULL, NULL, &det, gx, gy);
            double w = wts[qi] * wts[qj] * det;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    K[a * 4 + b] += w * (gx[a] * gx[b] + gy[a] * gy[b]);
        }
    }
}

/* Corner node indices and coordinates of element (i,j), counter-clockwise. */
static void element_nodes(int N, const double* xy, int i, int j, int* nodes, double* xq,
                          double* yq) {
    nodes[0] = j * N + i;
    nodes[1] = j * N + i + 1;
    nodes[2] = (j + 1) * N + i + 1;
    nodes[3] = (j + 1) * N + i;
    for (int a = 0; a < 4; ++a) {
        xq[a] = xy[2 * (size_t)nodes[a]];
        yq[a] = xy[2 * (size_t)nodes[a] + 1];
    }
}

/* Full assembly into the 9 bands (Sec. 2.1: the matrix is assembled fully
 * even on a simple grid).  Elements are visited lexicographically, j outer,
 * so A[p][q] and A[q][p] receive the same terms in the same order. */
void or_assemble(int N, const double* xy, int dirichlet, double* bands) {
    or_assemble_bc(N, xy, dirichlet ? OR_ALL_DIRICHLET : 0, bands);
}

void or_assemble_bc(int N, const double* xy, int dmask, double* bands) {
    size_t n = (size_t)N * N;
    memset(bands, 0, 9 * n * sizeof(double));
    for (int j = 0; j < N - 1; ++j) {
        for (int i = 0; i < N - 1; ++i) {
            int nodes[4];
            double xq[4], yq[4], K[16];
            element_nodes(N, xy, i, j, nodes, xq, yq);
            or_element_stiffness(xq, yq, K);
            for (int a = 0; a < 4; ++a) {
                int pa = nodes[a];
                for (int b = 0; b < 4; ++b) {
                    int pb = nodes[b];
                    int di = (pb % N) - (pa % N), dj = (pb / N) - (pa / N);
                    int k = (dj + 1) * 3 + (di + 1);
                    bands[(size_t)k * n + pa] += K[a * 4 + b];
                }
            }
        }
    }
    if (!dmask) return;
    for (int j = 0; j < N; ++j) {
        for (int i = 0; i < N; ++i) {
            size_t p = (size_t)j * N + i;
            if (is_dirichlet(N, i, j, dmask)) {
                for (int k = 0; k < 9; ++k) bands[(size_t)k * n + p] = 0.0;
                bands[4 * n + p] = 1.0;
            } else {
                for (int k = 0; k < 9; ++k) {
                    if (k == 4) continue;
                    if (is_dirichlet(N, i + band_di(k), j + band_dj(k), dmask))
                        bands[(size_t)k * n + p] = 0.0;
                }
            }
        }
    }
}

static double rhs_f(int fn, double x, double y) {
    if (fn == 1) return 1.0;
    if (fn == 2) return 2.0 * OR_PI * OR_PI * cos(OR_PI * x) * sin(OR_PI * y);
    if (fn == 3) return 0.5 * OR_PI * OR_PI * sin(0.5 * OR_PI * x) * sin(0.5 * OR_PI * y);
    return 2.0 * OR_PI * OR_PI * sin(OR_PI * x) * sin(OR_PI * y);
}

/* The exact solutions of the manufactured problems: -Laplace(u) = rhs_f. */
static double exact_u(int fn, double x, double y) {
    if (fn == 2) return cos(OR_PI * x) * sin(OR_PI * y);
    if (fn == 3) return sin(0.5 * OR_PI * x) * sin(0.5 * OR_PI * y);
    return sin(OR_PI * x) * sin(OR_PI * y);
}

void or_load_vector(int N, const double* xy, int fn, int dirichlet, double* b) {
    or_load_vector_bc(N, xy, fn, dirichlet ? OR_ALL_DIRICHLET : 0, b);
}

void or_load_vector_bc(int N, const double* xy, int fn, int dmask, double* b) {
    size_t n = (size_t)N * N;
    double pts[5], wts[5];
    gauss_rule(3, pts, wts);
    memset(b, 0, n * sizeof(double));
    for (int j = 0; j < N - 1; ++j) {
        for (int i = 0; i < N - 1; ++i) {
            int nodes[4];
            double xq[4], yq[4];
            element_nodes(N, xy, i, j, nodes, xq, yq);
            for (int qj = 0; qj < 3; ++qj) {
                for (int qi = 0; qi < 3; ++qi) {
                    double px, py, det;
                    map_point(xq, yq, pts[qi], pts[qj], &px, &py, &det, NULL, NULL);
                    double w = wts[qi] * wts[qj] * det * rhs_f(fn, px, py);
                    for (int a = 0; a < 4; ++a) b[nodes[a]] += w * phi_ref(a, pts[qi], pts[qj]);
                }
            }
        }
    }
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i)
            if (is_dirichlet(N, i, j, dmask)) b[(size_t)j * N + i] = 0.0;
}

/* Integral L2 norm of u - u_h (Sec. 6.2.1), u = sin(pi x) sin(pi y). */
double or_l2_error_sinsin(int N, const double* xy, const double* u) {
    return or_l2_error(N, xy, u, 0);
}

/* The same for the exact solution of manufactured problem fn. */
double or_l2_error(int N, const double* xy, const double* u, int fn) {
    double pts[5], wts[5], sum = 0.0;
    gauss_rule(5, pts, wts);
    for (int j = 0; j < N - 1; ++j) {
        for (int i = 0; i < N - 1; ++i) {
            int nodes[4];
            double xq[4], yq[4];
            element_nodes(N, xy, i, j, nodes, xq, yq);
            for (int qj = 0; qj < 5; ++qj) {
                for (int qi = 0; qi < 5; ++qi) {
                    double px, py, det;
                    map_point(xq, yq, pts[qi], pts[qj], &px, &py, &det, NULL, NULL);
                    double uh = 0.0;
                    for (int a = 0; a < 4; ++a) uh += u[nodes[a]] * phi_ref(a, pts[qi], pts[qj]);
                    double e = exact_u(fn, px, py) - uh;
                    sum += wts[qi] * wts[qj] * det * e * e;
                }
            }
        }
    }
    return sqrt(sum);
}

/* y_p = sum_k band_k[p] x[p + off_k]; neighbours outside the grid are
 * skipped (their band entries are zero). */
void or_spmv(int N, const double* bands, const double* x, double* y) {
    size_t n = (size_t)N * N;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < N; ++j) {
        for (int i = 0; i < N; ++i) {
            size_t p = (size_t)j * N + i;
            double s = 0.0;
            for (int k = 0; k < 9; ++k) {
                int ii = i + band_di(k), jj = j + band_dj(k);
                if (ii < 0 || jj < 0 || ii >= N || jj >= N) continue;
                s += bands[(size_t)k * n + p] * x[(size_t)jj * N + ii];
            }
            y[p] = s;
        }
    }
}

void or_defect(int N, const double* bands, const double* b, const double* x, double* d) {
    size_t n = (size_t)N * N;
    or_spmv(N, bands, x, d);
#pragma omp parallel for schedule(static)
    for (size_t p = 0; p < n; ++p) d[p] = b[p] - d[p];
}

/* Damped Jacobi (Sec. 6.2): x' = x + omega (b - A x) / a_pp, out of place. */
void or_jacobi(int N, const double* bands, const double* b, const double* x, double* x_out,
               double omega) {
    size_t n = (size_t)N * N;
    or_spmv(N, bands, x, x_out);
#pragma omp parallel for schedule(static)
    for (size_t p = 0; p < n; ++p)
        x_out[p] = x[p] + omega * (b[p] - x_out[p]) / bands[4 * n + p];
}

/* 1D bilinear interpolation weight between fine index f and coarse index c. */
static double w1d(int f, int c) {
    int d = f - 2 * c;
    if (d == 0) return 1.0;
    if (d == 1 || d == -1) return 0.5;
    return 0.0;
}

/* b_c[I,J] = sum_{fine (f,g)} P[(f,g),(I,J)] d_f[f,g]  (P^T), terms outside
 * the fine grid absent; then the coarse boundary is zeroed. */
void or_restrict(int Nf, const double* d_f, double* b_c, int filter) {
    or_restrict_bc(Nf, d_f, b_c, filter ? OR_ALL_DIRICHLET : 0);
}

/* The same with the coarse Dirichlet nodes of the sides in dmask zeroed. */
void or_restrict_bc(int Nf, const double* d_f, double* b_c, int dmask) {
    int Nc = (Nf - 1) / 2 + 1;
#pragma omp parallel for schedule(static)
    for (int J = 0; J < Nc; ++J) {
        for (int I = 0; I < Nc; ++I) {
            double s = 0.0;
            for (int g = 2 * J - 1; g <= 2 * J + 1; ++g) {
                for (int f = 2 * I - 1; f <= 2 * I + 1; ++f) {
                    if (f < 0 || g < 0 || f >= Nf || g >= Nf) continue;
                    s += w1d(f, I) * w1d(g, J) * d_f[(size_t)g * Nf + f];
                }
            }
            if (is_dirichlet(Nc, I, J, dmask)) s = 0.0;
            b_c[(size_t)J * Nc + I] = s;
        }
    }
}

/* x_f[f,g] += sum_{(I,J)} P[(f,g),(I,J)] x_c[I,J]  (bilinear in index space). */
void or_prolong_add(int Nf, const double* x_c, double* x_f) {
    int Nc = (Nf - 1) / 2 + 1;
#pragma omp parallel for schedule(static)
    for (int g = 0; g < Nf; ++g) {
        for (int f = 0; f < Nf; ++f) {
            double s = 0.0;
            for (int J = (g - 1) / 2; J <= (g + 1) / 2; ++J) {
                for (int I = (f - 1) / 2; I <= (f + 1) / 2; ++I) {
                    if (I < 0 || J < 0 || I >= Nc || J >= Nc) continue;
                    s += w1d(f, I) * w1d(g, J) * x_c[(size_t)J * Nc + I];
                }
            }
            x_f[(size_t)g * Nf + f] += s;
        }
    }
}

double or_norm2(size_t n, const double* v) {
    double s = 0.0;
    for (size_t p = 0; p < n; ++p) s += v[p] * v[p];
    return sqrt(s);
}

int or_cholesky(int m, double* A) {
    for (int c = 0; c < m; ++c) {
        double s = A[(size_t)c * m + c];
        for (int k = 0; k < c; ++k) s -= A[(size_t)c * m + k] * A[(size_t)c * m + k];
        if (!(s > 0.0)) return -1;
        double d = sqrt(s);
        A[(size_t)c * m + c] = d;
        for (int r = c + 1; r < m; ++r) {
            double t = A[(size_t)r * m + c];
            for (int k = 0; k < c; ++k) t -= A[(size_t)r * m + k] * A[(size_t)c * m + k];
            A[(size_t)r * m + c] = t / d;
        }
        for (int r = 0; r < c; ++r) A[(size_t)r * m + c] = 0.0;
    }
    return 0;
}

void or_cholesky_solve(int m, const double* Lf, double* b) {
    for (int r = 0; r < m; ++r) {
        double s = b[r];
        for (int k = 0; k < r; ++k) s -= Lf[(size_t)r * m + k] * b[k];
        b[r] = s / Lf[(size_t)r * m + r];
    }
    for (int r = m - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < m; ++k) s -= Lf[(size_t)k * m + r] * b[k];
        b[r] = s / Lf[(size_t)r * m + r];
    }
}

/* u_new = u + sum_i M_i v_i (+ s) with four-band M_i (Sec. 2.2 prediction
 * step): band k of term i holds M_i[p][p + off[4i+k]] at bands[i][k*bs + p];
 * neighbours outside [0, n) are absent. */
void or_band4_combine(size_t n, int m, const double* const* bands, size_t bs, const int* off,
                      const double* const* v, const double* u, const double* s, double* out) {
    for (size_t p = 0; p < n; ++p) {
        double acc = u[p];
        for (int i = 0; i < m; ++i)
            for (int k = 0; k < 4; ++k) {
                long long q = (long long)p + off[4 * i + k];
                if (q < 0 || q >= (long long)n) continue;
                acc += bands[i][(size_t)k * bs + p] * v[i][q];
            }
        if (s) acc += s[p];
        out[p] = acc;
    }
}

/* y = alpha x + y (Sec. 6.1 axpy), in index order. */
void or_axpy(size_t n, double alpha, const double* x, double* y) {
    for (size_t p = 0; p < n; ++p) y[p] = alpha * x[p] + y[p];
}

double or_dot(size_t n, const double* u, const double* v) {
    double s = 0.0;
    for (size_t p = 0; p < n; ++p) s += u[p] * v[p];
    return s;
}

/* Unpreconditioned conjugate gradients (Hestenes and Stiefel), the coarse
 * grid solver of Sec. 6.2, on the full banded system of one level: from the
 * iterate in x, r = b - A x, p = r; each step q = A p, alpha = (r.r)/(p.q),
 * x += alpha p, r -= alpha q, beta = (r'.r')/(r.r), p = r' + beta p.  Stops
 * before a step once ||r|| <= tol ||b|| or after max_iter steps.  Dirichlet
 * rows (identity, zero right-hand side) stay at zero from a zero start.
 * Returns the number of steps taken. */
int or_cg(int N, const double* bands, const double* b, double* x, double tol, int max_iter) {
    size_t n = (size_t)N * N;
    double* r = (double*)malloc(n * sizeof(double));
    double* p = (double*)malloc(n * sizeof(double));
    double* q = (double*)malloc(n * sizeof(double));
    or_defect(N, bands, b, x, r);
    memcpy(p, r, n * sizeof(double));
    double rr = or_dot(n, r, r);
    double stop = tol * or_norm2(n, b);
    int k = 0;
    while (k < max_iter && sqrt(rr) > stop) {
        or_spmv(N, bands, p, q);
        double alpha = rr / or_dot(n, p, q);
        for (size_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (size_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        double rr_new = or_dot(n, r, r);
        double beta = rr_new / rr;
        for (size_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        ++k;
    }
    free(r); free(p); free(q);
    return k;
}

/* ---- single precision band operations (emulated FP32 inner cycles) ---- */
void or_spmv_f32(int N, const float* bands, const float* x, float* y) {
    size_t n = (size_t)N * N;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < N; ++j) {
        for (int i = 0; i < N; ++i) {
            size_t p = (size_t)j * N + i;
            float s = 0.0f;
            for (int k = 0; k < 9; ++k) {
                int ii = i + band_di(k), jj = j + band_dj(k);
                if (ii < 0 || jj < 0 || ii >= N || jj >= N) continue;
                s += bands[(size_t)k * n + p] * x[(size_t)jj * N + ii];
            }
            y[p] = s;
        }
    }
}

void or_jacobi_f32(int N, const float* bands, const float* b, const float* x, float* x_out,
                   float omega) {
    size_t n = (size_t)N * N;
    or_spmv_f32(N, bands, x, x_out);
#pragma omp parallel for schedule(static)
    for (size_t p = 0; p < n; ++p)
        x_out[p] = x[p] + omega * (b[p] - x_out[p]) / bands[4 * n + p];
}

void or_restrict_f32(int Nf, const float* d_f, float* b_c) {
    or_restrict_f32_bc(Nf, d_f, b_c, OR_ALL_DIRICHLET);
}

void or_restrict_f32_bc(int Nf, const float* d_f, float* b_c, int dmask) {
    int Nc = (Nf - 1) / 2 + 1;
#pragma omp parallel for schedule(static)
    for (int J = 0; J < Nc; ++J) {
        for (int I = 0; I < Nc; ++I) {
            float s = 0.0f;
            if (!is_dirichlet(Nc, I, J, dmask)) {
                for (int g = 2 * J - 1; g <= 2 * J + 1; ++g)
                    for (int f = 2 * I - 1; f <= 2 * I + 1; ++f) {
                        if (f < 0 || g < 0 || f >= Nf || g >= Nf) continue;
                        s += (float)(w1d(f, I) * w1d(g, J)) * d_f[(size_t)g * Nf + f];
                    }
            }
            b_c[(size_t)J * Nc + I] = s;
        }
    }
}

void or_prolong_add_f32(int Nf, const float* x_c, float* x_f) {
    int Nc = (Nf - 1) / 2 + 1;
#pragma omp parallel for schedule(static)
    for (int g = 0; g < Nf; ++g) {
        for (int f = 0; f < Nf; ++f) {
            float s = 0.0f;
            for (int J = (g - 1) / 2; J <= (g + 1) / 2; ++J)
                for (int I = (f - 1) / 2; I <= (f + 1) / 2; ++I) {
                    if (I < 0 || J < 0 || I >= Nc || J >= Nc) continue;
                    s += (float)(w1d(f, I) * w1d(g, J)) * x_c[(size_t)J * Nc + I];
                }
            x_f[(size_t)g * Nf + f] += s;
        }
    }
}

/* ---- hierarchy ---- */
#define OR_MAXL 16

struct or_hier {
    int L, Lc;
    int N[OR_MAXL + 1];
    double* xy[OR_MAXL + 1];
    double* bands[OR_MAXL + 1];
    float* bands32[OR_MAXL + 1];
    double *x[OR_MAXL + 1], *b[OR_MAXL + 1], *t[OR_MAXL + 1];
    float *x32[OR_MAXL + 1], *b32[OR_MAXL + 1], *t32[OR_MAXL + 1];
    int dmask;      /* Dirichlet sides */
    int m;          /* unknowns at Lc: the nodes not on a Dirichlet side */
    int* cnode;     /* m node indices of the unknowns, in index order */
    double* chol;   /* m x m lower Cholesky factor of their block */
    double* cwork;  /* m */
};

or_hier* or_hier_create(int L, int Lc, const double* xy_fine) {
    return or_hier_create_bc(L, Lc, xy_fine, OR_ALL_DIRICHLET);
}

or_hier* or_hier_create_bc(int L, int Lc, const double* xy_fine, int dmask) {
    if (L < 1 || L > OR_MAXL || Lc < 1 || Lc > L || dmask <= 0 || dmask > OR_ALL_DIRICHLET)
        return NULL;
    or_hier* h = (or_hier*)calloc(1, sizeof(or_hier));
    h->L = L;
    h->Lc = Lc;
    h->dmask = dmask;
    int Nf = (1 << L) + 1;
    for (int l = Lc; l <= L; ++l) {
        int N = (1 << l) + 1, s = 1 << (L - l);
        size_t n = (size_t)N * N;
        h->N[l] = N;
        h->xy[l] = (double*)malloc(2 * n * sizeof(double));
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                size_t pf = (size_t)(j * s) * Nf + (size_t)(i * s);
                h->xy[l][2 * ((size_t)j * N + i)] = xy_fine[2 * pf];
                h->xy[l][2 * ((size_t)j * N + i) + 1] = xy_fine[2 * pf + 1];
            }
        h->bands[l] = (double*)malloc(9 * n * sizeof(double));
        or_assemble_bc(N, h->xy[l], dmask, h->bands[l]);
        h->bands32[l] = (float*)malloc(9 * n * sizeof(float));
        for (size_t q = 0; q < 9 * n; ++q) h->bands32[l][q] = (float)h->bands[l][q];
        h->x[l] = (double*)calloc(n, sizeof(double));
        h->b[l] = (double*)calloc(n, sizeof(double));
        h->t[l] = (double*)calloc(n, sizeof(double));
        h->x32[l] = (float*)calloc(n, sizeof(float));
        h->b32[l] = (float*)calloc(n, sizeof(float));
        h->t32[l] = (float*)calloc(n, sizeof(float));
    }
    /* Coarse-grid direct solver (replaces the paper's unpreconditioned CG
     * of Sec. 6.2 by an exact dense factorisation of the interior block). */
    int Nc = h->N[Lc];
    size_t nc = (size_t)Nc * Nc;
    int* col = (int*)malloc(nc * sizeof(int));  /* node -> unknown, or -1 */
    h->cnode = (int*)malloc(nc * sizeof(int));
    h->m = 0;
    for (int j = 0; j < Nc; ++j)
        for (int i = 0; i < Nc; ++i) {
            size_t p = (size_t)j * Nc + i;
            col[p] = -1;
            if (!is_dirichlet(Nc, i, j, dmask)) {
                col[p] = h->m;
                h->cnode[h->m++] = (int)p;
            }
        }
    h->chol = (double*)calloc((size_t)h->m * h->m, sizeof(double));
    h->cwork = (double*)calloc((size_t)h->m, sizeof(double));
    for (int r = 0; r < h->m; ++r) {
        int p = h->cnode[r], i = p % Nc, j = p / Nc;
        for (int k = 0; k < 9; ++k) {
            int ii = i + band_di(k), jj = j + band_dj(k);
            if (ii < 0 || jj < 0 || ii >= Nc || jj >= Nc) continue;
            int c = col[jj * Nc + ii];
            if (c < 0) continue;
            h->chol[(size_t)r * h->m + c] = h->bands[Lc][(size_t)k * nc + p];
        }
    }
    free(col);
    if (or_cholesky(h->m, h->chol) != 0) {
        or_hier_destroy(h);
        return NULL;
    }
    return h;
}

void or_hier_destroy(or_hier* h) {
    if (!h) return;
    for (int l = h->Lc; l <= h->L; ++l) {
        free(h->xy[l]); free(h->bands[l]); free(h->bands32[l]);
        free(h->x[l]); free(h->b[l]); free(h->t[l]);
        free(h->x32[l]); free(h->b32[l]); free(h->t32[l]);
    }
    free(h->chol);
    free(h->cwork);
    free(h->cnode);
    free(h);
}

int or_hier_N(const or_hier* h, int l) { return h->N[l]; }
const double* or_hier_bands(const or_hier* h, int l) { return h->bands[l]; }
const double* or_hier_coords(const or_hier* h, int l) { return h->xy[l]; }

/* Solve at the coarsest level: with o->coarse_cg by CG from a zero iterate
 * (Sec. 6.2), else directly: the unknowns by Cholesky, Dirichlet rows are
 * identity rows. */
static void coarse_solve(or_hier* h, double* x, const double* b, const or_opts* o) {
    int Nc = h->N[h->Lc];
    if (o->coarse_cg) {
        memset(x, 0, (size_t)Nc * Nc * sizeof(double));
        or_cg(Nc, h->bands[h->Lc], b, x, o->coarse_tol, o->coarse_max_iter);
        return;
    }
    for (int j = 0; j < Nc; ++j)
        for (int i = 0; i < Nc; ++i)
            if (is_dirichlet(Nc, i, j, h->dmask)) x[(size_t)j * Nc + i] = b[(size_t)j * Nc + i];
    for (int r = 0; r < h->m; ++r) h->cwork[r] = b[h->cnode[r]];
    or_cholesky_solve(h->m, h->chol, h->cwork);
    for (int r = 0; r < h->m; ++r) x[h->cnode[r]] = h->cwork[r];
}

/* V(nu_pre, nu_post) cycle (Sec. 6.2): smooth, restrict the defect, recurse
 * with a zero initial guess, prolongate and correct, smooth. */
int or_vcycle(or_hier* h, int l, double* x, const double* b, const or_opts* o) {
    int N = h->N[l];
    size_t n = (size_t)N * N;
    if (l == h->Lc) {
        coarse_solve(h, x, b, o);
        return 0;
    }
    double* t = h->t[l];
    for (int s = 0; s < o->nu_pre; ++s) {
        or_jacobi(N, h->bands[l], b, x, t, o->omega);
        memcpy(x, t, n * sizeof(double));
    }
    or_defect(N, h->bands[l], b, x, t);
    or_restrict_bc(N, t, h->b[l - 1], h->dmask);
    size_t nc = (size_t)h->N[l - 1] * h->N[l - 1];
    memset(h->x[l - 1], 0, nc * sizeof(double));
    or_vcycle(h, l - 1, h->x[l - 1], h->b[l - 1], o);
    or_prolong_add(N, h->x[l - 1], x);
    for (int s = 0; s < o->nu_post; ++s) {
        or_jacobi(N, h->bands[l], b, x, t, o->omega);
        memcpy(x, t, n * sizeof(double));
    }
    return 0;
}

static double residual_norm(or_hier* h, const double* b, const double* x) {
    int N = h->N[h->L];
    size_t n = (size_t)N * N;
    double* d = (double*)malloc(n * sizeof(double));
    or_defect(N, h->bands[h->L], b, x, d);
    double r = or_norm2(n, d);
    free(d);
    return r;
}

/* Relative-residual stopping: ||b - A x|| <= tol ||b|| (the paper is silent;
 * the norm is Euclidean over all n entries). */
int or_solve_fp64(or_hier* h, const double* b, double* x, const or_opts* o, or_stats* st) {
    int N = h->N[h->L];
    size_t n = (size_t)N * N;
    memset(st, 0, sizeof(*st));
    double bn = or_norm2(n, b);
    st->bnorm = bn;
    if (bn == 0.0) {
        memset(x, 0, n * sizeof(double));
        return 0;
    }
    double r = residual_norm(h, b, x);
    st->rel_res = r / bn;
    for (int k = 1;; ++k) {
        if (o->fixed_cycles > 0) {
            if (k > o->fixed_cycles) break;
        } else {
            if (r <= o->rel_tol * bn) break;
            if (k > o->max_cycles) { st->status = 3; break; }
        }
        or_vcycle(h, h->L, x, b, o);
        r = residual_norm(h, b, x);
        st->cycles = k;
        st->rel_res = r / bn;
        if (st->n_hist < 256) st->res_hist[st->n_hist++] = r / bn;
        if (!(r == r) || r > 1e3 * bn) { st->status = 4; break; }
    }
    return st->status;
}

/* Single precision V-cycle with the coarse solve done in FP64. */
static void vcycle32(or_hier* h, int l, float* x, const float* b, const or_opts* o) {
    int N = h->N[l];
    size_t n = (size_t)N * N;
    if (l == h->Lc) {
        double* bd = h->b[l];
        double* xd = h->x[l];
        for (size_t p = 0; p < n; ++p) bd[p] = (double)b[p];
        coarse_solve(h, xd, bd, o);
        for (size_t p = 0; p < n; ++p) x[p] = (float)xd[p];
        return;
    }
    float* t = h->t32[l];
    float om = (float)o->omega;
    for (int s = 0; s < o->nu_pre; ++s) {
        or_jacobi_f32(N, h->bands32[l], b, x, t, om);
        memcpy(x, t, n * sizeof(float));
    }
    or_spmv_f32(N, h->bands32[l], x, t);
    for (size_t p = 0; p < n; ++p) t[p] = b[p] - t[p];
    or_restrict_f32_bc(N, t, h->b32[l - 1], h->dmask);
    size_t nc = (size_t)h->N[l - 1] * h->N[l - 1];
    memset(h->x32[l - 1], 0, nc * sizeof(float));
    vcycle32(h, l - 1, h->x32[l - 1], h->b32[l - 1], o);
    or_prolong_add_f32(N, h->x32[l - 1], x);
    for (int s = 0; s < o->nu_post; ++s) {
        or_jacobi_f32(N, h->bands32[l], b, x, t, om);
        memcpy(x, t, n * sizeof(float));
    }
}

static double norm_f32_in_f64(size_t n, const float* v) {
    double s = 0.0;
    for (size_t p = 0; p < n; ++p) s += (double)v[p] * (double)v[p];
    return sqrt(s);
}

/* The power of two that brings the defects into single-precision range
 * (the paper does not say how; a power of two scales exactly in binary
 * arithmetic, so the single-precision cycles compute the same digits for
 * any exponent): 2^-e for ||b|| = m 2^e, m in [0.5, 1), e clamped to
 * [-1020, 1020]. */
static int pow2_exponent(double v) {
    int e = 0;
    (void)frexp(v, &e);
    return e < -1020 ? -1020 : (e > 1020 ? 1020 : e);
}

/* Mixed precision defect correction (Sec. 6.2): FP64 defect d = b - A x,
 * single-precision multigrid cycles on d scaled by sc = 2^-e (e from
 * ||b||, pow2_exponent) until the FP32 residual has dropped by
 * inner_reduction relative to the scaled defect's norm sc ||d||, FP64
 * update x += 2^e c. */
int or_solve_mixed_emulated(or_hier* h, const double* b, double* x, const or_opts* o,
                            or_stats* st) {
    int N = h->N[h->L];
    size_t n = (size_t)N * N;
    memset(st, 0, sizeof(*st));
    double bn = or_norm2(n, b);
    st->bnorm = bn;
    if (bn == 0.0) {
        memset(x, 0, n * sizeof(double));
        return 0;
    }
    const double sc = ldexp(1.0, -pow2_exponent(bn));
    const double unscale = ldexp(1.0, pow2_exponent(bn));
    double* d = (double*)malloc(n * sizeof(double));
    float* d32 = (float*)malloc(n * sizeof(float));
    float* c32 = (float*)malloc(n * sizeof(float));
    float* r32 = (float*)malloc(n * sizeof(float));
    for (int k = 1;; ++k) {
        or_defect(N, h->bands[h->L], b, x, d);
        double s = or_norm2(n, d);
        st->rel_res = s / bn;
        if (k > 1 && st->n_hist < 256) st->res_hist[st->n_hist++] = s / bn;
        if (!(s == s) || s > 1e3 * bn) { st->status = 4; break; }
        if (o->fixed_cycles > 0) {
            if (k > o->fixed_cycles) break;
        } else {
            if (s <= o->rel_tol * bn) break;
            if (k > o->max_cycles) { st->status = 3; break; }
        }
        if (s == 0.0) break;
        for (size_t p = 0; p < n; ++p) d32[p] = (float)(d[p] * sc);
        memset(c32, 0, n * sizeof(float));
        const double dn = sc * s;
        for (int it = 1; it <= o->inner_max_cycles; ++it) {
            vcycle32(h, h->L, c32, d32, o);
            st->cycles++;
            or_spmv_f32(N, h->bands32[h->L], c32, r32);
            for (size_t p = 0; p < n; ++p) r32[p] = d32[p] - r32[p];
            if (norm_f32_in_f64(n, r32) <= o->inner_reduction * dn) break;
        }
        for (size_t p = 0; p < n; ++p) x[p] += unscale * (double)c32[p];
        st->outer_steps = k;
    }
    free(d); free(d32); free(c32); free(r32);
    return st->status;
}

/* z = M r with M one V-cycle from a zero iterate: in FP64, or with
 * precond32 in single precision on r / ||r|| scaled back (the FP32 cycle of
 * the mixed scheme used as a preconditioner). */
static void precondition(or_hier* h, const double* r, double* z, const or_opts* o, int precond32,
                         float* r32, float* z32) {
    int N = h->N[h->L];
    size_t n = (size_t)N * N;
    if (!precond32) {
        memset(z, 0, n * sizeof(double));
        or_vcycle(h, h->L, z, r, o);
        return;
    }
    double s = or_norm2(n, r);
    if (s == 0.0) {
        memset(z, 0, n * sizeof(double));
        return;
    }
    for (size_t p = 0; p < n; ++p) r32[p] = (float)(r[p] / s);
    memset(z32, 0, n * sizeof(float));
    vcycle32(h, h->L, z32, r32, o);
    for (size_t p = 0; p < n; ++p) z[p] = s * (double)z32[p];
}

/* Conjugate gradients preconditioned by one multigrid cycle (Sec. 4.1: a
 * solver plugged into another as its preconditioner; the cycle of Sec. 6.2).  From
 * x: r = b - A x, z = M r, p = z; each step q = A p,
 * alpha = (r.z)/(p.q), x += alpha p, r -= alpha q, stop once
 * ||r|| <= rel_tol ||b|| (r updated by the recurrence), z' = M r',
 * beta = (r'.z')/(r.z), p = z' + beta p.  stats: cycles = steps (one
 * preconditioner cycle each), res_hist the recurrence residual after each
 * step, rel_res the true residual at exit. */
int or_solve_pcg(or_hier* h, const double* b, double* x, const or_opts* o, int precond32,
                 or_stats* st) {
    int N = h->N[h->L];
    size_t n = (size_t)N * N;
    memset(st, 0, sizeof(*st));
    double bn = or_norm2(n, b);
    st->bnorm = bn;
    if (bn == 0.0) {
        memset(x, 0, n * sizeof(double));
        return 0;
    }
    double* r = (double*)malloc(n * sizeof(double));
    double* z = (double*)malloc(n * sizeof(double));
    double* p = (double*)malloc(n * sizeof(double));
    double* q = (double*)malloc(n * sizeof(double));
    float* r32 = (float*)malloc(n * sizeof(float));
    float* z32 = (float*)malloc(n * sizeof(float));
    or_defect(N, h->bands[h->L], b, x, r);
    double rn = or_norm2(n, r);
    precondition(h, r, z, o, precond32, r32, z32);
    memcpy(p, z, n * sizeof(double));
    double rz = or_dot(n, r, z);
    for (int k = 1;; ++k) {
        if (o->fixed_cycles > 0) {
            if (k > o->fixed_cycles) break;
        } else {
            if (rn <= o->rel_tol * bn) break;
            if (k > o->max_cycles) { st->status = 3; break; }
        }
        or_spmv(N, h->bands[h->L], p, q);
        double alpha = rz / or_dot(n, p, q);
        for (size_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (size_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        rn = or_norm2(n, r);
        st->cycles = k;
        if (st->n_hist < 256) st->res_hist[st->n_hist++] = rn / bn;
        if (!(rn == rn) || rn > 1e3 * bn) { st->status = 4; break; }
        precondition(h, r, z, o, precond32, r32, z32);
        double rz_new = or_dot(n, r, z);
        double beta = rz_new / rz;
        for (size_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rz = rz_new;
    }
    st->rel_res = residual_norm(h, b, x) / bn;
    free(r); free(z); free(p); free(q); free(r32); free(z32);
    return st->status;
}
