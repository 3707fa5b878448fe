"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test targets a mistake the oracle could plausibly contain (a dropped
quadrature term, a transposed Jacobian, a wrong band index or weight, a
missing boundary treatment) and checks something that does not come from the
oracle itself: closed forms, exact invariants of the Q1 discretisation,
independent library routines (scipy sparse products, dense LAPACK solves) and
the behaviour the paper reports in Table 1 (Sec. 6.2.1).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth

# ---------------------------------------------------------------- helpers


def band_offsets(N):
    return [(k // 3 - 1) * N + (k % 3 - 1) for k in range(9)]


def bands_to_csr(N, bands):
    """Sparse matrix from the band storage, built by scipy (independent of
    the oracle's own band product)."""
    n = N * N
    rows, cols, vals = [], [], []
    ii = np.tile(np.arange(N), N)
    jj = np.repeat(np.arange(N), N)
    for k in range(9):
        di, dj = k % 3 - 1, k // 3 - 1
        ok = (ii + di >= 0) & (ii + di < N) & (jj + dj >= 0) & (jj + dj < N)
        p = np.nonzero(ok)[0]
        rows.append(p)
        cols.append(p + dj * N + di)
        vals.append(bands[k][p])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def shoelace(xq, yq):
    return 0.5 * sum(xq[a] * yq[(a + 1) % 4] - xq[(a + 1) % 4] * yq[a] for a in range(4))


# ---------------------------------------------------------------- element


def test_rectangle_element_matches_tensor_product(orc):
    """K_e on an hx x hy rectangle = Sx (x) My + Mx (x) Sy of 1D linear
    elements (closed form); catches quadrature-weight and Jacobian errors."""
    hx, hy = 0.3, 0.7
    S = lambda h: np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    M = lambda h: np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    corners = [(0, 0), (1, 0), (1, 1), (0, 1)]  # counter-clockwise (ax, ay)
    K_ref = np.zeros((4, 4))
    for a, (ax, ay) in enumerate(corners):
        for b, (bx, by) in enumerate(corners):
            K_ref[a, b] = S(hx)[ax, bx] * M(hy)[ay, by] + M(hx)[ax, bx] * S(hy)[ay, by]
    x0, y0 = 0.25, -0.4
    K = orc.element_stiffness([x0, x0 + hx, x0 + hx, x0], [y0, y0, y0 + hy, y0 + hy])
    np.testing.assert_allclose(K, K_ref, rtol=0, atol=1e-14)


def test_unit_square_element_textbook(orc):
    K = orc.element_stiffness([0, 1, 1, 0], [0, 0, 1, 1])
    ref = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0
    np.testing.assert_allclose(K, ref, atol=1e-15)


@pytest.mark.parametrize("quad", [
    ([0.0, 1.0, 1.3, 0.2], [0.0, 0.1, 0.9, 1.1]),     # general convex quad
    ([0.0, 2.0, 2.5, 0.5], [0.0, 0.0, 1.0, 1.0]),     # parallelogram (sheared)
    ([0.1, 0.35, 0.3, 0.05], [0.2, 0.22, 0.47, 0.41]),
])
def test_element_energy_of_linears_is_area(orc, quad):
    """For any convex quad, x^T K x = y^T K y = area (shoelace), x^T K y = 0
    and K 1 = 0: Q1 reproduces linear functions and 2x2 Gauss integrates
    det J exactly.  A transposed J^{-1} or a wrong det J fails this."""
    xq, yq = np.array(quad[0]), np.array(quad[1])
    K = orc.element_stiffness(xq, yq)
    area = shoelace(xq, yq)
    assert area > 0
    assert abs(xq @ K @ xq - area) < 1e-14
    assert abs(yq @ K @ yq - area) < 1e-14
    assert abs(xq @ K @ yq) < 1e-14
    np.testing.assert_allclose(K @ np.ones(4), 0, atol=1e-14)
    np.testing.assert_array_equal(K, K.T)


def test_element_rotation_translation_invariant(orc):
    xq, yq = np.array([0.0, 1.0, 1.3, 0.2]), np.array([0.0, 0.1, 0.9, 1.1])
    K = orc.element_stiffness(xq, yq)
    th = 0.7
    c, s = np.cos(th), np.sin(th)
    xr, yr = c * xq - s * yq + 3.0, s * xq + c * yq - 1.0
    np.testing.assert_allclose(orc.element_stiffness(xr, yr), K, atol=1e-13)


# ---------------------------------------------------------------- assembly


@pytest.mark.parametrize("L", [2, 3, 5])
def test_uniform_interior_stencil_is_textbook_q1(orc, L):
    """Uniform grid, interior row = (1/3)[-1 -1 -1; -1 8 -1; -1 -1 -1] for
    every h (the 2D Q1 Laplacian is h-independent)."""
    N = synth.grid_size(L)
    bands = orc.assemble(N, synth.coords(L), dirichlet=False)
    ref = np.array([-1, -1, -1, -1, 8, -1, -1, -1, -1]) / 3.0
    ii = np.tile(np.arange(N), N)
    jj = np.repeat(np.arange(N), N)
    interior = (ii > 0) & (jj > 0) & (ii < N - 1) & (jj < N - 1)
    for k in range(9):
        np.testing.assert_allclose(bands[k][interior], ref[k], rtol=0, atol=1e-14)


@pytest.mark.parametrize("L,a", [(3, 0.2), (4, 0.25), (5, 0.2)])
def test_patch_test_linear_functions(orc, L, a):
    """On a jittered grid without boundary treatment, A u = 0 at interior
    nodes for every linear u, and u^T A u = |grad u|^2 * area(unit square)."""
    N = synth.grid_size(L)
    xy = synth.coords(L, a, seed=7)
    A = bands_to_csr(N, orc.assemble(N, xy, dirichlet=False))
    x, y = xy[:, 0], xy[:, 1]
    u = 0.3 * x - 1.7 * y + 0.4
    r = A @ u
    mask = synth.interior_mask(L)
    assert np.max(np.abs(r[mask])) < 1e-13
    assert abs(x @ (A @ x) - 1.0) < 1e-12
    assert abs(y @ (A @ y) - 1.0) < 1e-12
    assert abs(x @ (A @ y)) < 1e-12


@pytest.mark.parametrize("L,a", [(2, 0.0), (4, 0.2), (6, 0.25)])
def test_bands_bitwise_symmetric_and_dirichlet(orc, L, a):
    N = synth.grid_size(L)
    n = N * N
    bands = orc.assemble(N, synth.coords(L, a, seed=11), dirichlet=True)
    offs = band_offsets(N)
    for k in range(9):
        kt = 8 - k  # the transposed band
        p = np.arange(n)
        q = p + offs[k]
        ok = (q >= 0) & (q < n)
        np.testing.assert_array_equal(bands[k][p[ok]], bands[kt][q[ok]])
    bnd = ~synth.interior_mask(L)
    assert np.all(bands[4][bnd] == 1.0)
    for k in range(9):
        if k != 4:
            assert np.all(bands[k][bnd] == 0.0)
    A = bands_to_csr(N, bands).toarray()
    assert np.all(A[:, bnd][~bnd] == 0.0)  # boundary columns zeroed
    assert np.count_nonzero(A, axis=1).max() <= 9


@pytest.mark.parametrize("L,a", [(1, 0.0), (2, 0.25), (3, 0.2), (4, 0.25)])
def test_interior_block_positive_definite(orc, L, a):
    N = synth.grid_size(L)
    A = bands_to_csr(N, orc.assemble(N, synth.coords(L, a, seed=3))).toarray()
    m = synth.interior_mask(L)
    Ai = A[np.ix_(m, m)]
    rc, _ = orc.cholesky(Ai)
    assert rc == 0
    assert np.linalg.eigvalsh(Ai).min() > 0


def test_load_vector_partition_of_unity(orc):
    """f = 1: sum_p b_p = area = 1 on any grid; uniform interior b_p = h^2."""
    L = 4
    N = synth.grid_size(L)
    b = orc.load_vector(N, synth.coords(L, 0.25, seed=5), fn=1, dirichlet=False)
    assert abs(b.sum() - 1.0) < 1e-13
    bu = orc.load_vector(N, synth.coords(L), fn=1, dirichlet=False)
    h = 1.0 / (N - 1)
    np.testing.assert_allclose(bu[synth.interior_mask(L)], h * h, rtol=1e-13)


def test_l2_norm_of_zero_is_norm_of_u(orc):
    """||u - 0||_L2 = ||sin(pi x) sin(pi y)||_L2 = 1/2 on the unit square."""
    L = 5
    N = synth.grid_size(L)
    err = orc.l2_error_sinsin(N, synth.coords(L, 0.2, seed=9), np.zeros(N * N))
    assert abs(err - 0.5) < 1e-10


# ---------------------------------------------------------------- band ops


@pytest.mark.parametrize("L", [2, 4, 5])
def test_spmv_defect_jacobi_match_scipy(orc, L):
    N = synth.grid_size(L)
    xy = synth.coords(L, 0.2, seed=21)
    bands = orc.assemble(N, xy)
    A = bands_to_csr(N, bands)
    rng = np.random.default_rng(L)
    x, b = rng.standard_normal(N * N), rng.standard_normal(N * N)
    np.testing.assert_allclose(orc.spmv(N, bands, x), A @ x, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(orc.defect(N, bands, b, x), b - A @ x, rtol=1e-14, atol=1e-14)
    diag = A.diagonal()
    np.testing.assert_allclose(orc.jacobi(N, bands, b, x, 0.7), x + 0.7 * (b - A @ x) / diag,
                               rtol=1e-13, atol=1e-13)


def _prolong_matrix(orc, Nf):
    Nc = (Nf - 1) // 2 + 1
    P = np.zeros((Nf * Nf, Nc * Nc))
    for c in range(Nc * Nc):
        e = np.zeros(Nc * Nc)
        e[c] = 1.0
        P[:, c] = orc.prolong_add(Nf, e, np.zeros(Nf * Nf))
    return P


def test_prolongation_reproduces_bilinear_index_functions(orc):
    Nf = 17
    Nc = 9
    I = np.tile(np.arange(Nc), Nc).astype(float)
    J = np.repeat(np.arange(Nc), Nc).astype(float)
    g = lambda a, b: 0.3 + 1.1 * a - 0.7 * b + 0.25 * a * b
    xf = orc.prolong_add(Nf, g(I, J), np.zeros(Nf * Nf))
    fi = np.tile(np.arange(Nf), Nf) / 2.0
    fj = np.repeat(np.arange(Nf), Nf) / 2.0
    np.testing.assert_allclose(xf, g(fi, fj), atol=1e-14)


def test_restriction_is_prolongation_transpose(orc):
    Nf = 17
    rng = np.random.default_rng(0)
    d = rng.standard_normal(Nf * Nf)
    xc = rng.standard_normal(81)
    lhs = orc.restrict(Nf, d, filter=False) @ xc
    rhs = d @ orc.prolong_add(Nf, xc, np.zeros(Nf * Nf))
    assert abs(lhs - rhs) < 1e-12
    # the filter zeroes exactly the coarse boundary
    bc = orc.restrict(Nf, d, filter=True)
    m = synth.interior_mask(3)
    np.testing.assert_array_equal(bc[~m], 0.0)
    np.testing.assert_array_equal(bc[m], orc.restrict(Nf, d, filter=False)[m])


def test_restriction_of_constant_is_four(orc):
    Nf = 33
    bc = orc.restrict(Nf, np.ones(Nf * Nf), filter=True).reshape(17, 17)
    np.testing.assert_array_equal(bc[1:-1, 1:-1], 4.0)


@pytest.mark.parametrize("L", [2, 3, 4])
def test_galerkin_identity_uniform(orc, L):
    """Rediscretised coarse operator = P^T A_f P on uniform grids (interior
    block), which fixes the scaling of restriction relative to prolongation."""
    Nf, Nc = synth.grid_size(L), synth.grid_size(L - 1)
    Af = bands_to_csr(Nf, orc.assemble(Nf, synth.coords(L))).toarray()
    Ac = bands_to_csr(Nc, orc.assemble(Nc, synth.coords(L - 1))).toarray()
    P = _prolong_matrix(orc, Nf)
    G = P.T @ Af @ P
    m = synth.interior_mask(L - 1)
    np.testing.assert_allclose(G[np.ix_(m, m)], Ac[np.ix_(m, m)], atol=1e-14)


# ---------------------------------------------------------------- solver


@pytest.mark.parametrize("L,a", [(2, 0.0), (3, 0.2), (4, 0.25)])
def test_mg_matches_dense_direct_solve(orc, L, a):
    N = synth.grid_size(L)
    xy = synth.coords(L, a, seed=31)
    h = orc.Hierarchy(L, xy)
    b = synth.rhs_uniform(L, 41)
    x, st = h.solve_fp64(b, o=orc.opts(rel_tol=1e-13))
    assert st.status == 0
    A = bands_to_csr(N, h.bands(L)).toarray()
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_coarse_level_equal_to_finest_is_direct(orc):
    L = 3
    N = synth.grid_size(L)
    xy = synth.coords(L, 0.2, seed=1)
    h = orc.Hierarchy(L, xy, Lc=3)
    b = synth.rhs_uniform(L, 2)
    x, st = h.solve_fp64(b, o=orc.opts(rel_tol=1e-12))
    assert st.cycles == 1 and st.rel_res < 1e-13
    A = bands_to_csr(N, h.bands(L)).toarray()
    np.testing.assert_allclose(x, np.linalg.solve(A, b), atol=1e-13)


@pytest.mark.parametrize("L,a", [(6, 0.0), (6, 0.2), (7, 0.2)])
def test_vcycle_contraction_below_0p2(orc, L, a):
    h = orc.Hierarchy(L, synth.coords(L, a, seed=L))
    b = synth.rhs_uniform(L, 100 + L)
    x, st = h.solve_fp64(b, o=orc.opts(rel_tol=1e-10))
    hist = [st.bnorm / st.bnorm] + orc.hist(st)
    rates = [hist[k + 1] / hist[k] for k in range(len(hist) - 1)]
    assert st.status == 0
    assert max(rates) < 0.2, rates


def test_cycle_count_independent_of_level(orc):
    counts = []
    for L in [4, 5, 6, 7, 8]:
        h = orc.Hierarchy(L, synth.coords(L, 0.2, seed=L))
        _, st = h.solve_fp64(synth.rhs_uniform(L, L), o=orc.opts(rel_tol=1e-8))
        assert st.status == 0
        counts.append(st.cycles)
    assert max(counts) - min(counts) <= 2, counts


def _sinsin_l2(orc, L, mode):
    N = synth.grid_size(L)
    xy = synth.coords(L)
    h = orc.Hierarchy(L, xy)
    b = orc.load_vector(N, xy, fn=0)
    if mode == "double":
        x, st = h.solve_fp64(b, o=orc.opts(rel_tol=1e-12))
    elif mode == "mixed":
        x, st = h.solve_mixed_emulated(b, o=orc.opts(rel_tol=1e-12))
    else:  # single: one outer step = FP32 multigrid on its own
        x, st = h.solve_mixed_emulated(
            b, o=orc.opts(fixed_cycles=1, inner_reduction=0.0, inner_max_cycles=30))
    return orc.l2_error_sinsin(N, xy, x)


def _table1():
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_l2_errors.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    return {int(r[0]): [float(v) for v in r[1:]] for r in rows}


def test_l2_error_reduction_is_h2_like_table1(orc):
    """Table 1: the double column reduces by 4.27, 4.07, 4.02, then 4.00;
    here (u = sin(pi x) sin(pi y), a smooth test function) the reduction
    factors must also tend to 4 and lie within the paper's spread."""
    t1 = _table1()
    errs = {L: _sinsin_l2(orc, L, "double") for L in range(2, 8)}
    for L in range(3, 8):
        red = errs[L - 1] / errs[L]
        paper = t1[L][3]
        assert 3.95 < red < 4.30, (L, red)
        if L >= 5:
            assert abs(red - paper) < 0.03, (L, red, paper)


def test_mixed_equals_double_and_single_breaks_down(orc):
    """Table 1: mixed reproduces the double-precision L2 error; a solve
    entirely in single precision loses accuracy as the level grows (here the
    single-precision error is within rounding noise of the double one up to
    L = 8 and far above it at L = 9, where the discretisation error has
    fallen below what single precision resolves)."""
    t1 = _table1()
    for L in [4, 6, 8]:
        ed = _sinsin_l2(orc, L, "double")
        em = _sinsin_l2(orc, L, "mixed")
        assert abs(em - ed) <= 1e-4 * ed, (L, em, ed)
        assert abs(t1[L][4] - t1[L][2]) <= 1e-4 * t1[L][2]  # the paper's own columns
    e_single9 = _sinsin_l2(orc, 9, "single")
    e_double9 = _sinsin_l2(orc, 9, "double")
    assert e_single9 > 5.0 * e_double9


@pytest.mark.parametrize("L", [6, 7])
def test_mixed_reaches_1e8_and_fp32_alone_stalls(orc, L):
    h = orc.Hierarchy(L, synth.coords(L, 0.2, seed=L))
    b = synth.rhs_uniform(L, 77)
    x, st = h.solve_mixed_emulated(b, o=orc.opts(rel_tol=1e-8))
    assert st.status == 0 and st.rel_res <= 1e-8
    assert st.outer_steps <= 6
    _, st32 = h.solve_mixed_emulated(
        b, o=orc.opts(fixed_cycles=1, inner_reduction=0.0, inner_max_cycles=40))
    assert st32.rel_res > 1e-8


@pytest.mark.parametrize("k", [-60, -1, 1, 45])
def test_mixed_solution_scales_exactly_with_b(orc, k):
    """The mixed scheme brings defects into single-precision range with a
    power of two taken from ||b||; powers of two scale exactly in binary
    arithmetic, so solving for 2^k b gives exactly 2^k times the solution
    for b, with the same relative residuals and cycle counts.  A correction
    not scaled back (or scaled by another factor) breaks it."""
    L = 6
    h = orc.Hierarchy(L, synth.coords(L, 0.2, seed=5))
    b = synth.rhs_uniform(L, 6)
    o = orc.opts(rel_tol=1e-9)
    x1, s1 = h.solve_mixed_emulated(b, o=o)
    x2, s2 = h.solve_mixed_emulated(np.ldexp(b, k), o=o)
    assert s1.status == 0 and s2.status == 0
    np.testing.assert_array_equal(x2, np.ldexp(x1, k))
    assert s2.bnorm == np.ldexp(s1.bnorm, k)
    assert (s2.rel_res, s2.cycles, s2.outer_steps) == (s1.rel_res, s1.cycles, s1.outer_steps)


def test_no_convergence_status(orc):
    L = 5
    h = orc.Hierarchy(L, synth.coords(L))
    _, st = h.solve_fp64(synth.rhs_uniform(L, 1), o=orc.opts(rel_tol=1e-12, max_cycles=2))
    assert st.status == 3 and st.cycles == 2


def test_zero_rhs_gives_zero(orc):
    L = 3
    h = orc.Hierarchy(L, synth.coords(L))
    x, st = h.solve_fp64(np.zeros(81), x0=np.ones(81))
    assert st.status == 0 and np.all(x == 0)


# ---------------------------------------------------------------- inputs


def test_synth_generator_properties():
    k = np.arange(100000, dtype=np.uint64)
    u = synth.uniform(123, k)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.005
    assert not np.array_equal(u, synth.uniform(124, k))
    xy = synth.coords(4, 0.25, seed=9)
    N = 17
    h = 1.0 / 16
    base = np.stack([np.tile(np.arange(N), N) * h, np.repeat(np.arange(N), N) * h], 1)
    m = synth.interior_mask(4)
    assert np.all(np.abs(xy - base)[m] <= 0.25 * h + 1e-17)
    np.testing.assert_array_equal(xy[~m], base[~m])


@pytest.mark.parametrize("L,rtol", [(3, 1e-7), (4, 1e-9), (5, 1e-10)])
def test_load_vector_sinsin_closed_form_uniform(orc, L, rtol):
    """Uniform grid: int sin(pi x) phi_i(x) dx = sin(pi x_i) 2(1 - cos(pi h))
    / (pi^2 h) for the 1D hat, so b_p = f(x_p) * that factor squared; the
    3x3 Gauss rule reproduces it to O(h^6)."""
    N = synth.grid_size(L)
    h = 1.0 / (N - 1)
    b = orc.load_vector(N, synth.coords(L), fn=0)
    xi = np.tile(np.arange(N), N) * h
    yj = np.repeat(np.arange(N), N) * h
    c = 2.0 * (1.0 - np.cos(np.pi * h)) / (np.pi ** 2 * h)
    ref = 2.0 * np.pi ** 2 * np.sin(np.pi * xi) * np.sin(np.pi * yj) * c * c
    m = synth.interior_mask(L)
    np.testing.assert_allclose(b[m], ref[m], rtol=rtol)
    np.testing.assert_array_equal(b[~m], 0.0)


# ---------------------------------------------------------------- mixed boundary conditions
# Dirichlet on the sides of a mask (1: x = 0, 2: x = 1, 4: y = 0, 8: y = 1),
# natural homogeneous Neumann condition on the others (Sec. 2.1).


def dirichlet_nodes(N, dmask):
    i = np.tile(np.arange(N), N)
    j = np.repeat(np.arange(N), N)
    return (((i == 0) & bool(dmask & 1)) | ((i == N - 1) & bool(dmask & 2)) |
            ((j == 0) & bool(dmask & 4)) | ((j == N - 1) & bool(dmask & 8)))


def _manufactured_l2(orc, L, fn, dmask, a=0.0):
    N = synth.grid_size(L)
    xy = synth.coords(L, a, seed=7)
    h = orc.Hierarchy(L, xy, dmask=dmask)
    b = orc.load_vector(N, xy, fn=fn, dmask=dmask)
    x, st = h.solve_fp64(b, o=orc.opts(rel_tol=1e-12))
    assert st.status == 0
    return orc.l2_error(N, xy, x, fn)


@pytest.mark.parametrize("fn,dmask", [(2, 12), (3, 5)])
def test_mixed_bc_manufactured_solution_h2(orc, fn, dmask):
    """u = cos(pi x) sin(pi y) (Neumann on x = 0, 1) and u = sin(pi x/2)
    sin(pi y/2) (Neumann on x = 1, y = 1): the L2 error falls by 4 per level
    only if the natural condition is left on exactly the Neumann sides."""
    errs = {L: _manufactured_l2(orc, L, fn, dmask) for L in range(3, 8)}
    for L in range(4, 8):
        red = errs[L - 1] / errs[L]
        assert 3.9 < red < 4.1, (L, red)
    jit = {L: _manufactured_l2(orc, L, fn, dmask, a=0.2) for L in range(4, 8)}
    for L in range(5, 8):
        assert 3.5 < jit[L - 1] / jit[L] < 4.5, (L, jit)
    # the same problem with Dirichlet everywhere misses the solution by O(1)
    assert _manufactured_l2(orc, 6, fn, 15) > 100 * errs[6]


@pytest.mark.parametrize("dmask", [1, 5, 12, 3])
def test_mixed_bc_rows_columns_and_symmetry(orc, dmask):
    L = 4
    N = synth.grid_size(L)
    xy = synth.coords(L, 0.2, seed=3)
    bands = orc.assemble(N, xy, dmask=dmask)
    A = bands_to_csr(N, bands).toarray()
    D = dirichlet_nodes(N, dmask)
    # Dirichlet rows and columns: identity
    np.testing.assert_array_equal(A[D][:, ~D], 0.0)
    np.testing.assert_array_equal(A[~D][:, D], 0.0)
    np.testing.assert_array_equal(np.diag(A)[D], 1.0)
    # bitwise symmetric; the non-Dirichlet block positive definite
    np.testing.assert_array_equal(A, A.T)
    assert np.linalg.eigvalsh(A[np.ix_(~D, ~D)]).min() > 0
    # rows away from Dirichlet nodes, including Neumann boundary rows, sum to
    # zero (constants are in the kernel of the Neumann operator)
    near = (A[:, D] != 0).any(axis=1) | D
    full = bands_to_csr(N, orc.assemble(N, xy, dirichlet=False)).toarray()
    near |= (full[:, D] != 0).any(axis=1)
    rows = ~near
    bnd = ~synth.interior_mask(L)
    assert (rows & bnd).any()  # some Neumann boundary rows are checked
    scale = np.abs(A).max(axis=1)
    assert np.all(np.abs(A[rows].sum(axis=1)) <= 1e-13 * scale[rows])


@pytest.mark.parametrize("dmask", [5, 12, 3])
@pytest.mark.parametrize("L", [2, 3, 4])
def test_mixed_bc_galerkin_identity_uniform(orc, L, dmask):
    Nf, Nc = synth.grid_size(L), synth.grid_size(L - 1)
    Af = bands_to_csr(Nf, orc.assemble(Nf, synth.coords(L), dmask=dmask)).toarray()
    Ac = bands_to_csr(Nc, orc.assemble(Nc, synth.coords(L - 1), dmask=dmask)).toarray()
    P = _prolong_matrix(orc, Nf)
    G = P.T @ Af @ P
    m = ~dirichlet_nodes(Nc, dmask)
    np.testing.assert_allclose(G[np.ix_(m, m)], Ac[np.ix_(m, m)], atol=1e-14)


def test_mixed_bc_restriction_filters_only_dirichlet_sides(orc):
    Nf, dmask = 17, 6
    d = np.random.default_rng(1).standard_normal(Nf * Nf)
    bc = orc.restrict(Nf, d, dmask=dmask)
    free = orc.restrict(Nf, d, filter=False)
    D = dirichlet_nodes(9, dmask)
    np.testing.assert_array_equal(bc[D], 0.0)
    np.testing.assert_array_equal(bc[~D], free[~D])
    bc32 = orc.restrict_f32(Nf, d.astype(np.float32), dmask=dmask)
    np.testing.assert_array_equal(bc32[D], 0.0)
    np.testing.assert_allclose(bc32[~D], free[~D], rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("L,dmask", [(3, 1), (4, 12), (4, 6)])
def test_mixed_bc_mg_matches_dense_direct_solve(orc, L, dmask):
    N = synth.grid_size(L)
    xy = synth.coords(L, 0.2, seed=5)
    h = orc.Hierarchy(L, xy, dmask=dmask)
    D = dirichlet_nodes(N, dmask)
    b = synth.rhs_uniform(L, 6)
    b = np.where(D, 0.0, np.random.default_rng(L).uniform(-1, 1, N * N))
    x, st = h.solve_fp64(b, o=orc.opts(rel_tol=1e-13))
    assert st.status == 0
    A = bands_to_csr(N, h.bands(L)).toarray()
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)
    xm, sm = h.solve_mixed_emulated(b, o=orc.opts(rel_tol=1e-8))
    assert sm.status == 0 and sm.rel_res <= 1e-8


@pytest.mark.parametrize("dmask", [12, 5])
def test_mixed_bc_vcycle_contraction(orc, dmask):
    L = 6
    h = orc.Hierarchy(L, synth.coords(L, 0.2, seed=L), dmask=dmask)
    N = synth.grid_size(L)
    b = np.where(dirichlet_nodes(N, dmask), 0.0, np.random.default_rng(9).uniform(-1, 1, N * N))
    x, st = h.solve_fp64(b, o=orc.opts(rel_tol=1e-10))
    hist = [1.0] + orc.hist(st)
    rates = [hist[k + 1] / hist[k] for k in range(len(hist) - 1)]
    assert st.status == 0
    assert max(rates) < 0.2, rates


# ---------------------------------------------------------------- conjugate gradients


def _scipy_cg_iterates(A, b, steps, M=None):
    """Iterates of scipy's own CG (an independent implementation of the same
    recurrences), one per step, from x0 = 0 with the stopping test off."""
    from scipy.sparse.linalg import cg
    out = []
    cg(A, b, x0=np.zeros_like(b), rtol=0.0, atol=0.0, maxiter=steps, M=M,
       callback=lambda xk: out.append(np.array(xk, copy=True)))
    return out


@pytest.mark.parametrize("L,a,dmask", [(3, 0.0, 15), (4, 0.2, 15), (4, 0.2, 5)])
def test_cg_iterates_match_scipy_cg(orc, L, a, dmask):
    N = synth.grid_size(L)
    h = orc.Hierarchy(L, synth.coords(L, a, seed=8), dmask=dmask)
    bands = h.bands(L)
    b = synth.rhs_uniform(L, 12, dmask)
    A = bands_to_csr(N, bands)
    ref = _scipy_cg_iterates(A, b, 6)
    for k in range(1, 7):
        x, steps = orc.cg(N, bands, b, tol=0.0, max_iter=k)
        assert steps == k
        assert np.linalg.norm(x - ref[k - 1]) <= 1e-12 * np.linalg.norm(ref[k - 1])


@pytest.mark.parametrize("L,dmask", [(2, 15), (3, 15), (3, 12), (4, 1)])
def test_cg_solves_to_tolerance_and_stops_there(orc, L, dmask):
    N = synth.grid_size(L)
    h = orc.Hierarchy(L, synth.coords(L, 0.2, seed=4), dmask=dmask)
    bands = h.bands(L)
    b = synth.rhs_uniform(L, 3, dmask)
    A = bands_to_csr(N, bands).toarray()
    xd = np.linalg.solve(A, b)
    x, steps = orc.cg(N, bands, b, tol=1e-13, max_iter=1000)
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)
    # the stop test: the step before the last had not yet reached the bound
    assert np.linalg.norm(b - A @ x) <= 1.01e-13 * np.linalg.norm(b)
    xp, _ = orc.cg(N, bands, b, tol=0.0, max_iter=steps - 1)
    assert np.linalg.norm(b - A @ xp) > 1e-13 * np.linalg.norm(b) * 0.99
    # Dirichlet nodes keep their zero start
    D = dirichlet_nodes(N, dmask)
    assert np.all(x[D] == 0.0)
    # zero right-hand side: no step
    z, k0 = orc.cg(N, bands, np.zeros(N * N), tol=1e-10, max_iter=50)
    assert k0 == 0 and not z.any()


def test_cg_residuals_orthogonal_and_energy_error_decreasing(orc):
    L = 4
    N = synth.grid_size(L)
    h = orc.Hierarchy(L, synth.coords(L, 0.25, seed=19))
    bands = h.bands(L)
    b = synth.rhs_uniform(L, 20)
    A = bands_to_csr(N, bands).toarray()
    xd = np.linalg.solve(A, b)
    rs, errs = [], []
    for k in range(0, 8):
        x, _ = orc.cg(N, bands, b, tol=0.0, max_iter=k)
        rs.append(b - A @ x)
        e = x - xd
        errs.append(np.sqrt(e @ A @ e))
    for i in range(len(rs)):
        for j in range(i):
            assert abs(rs[i] @ rs[j]) <= 1e-10 * np.linalg.norm(rs[i]) * np.linalg.norm(rs[j])
    assert all(errs[k + 1] < errs[k] for k in range(len(errs) - 1))


@pytest.mark.parametrize("Lc", [1, 2, 3, 4])
def test_cg_coarse_solver_matches_cholesky_cycle(orc, Lc):
    L = 6
    h = orc.Hierarchy(L, synth.coords(L, 0.2, seed=2), Lc=Lc)
    b = synth.rhs_uniform(L, 5)
    x0 = np.zeros(b.size)
    xc = h.vcycle(L, x0, b, orc.opts())
    xg = h.vcycle(L, x0, b, orc.opts(coarse_cg=True, coarse_tol=1e-14, coarse_max_iter=1000))
    assert np.linalg.norm(xg - xc) <= 1e-12 * np.linalg.norm(xc)
    # a loose coarse tolerance still converges, in about as many cycles
    _, s0 = h.solve_fp64(b, o=orc.opts())
    _, s1 = h.solve_fp64(b, o=orc.opts(coarse_cg=True, coarse_tol=1e-3))
    assert s1.status == 0 and abs(s1.cycles - s0.cycles) <= 1


@pytest.mark.parametrize("L,a,dmask", [(4, 0.2, 15), (5, 0.25, 12)])
def test_pcg_iterates_match_scipy_pcg_with_the_cycle_as_preconditioner(orc, L, a, dmask):
    from scipy.sparse.linalg import LinearOperator
    N = synth.grid_size(L)
    h = orc.Hierarchy(L, synth.coords(L, a, seed=3), dmask=dmask)
    b = synth.rhs_uniform(L, 4, dmask)
    A = bands_to_csr(N, h.bands(L))
    n = N * N
    M = LinearOperator((n, n), dtype=np.float64,
                       matvec=lambda r: h.vcycle(L, np.zeros(n), np.ravel(r).astype(np.float64)))
    ref = _scipy_cg_iterates(A, b, 4, M=M)
    for k in range(1, 5):
        x, st = h.solve_pcg(b, o=orc.opts(fixed_cycles=k))
        assert st.cycles == k
        assert np.linalg.norm(x - ref[k - 1]) <= 1e-12 * np.linalg.norm(ref[k - 1])
        assert abs(st.rel_res - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) <= 1e-12


@pytest.mark.parametrize("precond32", [False, True])
def test_pcg_reaches_tolerance_with_fewer_steps_than_cycles(orc, precond32):
    for L in (6, 8):
        h = orc.Hierarchy(L, synth.coords(L, 0.2, seed=1002))
        b = synth.rhs_uniform(L, 2002)
        xm, sm = h.solve_fp64(b, o=orc.opts(rel_tol=1e-10))
        xp, sp_ = h.solve_pcg(b, o=orc.opts(rel_tol=1e-10), precond32=precond32)
        assert sp_.status == 0 and sp_.rel_res <= 1.01e-10
        assert sp_.cycles < sm.cycles
        assert np.linalg.norm(xp - xm) <= 1e-8 * np.linalg.norm(xm)
        # residual history falls monotonically by at least 5x per step
        hist = [1.0] + orc.hist(sp_)
        assert all(hist[k + 1] < 0.2 * hist[k] for k in range(len(hist) - 1)), hist


# ---------------------------------------------------------------- BLAS level 1


def test_blas1_closed_forms(orc):
    n = 1000
    i = np.arange(1, n + 1, dtype=np.float64)
    assert orc.dot(i, i) == n * (n + 1) * (2 * n + 1) / 6
    assert orc.dot(i, np.ones(n)) == n * (n + 1) / 2
    assert orc.norm2(np.full(n, 3.0)) == 3.0 * np.sqrt(n)
    y = orc.axpy(2.0, i, np.ones(n))
    np.testing.assert_array_equal(y, 2 * i + 1)
    np.testing.assert_array_equal(orc.axpy(0.0, i, i), i)
    y32 = orc.axpy(-1.0, i.astype(np.float32), i.astype(np.float32))
    assert y32.dtype == np.float32 and not y32.any()


def test_blas1_dot_against_exactly_rounded_sum(orc):
    import math
    rng = np.random.default_rng(5)
    x = rng.standard_normal(4097)
    y = rng.standard_normal(4097)
    exact = math.fsum(float(a) * float(b) for a, b in zip(x, y))
    s = orc.dot(x, y)
    # recursive summation: |error| <= gamma_n sum |x y| (products exact in fsum
    # up to their own rounding, u each)
    bound = (x.size + 1) * 2.0 ** -53 * float(np.sum(np.abs(x * y)))
    assert abs(s - exact) <= bound
    # FP32 axpy: the correctly rounded image of the FP64 value
    x32 = x.astype(np.float32)
    y32 = y.astype(np.float32)
    r = orc.axpy(0.3, x32, y32)
    ref = np.float32(0.3).astype(np.float64) * x32.astype(np.float64) + y32.astype(np.float64)
    assert np.all(np.abs(r.astype(np.float64) - ref) <= 2.0 ** -24 * np.abs(ref))


# ---------------------------------------------------------------- four-band combination


def _band4_csr(n, band, offs):
    """scipy matrix of one four-band term, built from the band definition."""
    rows, cols, vals = [], [], []
    p = np.arange(n)
    for k, o in enumerate(offs):
        ok = (p + o >= 0) & (p + o < n)
        rows.append(p[ok])
        cols.append(p[ok] + o)
        vals.append(band[k][ok])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def test_band4_matches_scipy_products(orc):
    N = 37
    n = N * N
    rng = np.random.default_rng(4)
    offsets = [(-2, -1, 1, 2), (-2 * N, -N, N, 2 * N), (-1, 0, 1, N), (-N - 1, -N + 1, N - 1, N + 1)]
    bands = [rng.standard_normal((4, n)) for _ in offsets]
    vs = [rng.standard_normal(n) for _ in offsets]
    u = rng.standard_normal(n)
    s = rng.standard_normal(n)
    ref = u + s
    for b, o, v in zip(bands, offsets, vs):
        ref = ref + _band4_csr(n, b, o) @ v
    got = orc.band4_combine(bands, offsets, vs, u, s)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
    # fewer terms, no source
    got2 = orc.band4_combine(bands[:1], offsets[:1], vs[:1], u)
    np.testing.assert_allclose(got2, u + _band4_csr(n, bands[0], offsets[0]) @ vs[0], atol=1e-13)


def test_band4_central_differences_of_linear_functions_are_exact(orc):
    # d/dx and d/dy by central differences (the second-order space
    # discretisation of the shallow-water scheme) of f = 3x - 2y on a grid of
    # spacing 1: 3 and -2 at every interior node
    N = 20
    n = N * N
    i = np.tile(np.arange(N), N).astype(np.float64)
    j = np.repeat(np.arange(N), N).astype(np.float64)
    f = 3 * i - 2 * j
    dx = np.zeros((4, n))
    dx[0], dx[1] = -0.5, 0.5      # offsets -1, +1
    dy = np.zeros((4, n))
    dy[2], dy[3] = -0.5, 0.5      # offsets -N, +N
    zero = np.zeros(n)
    gx = orc.band4_combine([dx], [(-1, 1, -N, N)], [f], zero)
    gy = orc.band4_combine([dy], [(-1, 1, -N, N)], [f], zero)
    inner = (i > 0) & (i < N - 1) & (j > 0) & (j < N - 1)
    assert np.all(gx[inner] == 3.0) and np.all(gy[inner] == -2.0)
    # a pure shift: v moved by one, the last entry has no neighbour
    sh = np.zeros((4, 5))
    sh[0] = 1.0
    v = np.arange(1.0, 6.0)
    np.testing.assert_array_equal(orc.band4_combine([sh], [(1, 2, 3, 4)], [v], np.zeros(5)),
                                  [2.0, 3.0, 4.0, 5.0, 0.0])
