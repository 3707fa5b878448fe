"""The OpenMP build of the oracle (all host cores, used for the benchmark's
all-core CPU timing) gives the same bits as the one-thread build: only loops
whose iterations write disjoint outputs are threaded, every sum stays a
sequential loop."""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def problem(orc):
    L, a, gs = 7, 0.2, 1002
    return L, synth.coords(L, a, gs), synth.rhs_uniform(L, 2002)


def test_threaded_build_uses_threads(orc):
    assert orc.threads(False) == 1
    assert orc.threads(True) >= 1


@pytest.mark.parametrize("dmask", [15, 5])
def test_threaded_solves_are_bitwise_equal(orc, problem, dmask):
    L, xy, _ = problem
    b = synth.rhs_uniform(L, 2002, dirichlet_sides=dmask)
    h1 = orc.Hierarchy(L, xy, dmask=dmask)
    hn = orc.Hierarchy(L, xy, dmask=dmask, threaded=True)
    try:
        np.testing.assert_array_equal(h1.bands(L), hn.bands(L))
        x1, s1 = h1.solve_fp64(b)
        xn, sn = hn.solve_fp64(b)
        assert s1.cycles == sn.cycles and s1.cycles > 0
        np.testing.assert_array_equal(x1, xn)
        assert orc.hist(s1) == orc.hist(sn)
        m1, t1 = h1.solve_mixed_emulated(b)
        mn, tn = hn.solve_mixed_emulated(b)
        assert (t1.outer_steps, t1.cycles) == (tn.outer_steps, tn.cycles)
        np.testing.assert_array_equal(m1, mn)
        p1, u1 = h1.solve_pcg(b, precond32=True)
        pn, un = hn.solve_pcg(b, precond32=True)
        assert u1.cycles == un.cycles
        np.testing.assert_array_equal(p1, pn)
    finally:
        h1.close()
        hn.close()


def test_threaded_band_operations_are_bitwise_equal(orc, problem):
    L, xy, b = problem
    N = (1 << L) + 1
    bands = orc.assemble(N, xy)
    x = np.random.default_rng(3).standard_normal(N * N)
    one, many = orc.lib(), orc.lib_omp()
    outs = []
    for lib in (one, many):
        y = np.zeros(N * N)
        lib.or_spmv(N, orc._d(bands.reshape(-1)), orc._d(x), orc._d(y))
        z = np.zeros(N * N)
        lib.or_jacobi(N, orc._d(bands.reshape(-1)), orc._d(b), orc._d(x), orc._d(z), 0.7)
        Nc = (N - 1) // 2 + 1
        bc = np.zeros(Nc * Nc)
        lib.or_restrict_bc(N, orc._d(x), orc._d(bc), 15)
        xf = x.copy()
        lib.or_prolong_add(N, orc._d(bc), orc._d(xf))
        outs.append((y, z, bc, xf))
    for a, c in zip(*outs):
        np.testing.assert_array_equal(a, c)
