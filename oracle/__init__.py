"""TEST INFRASTRUCTURE ONLY: ctypes binding of the plain FP64 CPU oracle.

The oracle (``mg_oracle.c``) is a slow, obviously correct implementation of
the Q1 finite-element multigrid Poisson solver of HONEI (arXiv 0904.4152,
Sec. 2.1 and Sec. 6.2).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the GPU product
path never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
_HDR = os.path.join(_HERE, "mg_oracle.h")
_LIB = os.path.join(_HERE, "libmg_oracle.so")
# The same source built with -fopenmp: element-wise loops on every host core,
# sums sequential (bitwise the results of the one-thread build).
_LIB_OMP = os.path.join(_HERE, "libmg_oracle_omp.so")

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)


def _compile(out: str, extra, force: bool) -> str:
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_HDR))
    if force or not os.path.exists(out) or os.path.getmtime(out) < newest:
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-ffp-contract=off"] + list(extra) + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction), one
    thread; with ``force`` also the OpenMP build."""
    if force:
        build_omp(force=True)
    return _compile(_LIB, [], force)


def build_omp(force: bool = False) -> str:
    """The same source with -fopenmp (the all-core timing of the benchmark)."""
    return _compile(_LIB_OMP, ["-fopenmp"], force)


class OrOpts(ctypes.Structure):
    _fields_ = [("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("omega", ctypes.c_double), ("rel_tol", ctypes.c_double),
                ("max_cycles", ctypes.c_int), ("fixed_cycles", ctypes.c_int),
                ("inner_reduction", ctypes.c_double), ("inner_max_cycles", ctypes.c_int),
                ("coarse_cg", ctypes.c_int), ("coarse_tol", ctypes.c_double),
                ("coarse_max_iter", ctypes.c_int)]


class OrStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cycles", ctypes.c_int),
                ("outer_steps", ctypes.c_int), ("bnorm", ctypes.c_double),
                ("rel_res", ctypes.c_double), ("n_hist", ctypes.c_int),
                ("res_hist", ctypes.c_double * 256)]


_lib = None
_lib_omp = None


def lib():
    """The one-thread oracle library."""
    global _lib
    if _lib is None:
        _lib = _declare(ctypes.CDLL(build()))
    return _lib


def lib_omp():
    """The OpenMP build of the same source (element-wise loops threaded)."""
    global _lib_omp
    if _lib_omp is None:
        _lib_omp = _declare(ctypes.CDLL(build_omp()))
    return _lib_omp


def threads(threaded: bool = True) -> int:
    """Host threads the chosen build's element-wise loops use."""
    return (lib_omp() if threaded else lib()).or_threads()


def _declare(L):
    """Argument and result types of every exported function."""
    L.or_element_stiffness.argtypes = [_dp, _dp, _dp]
    L.or_assemble.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp]
    L.or_load_vector.argtypes = [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, _dp]
    L.or_l2_error_sinsin.argtypes = [ctypes.c_int, _dp, _dp]
    L.or_l2_error_sinsin.restype = ctypes.c_double
    L.or_spmv.argtypes = [ctypes.c_int, _dp, _dp, _dp]
    L.or_defect.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
    L.or_jacobi.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_double]
    L.or_restrict.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int]
    L.or_prolong_add.argtypes = [ctypes.c_int, _dp, _dp]
    L.or_norm2.argtypes = [ctypes.c_size_t, _dp]
    L.or_norm2.restype = ctypes.c_double
    L.or_cholesky.argtypes = [ctypes.c_int, _dp]
    L.or_cholesky_solve.argtypes = [ctypes.c_int, _dp, _dp]
    L.or_spmv_f32.argtypes = [ctypes.c_int, _fp, _fp, _fp]
    L.or_jacobi_f32.argtypes = [ctypes.c_int, _fp, _fp, _fp, _fp, ctypes.c_float]
    L.or_restrict_f32.argtypes = [ctypes.c_int, _fp, _fp]
    L.or_prolong_add_f32.argtypes = [ctypes.c_int, _fp, _fp]
    L.or_hier_create.argtypes = [ctypes.c_int, ctypes.c_int, _dp]
    L.or_hier_create.restype = ctypes.c_void_p
    L.or_hier_create_bc.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int]
    L.or_hier_create_bc.restype = ctypes.c_void_p
    L.or_assemble_bc.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp]
    L.or_load_vector_bc.argtypes = [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, _dp]
    L.or_l2_error.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int]
    L.or_l2_error.restype = ctypes.c_double
    L.or_restrict_bc.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int]
    L.or_restrict_f32_bc.argtypes = [ctypes.c_int, _fp, _fp, ctypes.c_int]
    L.or_hier_destroy.argtypes = [ctypes.c_void_p]
    L.or_hier_N.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.or_hier_bands.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.or_hier_bands.restype = _dp
    L.or_hier_coords.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.or_hier_coords.restype = _dp
    L.or_vcycle.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, ctypes.POINTER(OrOpts)]
    L.or_solve_fp64.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.POINTER(OrOpts),
                                ctypes.POINTER(OrStats)]
    L.or_solve_mixed_emulated.argtypes = [ctypes.c_void_p, _dp, _dp,
                                          ctypes.POINTER(OrOpts), ctypes.POINTER(OrStats)]
    L.or_axpy.argtypes = [ctypes.c_size_t, ctypes.c_double, _dp, _dp]
    L.or_band4_combine.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_dp),
                                   ctypes.c_size_t, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(_dp), _dp, _dp, _dp]
    L.or_dot.argtypes = [ctypes.c_size_t, _dp, _dp]
    L.or_dot.restype = ctypes.c_double
    L.or_cg.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int]
    L.or_cg.restype = ctypes.c_int
    L.or_solve_pcg.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.POINTER(OrOpts),
                               ctypes.c_int, ctypes.POINTER(OrStats)]
    L.or_threads.argtypes = []
    L.or_threads.restype = ctypes.c_int
    return L


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f(a: np.ndarray):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(_fp)


def opts(nu_pre=2, nu_post=2, omega=0.7, rel_tol=1e-8, max_cycles=100, fixed_cycles=0,
         inner_reduction=1e-2, inner_max_cycles=8, coarse_cg=False, coarse_tol=1e-10,
         coarse_max_iter=200) -> OrOpts:
    return OrOpts(nu_pre, nu_post, omega, rel_tol, max_cycles, fixed_cycles,
                  inner_reduction, inner_max_cycles, int(coarse_cg), coarse_tol, coarse_max_iter)


def element_stiffness(xq, yq) -> np.ndarray:
    xq = np.ascontiguousarray(xq, dtype=np.float64)
    yq = np.ascontiguousarray(yq, dtype=np.float64)
    K = np.zeros(16)
    lib().or_element_stiffness(_d(xq), _d(yq), _d(K))
    return K.reshape(4, 4)


ALL_DIRICHLET = 15  # Dirichlet side bits: 1 x = 0, 2 x = 1, 4 y = 0, 8 y = 1


def assemble(N: int, xy: np.ndarray, dirichlet: bool = True, dmask: int | None = None):
    """Bands of the stiffness matrix; Dirichlet treatment on the sides in
    ``dmask`` (default: every side if ``dirichlet``, none otherwise)."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    bands = np.zeros(9 * N * N)
    if dmask is None:
        dmask = ALL_DIRICHLET if dirichlet else 0
    lib().or_assemble_bc(N, _d(xy), int(dmask), _d(bands))
    return bands.reshape(9, N * N)


def load_vector(N: int, xy: np.ndarray, fn: int = 0, dirichlet: bool = True,
                dmask: int | None = None) -> np.ndarray:
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    b = np.zeros(N * N)
    if dmask is None:
        dmask = ALL_DIRICHLET if dirichlet else 0
    lib().or_load_vector_bc(N, _d(xy), fn, int(dmask), _d(b))
    return b


def l2_error_sinsin(N: int, xy: np.ndarray, u: np.ndarray) -> float:
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    return lib().or_l2_error_sinsin(N, _d(xy), _d(np.ascontiguousarray(u)))


def l2_error(N: int, xy: np.ndarray, u: np.ndarray, fn: int) -> float:
    """L2 error against the exact solution of manufactured load ``fn``."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    return lib().or_l2_error(N, _d(xy), _d(np.ascontiguousarray(u)), fn)


def spmv(N, bands, x):
    y = np.zeros(N * N)
    lib().or_spmv(N, _d(np.ascontiguousarray(bands).reshape(-1)), _d(x), _d(y))
    return y


def defect(N, bands, b, x):
    d = np.zeros(N * N)
    lib().or_defect(N, _d(np.ascontiguousarray(bands).reshape(-1)), _d(b), _d(x), _d(d))
    return d


def jacobi(N, bands, b, x, omega=0.7):
    y = np.zeros(N * N)
    lib().or_jacobi(N, _d(np.ascontiguousarray(bands).reshape(-1)), _d(b), _d(x), _d(y), omega)
    return y


def restrict(Nf, d_f, filter=True, dmask: int | None = None):
    Nc = (Nf - 1) // 2 + 1
    bc = np.zeros(Nc * Nc)
    if dmask is None:
        dmask = ALL_DIRICHLET if filter else 0
    lib().or_restrict_bc(Nf, _d(d_f), _d(bc), int(dmask))
    return bc


def prolong_add(Nf, x_c, x_f):
    out = np.array(x_f, dtype=np.float64, copy=True)
    lib().or_prolong_add(Nf, _d(np.ascontiguousarray(x_c)), _d(out))
    return out


def norm2(v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().or_norm2(v.size, _d(v))


def cholesky(A: np.ndarray):
    Lf = np.array(A, dtype=np.float64, copy=True, order="C")
    rc = lib().or_cholesky(Lf.shape[0], _d(Lf))
    return rc, Lf


def spmv_f32(N, bands32, x32):
    y = np.zeros(N * N, dtype=np.float32)
    lib().or_spmv_f32(N, _f(np.ascontiguousarray(bands32).reshape(-1)), _f(x32), _f(y))
    return y


def jacobi_f32(N, bands32, b32, x32, omega=0.7):
    y = np.zeros(N * N, dtype=np.float32)
    lib().or_jacobi_f32(N, _f(np.ascontiguousarray(bands32).reshape(-1)), _f(b32), _f(x32),
                        _f(y), omega)
    return y


def restrict_f32(Nf, d_f32, dmask: int = ALL_DIRICHLET):
    Nc = (Nf - 1) // 2 + 1
    bc = np.zeros(Nc * Nc, dtype=np.float32)
    lib().or_restrict_f32_bc(Nf, _f(d_f32), _f(bc), int(dmask))
    return bc


def prolong_add_f32(Nf, x_c32, x_f32):
    out = np.array(x_f32, dtype=np.float32, copy=True)
    lib().or_prolong_add_f32(Nf, _f(np.ascontiguousarray(x_c32)), _f(out))
    return out


class Hierarchy:
    """Oracle multigrid hierarchy on the finest coordinates ``xy`` (2*n)."""

    def __init__(self, L: int, xy: np.ndarray, Lc: int = 1, dmask: int = ALL_DIRICHLET,
                 threaded: bool = False):
        """threaded: run on the OpenMP build (all host cores; same results)."""
        self.L, self.Lc, self.dmask = L, Lc, dmask
        self._lib = lib_omp() if threaded else lib()
        self._xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
        self._h = self._lib.or_hier_create_bc(L, Lc, _d(self._xy), int(dmask))
        if not self._h:
            raise ValueError("oracle hierarchy creation failed (L=%d, Lc=%d, dmask=%d)"
                             % (L, Lc, dmask))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.or_hier_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def N(self, l: int) -> int:
        return (1 << l) + 1

    def bands(self, l: int) -> np.ndarray:
        n = self.N(l) ** 2
        ptr = self._lib.or_hier_bands(self._h, l)
        return np.ctypeslib.as_array(ptr, shape=(9 * n,)).copy().reshape(9, n)

    def coords(self, l: int) -> np.ndarray:
        n = self.N(l) ** 2
        ptr = self._lib.or_hier_coords(self._h, l)
        return np.ctypeslib.as_array(ptr, shape=(2 * n,)).copy()

    def vcycle(self, l: int, x: np.ndarray, b: np.ndarray, o: OrOpts | None = None):
        x = np.array(x, dtype=np.float64, copy=True)
        self._lib.or_vcycle(self._h, l, _d(x), _d(np.ascontiguousarray(b)),
                        ctypes.byref(o or opts()))
        return x

    def solve_fp64(self, b: np.ndarray, x0: np.ndarray | None = None, o: OrOpts | None = None):
        n = self.N(self.L) ** 2
        x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        st = OrStats()
        self._lib.or_solve_fp64(self._h, _d(np.ascontiguousarray(b)), _d(x),
                            ctypes.byref(o or opts()), ctypes.byref(st))
        return x, st

    def solve_pcg(self, b, x0=None, o: OrOpts | None = None, precond32: bool = False):
        """CG preconditioned by one V-cycle (FP64, or FP32 with precond32)."""
        n = self.N(self.L) ** 2
        x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        st = OrStats()
        self._lib.or_solve_pcg(self._h, _d(np.ascontiguousarray(b)), _d(x),
                           ctypes.byref(o or opts()), int(precond32), ctypes.byref(st))
        return x, st

    def solve_mixed_emulated(self, b, x0=None, o: OrOpts | None = None):
        n = self.N(self.L) ** 2
        x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        st = OrStats()
        self._lib.or_solve_mixed_emulated(self._h, _d(np.ascontiguousarray(b)), _d(x),
                                      ctypes.byref(o or opts()), ctypes.byref(st))
        return x, st


def cg(N, bands, b, x0=None, tol=1e-10, max_iter=200):
    """Unpreconditioned CG on one level's banded system; returns (x, steps)."""
    x = np.zeros(N * N) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    k = lib().or_cg(N, _d(np.ascontiguousarray(bands, dtype=np.float64).reshape(-1)),
                    _d(np.ascontiguousarray(b, dtype=np.float64)), _d(x), tol, max_iter)
    return x, k


def axpy(alpha, x, y):
    """y = alpha x + y (Sec. 6.1).  FP64 inputs: FP64 arithmetic in index
    order.  FP32 inputs: alpha rounded to FP32, then alpha x + y evaluated
    in FP64 (the product is exact there) and rounded once to FP32."""
    if np.asarray(x).dtype == np.float32:
        a32 = float(np.float32(alpha))
        return (a32 * x.astype(np.float64) + y.astype(np.float64)).astype(np.float32)
    out = np.array(y, dtype=np.float64, copy=True)
    lib().or_axpy(out.size, float(alpha), _d(np.ascontiguousarray(x, dtype=np.float64)), _d(out))
    return out


def band4_combine(bands, offsets, vs, u, s=None):
    """u + sum_i M_i v_i (+ s) for four-band M_i: bands[i] has shape (4, n),
    offsets[i] four ints, vs[i] a vector of n (Sec. 2.2 prediction step)."""
    n = len(u)
    m = len(bands)
    bs_ = [np.ascontiguousarray(b, dtype=np.float64).reshape(-1) for b in bands]
    vs_ = [np.ascontiguousarray(v, dtype=np.float64) for v in vs]
    off = (ctypes.c_int * (4 * m))(*[int(o) for row in offsets for o in row])
    bp = (_dp * m)(*[_d(b) for b in bs_])
    vp = (_dp * m)(*[_d(v) for v in vs_])
    ud = np.ascontiguousarray(u, dtype=np.float64)
    sd = None if s is None else np.ascontiguousarray(s, dtype=np.float64)
    out = np.zeros(n)
    lib().or_band4_combine(n, m, bp, n, off, vp, _d(ud), None if sd is None else _d(sd), _d(out))
    return out


def dot(x, y) -> float:
    """x . y in FP64, summed in index order (FP32 inputs widened exactly)."""
    xd = np.ascontiguousarray(x, dtype=np.float64)
    yd = np.ascontiguousarray(y, dtype=np.float64)
    return lib().or_dot(xd.size, _d(xd), _d(yd))


def hist(st: OrStats):
    return [st.res_hist[i] for i in range(st.n_hist)]
