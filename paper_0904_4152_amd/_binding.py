"""ctypes marshalling for libmgfem.so (see include/mgfem.h for semantics)."""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime the library links against (one runtime per process)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmgfem.so")

MG_OK, MG_ERR_INVALID, MG_ERR_NOMEM, MG_ERR_NOCONV, MG_ERR_NUMERIC, MG_ERR_DEVICE, MG_ERR_BUSY = \
    range(7)
MG_PREC_FP64, MG_PREC_MIXED = 0, 1
MG_F64, MG_F32 = 0, 1
MG_HIST = 128
# Side bits of dirichlet_sides: x = 0, x = 1, y = 0, y = 1.
SIDE_X0, SIDE_X1, SIDE_Y0, SIDE_Y1 = 1, 2, 4, 8
ALL_DIRICHLET = 15
MG_COARSE_CHOLESKY, MG_COARSE_CG = 0, 1

_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_sz = ctypes.c_size_t
_u64 = ctypes.c_uint64
_i64 = ctypes.c_int64


class SolveOpts(ctypes.Structure):
    _fields_ = [("nu_pre", _i), ("nu_post", _i), ("omega", _d), ("rel_tol", _d),
                ("max_cycles", _i), ("precision", _i), ("inner_reduction", _d),
                ("inner_max_cycles", _i), ("fixed_cycles", _i), ("use_graph", _i),
                ("krylov", _i), ("zero_guess", _i)]


class TileChoice(ctypes.Structure):
    _fields_ = [("level", _i), ("problems", _i), ("tile_rows", _i), ("row_waves", _i),
                ("tile_cols", _i), ("us", _d)]


class Stats(ctypes.Structure):
    _fields_ = [("status", _i), ("cycles", _i), ("outer_steps", _i), ("bnorm", _d),
                ("rel_res", _d), ("seconds", _d), ("alg_bytes", _d), ("n_hist", _i),
                ("res_hist", _d * MG_HIST), ("queue_seconds", _d)]

    def hist(self):
        return [self.res_hist[k] for k in range(self.n_hist)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("completed", _u64), ("queued", _sz), ("live", _i), ("queue_high_water", _sz),
                ("bytes", _sz), ("bytes_high_water", _sz), ("busy_seconds", _d)]


class MgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_status_name(status), msg))
        self.status = status


_SIGS = {
    "mg_default_opts": (None, [ctypes.POINTER(SolveOpts)]),
    "mg_last_error": (ctypes.c_char_p, []),
    "mg_status_string": (ctypes.c_char_p, [_i]),
    "mg_context_create": (_i, [_i, _sz, ctypes.POINTER(_vp)]),
    "mg_context_destroy": (_i, [_vp]),
    "mg_context_memory": (_i, [_vp, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "mg_hierarchy_create": (_i, [_vp, _i, _i, _d, _u64, _vp, ctypes.POINTER(_vp)]),
    "mg_hierarchy_create_bc": (_i, [_vp, _i, _i, _d, _u64, _vp, _i, ctypes.POINTER(_vp)]),
    "mg_hierarchy_bytes": (_sz, [_i, _i]),
    "mg_hierarchy_set_coarse_solver": (_i, [_vp, _i, _d, _i]),
    "mg_hierarchy_assemble": (_i, [_vp, _vp]),
    "mg_hierarchy_destroy": (_i, [_vp]),
    "mg_hierarchy_info": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i64)]),
    "mg_get_bands": (_i, [_vp, _i, _i, _vp]),
    "mg_get_coords": (_i, [_vp, _i, _vp]),
    "mg_rhs_sinsin": (_i, [_vp, _vp, _vp]),
    "mg_rhs_uniform": (_i, [_vp, _u64, _vp, _vp]),
    "mg_solve": (_i, [_vp, _vp, _vp, ctypes.POINTER(SolveOpts), _vp, ctypes.POINTER(Stats)]),
    "mg_spmv": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "mg_defect": (_i, [_vp, _i, _i, _vp, _vp, _vp, ctypes.POINTER(_d), _vp]),
    "mg_smooth": (_i, [_vp, _i, _i, _vp, _vp, _i, _d, _vp]),
    "mg_jacobi": (_i, [_vp, _i, _i, _vp, _vp, _vp, _d, _vp]),
    "mg_pre_smooth": (_i, [_vp, _i, _i, _vp, _vp, _i, _d, _vp, _vp, _vp]),
    "mg_post_smooth": (_i, [_vp, _i, _i, _vp, _vp, _vp, _d, _vp, ctypes.POINTER(_d), _vp]),
    "mg_restrict": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "mg_prolong": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "mg_coarse_solve": (_i, [_vp, _i, _vp, _vp, _vp]),
    "mg_vcycle": (_i, [_vp, _i, _i, _vp, _vp, _i, _i, _d, _i, _vp]),
    "mg_server_create": (_i, [_vp, _i, _sz, _i, _i, ctypes.POINTER(SolveOpts),
                              ctypes.POINTER(_vp)]),
    "mg_server_submit": (_i, [_vp, _i, _d, _d, _u64, _u64, _i, ctypes.POINTER(_u64)]),
    "mg_server_poll": (_i, [_vp, _u64, _vp, ctypes.POINTER(Stats)]),
    "mg_server_next": (_i, [_vp, _d, ctypes.POINTER(_u64), _vp, ctypes.POINTER(Stats)]),
    "mg_server_info": (_i, [_vp, ctypes.POINTER(ServerInfo)]),
    "mg_server_destroy": (_i, [_vp]),
    "mg_axpy": (_i, [_vp, _i, _i64, _d, _vp, _vp, _vp]),
    "mg_dot": (_i, [_vp, _i, _i64, _vp, _vp, ctypes.POINTER(_d), _vp]),
    "mg_norm2": (_i, [_vp, _i, _i64, _vp, ctypes.POINTER(_d), _vp]),
    "mg_dot_noalloc": (_i, [_vp, _i, _i64, _vp, _vp, _vp, _vp]),
    "mg_band4_combine": (_i, [_vp, _i, _i64, _i, ctypes.POINTER(_vp), _i64, ctypes.POINTER(_i),
                              ctypes.POINTER(_vp), _vp, _vp, _vp, _vp]),
    "mg_batch_autotune": (_i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(SolveOpts), _i,
                               ctypes.POINTER(TileChoice), _i, ctypes.POINTER(_i)]),
    "mg_batch_set_tile": (_i, [_i, _i, _i, _i, _i]),
    "mg_batch_clear_tiles": (_i, []),
    "mg_hierarchy_autotune": (_i, [_vp, _i, ctypes.POINTER(TileChoice), _i, ctypes.POINTER(_i)]),
    "mg_solve_batch": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i,
                            ctypes.POINTER(SolveOpts), _vp, ctypes.POINTER(Stats)]),
}

_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError("libmgfem.so is not built (run __graft_entry__.build() or "
                              "python paper_0904_4152_amd/build.py)")
        L = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _status_name(s: int) -> str:
    try:
        return lib().mg_status_string(s).decode()
    except Exception:  # library not loadable
        return "status %d" % s


def check(status: int) -> int:
    if status != MG_OK:
        raise MgError(status, lib().mg_last_error().decode())
    return status


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().mg_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _ptr_array(ts):
    """Device addresses of a list of contiguous device tensors, as a C array
    (the batched calls marshal hundreds per call)."""
    addrs = []
    for t in ts:
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("expected contiguous device tensors")
        addrs.append(t.data_ptr())
    return (_vp * len(addrs))(*addrs)


def _dt(t) -> int:
    if t.dtype == torch.float64:
        return MG_F64
    if t.dtype == torch.float32:
        return MG_F32
    raise TypeError("tensors must be float64 or float32")


class Context:
    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = _vp()
        check(lib().mg_context_create(device, budget_bytes, ctypes.byref(h)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def memory(self):
        a, b = _sz(), _sz()
        check(lib().mg_context_memory(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def axpy(self, alpha: float, x, y, stream=None):
        """y = alpha x + y on device vectors of equal length (BLAS level 1)."""
        if x.numel() != y.numel() or x.dtype != y.dtype:
            raise ValueError("x and y must have the same length and dtype")
        check(lib().mg_axpy(self._h, _dt(x), x.numel(), alpha, _ptr(x), _ptr(y),
                            _stream(stream)))

    def dot(self, x, y, stream=None) -> float:
        if x.numel() != y.numel() or x.dtype != y.dtype:
            raise ValueError("x and y must have the same length and dtype")
        out = _d()
        check(lib().mg_dot(self._h, _dt(x), x.numel(), _ptr(x), _ptr(y), ctypes.byref(out),
                           _stream(stream)))
        return out.value

    def dot_noalloc(self, x, y, out, stream=None):
        """out[0] = x . y (device float64 tensor), asynchronously; allocates
        nothing (mg_dot_noalloc)."""
        if x.numel() != y.numel() or x.dtype != y.dtype:
            raise ValueError("x and y must have the same length and dtype")
        if out.dtype != torch.float64 or out.numel() < 1:
            raise ValueError("out must be a float64 device tensor with at least one element")
        check(lib().mg_dot_noalloc(self._h, _dt(x), x.numel(), _ptr(x), _ptr(y), _ptr(out),
                                   _stream(stream)))

    def band4_combine(self, bands, offsets, vs, u, u_new, s=None, stream=None):
        """u_new = u + sum_i M_i v_i (+ s): bands[i] a device tensor of shape
        (4, n) or (4, stride), offsets[i] four ints, vs[i] device vectors."""
        m = len(bands)
        n = u.numel()
        stride = bands[0].shape[-1]
        for b in bands:
            if b.dim() != 2 or b.shape[0] != 4 or b.shape[1] != stride or not b.is_contiguous():
                raise ValueError("bands must be contiguous (4, stride) tensors of one stride")
        bp = (_vp * m)(*[b.data_ptr() for b in bands])
        vp = (_vp * m)(*[v.data_ptr() for v in vs])
        off = (_i * (4 * m))(*[int(o) for row in offsets for o in row])
        check(lib().mg_band4_combine(self._h, _dt(u), n, m, bp, stride, off, vp, _ptr(u),
                                     _ptr(s) if s is not None else None, _ptr(u_new),
                                     _stream(stream)))

    def norm2(self, x, stream=None) -> float:
        out = _d()
        check(lib().mg_norm2(self._h, _dt(x), x.numel(), _ptr(x), ctypes.byref(out),
                             _stream(stream)))
        return out.value

    def close(self):
        if self._h:
            lib().mg_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hierarchy:
    """Device hierarchy; methods call the C ABI with tensor pointers."""

    def __init__(self, ctx: Context, L: int, coarse_level: int = 1, jitter: float = 0.0,
                 seed: int = 0, xy=None, assemble: bool = True,
                 dirichlet_sides: int = ALL_DIRICHLET):
        h = _vp()
        xy_ptr = None
        if xy is not None:
            import numpy as np
            self._xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
            xy_ptr = self._xy.ctypes.data_as(_vp)
        check(lib().mg_hierarchy_create_bc(ctx.handle, L, coarse_level, jitter, seed, xy_ptr,
                                           dirichlet_sides, ctypes.byref(h)))
        self._h = h
        self.dirichlet_sides = dirichlet_sides
        self.ctx = ctx
        self.L = L
        self.Lc = coarse_level
        self.N = (1 << L) + 1
        self.n = self.N * self.N
        if assemble:
            self.assemble()

    @staticmethod
    def bytes_needed(L: int, coarse_level: int = 1) -> int:
        return lib().mg_hierarchy_bytes(L, coarse_level)

    @property
    def handle(self):
        return self._h

    def assemble(self, stream=None):
        check(lib().mg_hierarchy_assemble(self._h, _stream(stream)))

    def set_coarse_solver(self, solver: int, tol: float = 1e-10, max_iter: int = 200):
        check(lib().mg_hierarchy_set_coarse_solver(self._h, solver, tol, max_iter))

    def close(self):
        if self._h:
            lib().mg_hierarchy_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_size(self, l: int) -> int:
        return ((1 << l) + 1) ** 2

    def bands(self, level: int, dtype=torch.float64):
        import numpy as np
        n = self.level_size(level)
        out = np.zeros(9 * n, dtype=np.float64 if dtype == torch.float64 else np.float32)
        check(lib().mg_get_bands(self._h, level, MG_F64 if dtype == torch.float64 else MG_F32,
                                 out.ctypes.data_as(_vp)))
        return out.reshape(9, n)

    def coords(self, level: int):
        import numpy as np
        out = np.zeros(2 * self.level_size(level))
        check(lib().mg_get_coords(self._h, level, out.ctypes.data_as(_vp)))
        return out

    def rhs_sinsin(self, b, stream=None):
        check(lib().mg_rhs_sinsin(self._h, _ptr(b), _stream(stream)))

    def rhs_uniform(self, seed: int, b, stream=None):
        check(lib().mg_rhs_uniform(self._h, seed, _ptr(b), _stream(stream)))

    def solve(self, b, x, opts: SolveOpts | None = None, stream=None, raise_on_error=True):
        st = Stats()
        rc = lib().mg_solve(self._h, _ptr(b), _ptr(x),
                            ctypes.byref(opts) if opts is not None else None, _stream(stream),
                            ctypes.byref(st))
        if raise_on_error:
            check(rc)
        return st

    def spmv(self, level, x, y, stream=None):
        check(lib().mg_spmv(self._h, level, _dt(x), _ptr(x), _ptr(y), _stream(stream)))

    def defect(self, level, b, x, d=None, norm=False, stream=None):
        nv = _d()
        check(lib().mg_defect(self._h, level, _dt(x), _ptr(b), _ptr(x), _ptr(d),
                              ctypes.byref(nv) if norm else None, _stream(stream)))
        return nv.value if norm else None

    def smooth(self, level, b, x, sweeps=1, omega=0.7, stream=None):
        check(lib().mg_smooth(self._h, level, _dt(x), _ptr(b), _ptr(x), sweeps, omega,
                              _stream(stream)))

    def jacobi(self, level, b, x, x_out, omega=0.7, stream=None):
        check(lib().mg_jacobi(self._h, level, _dt(x), _ptr(b), _ptr(x), _ptr(x_out), omega,
                              _stream(stream)))

    def pre_smooth(self, level, b, x, x2, b_c, x_zero=False, omega=0.7, stream=None):
        check(lib().mg_pre_smooth(self._h, level, _dt(b), _ptr(b), _ptr(x), int(x_zero), omega,
                                  _ptr(x2), _ptr(b_c), _stream(stream)))

    def post_smooth(self, level, b, x, x_c, x_out, omega=0.7, norm=False, stream=None):
        nv = _d()
        check(lib().mg_post_smooth(self._h, level, _dt(b), _ptr(b), _ptr(x), _ptr(x_c), omega,
                                   _ptr(x_out), ctypes.byref(nv) if norm else None,
                                   _stream(stream)))
        return nv.value if norm else None

    def restrict(self, fine_level, d_f, b_c, stream=None):
        check(lib().mg_restrict(self._h, fine_level, _dt(d_f), _ptr(d_f), _ptr(b_c),
                                _stream(stream)))

    def prolong(self, fine_level, x_c, x_f, stream=None):
        check(lib().mg_prolong(self._h, fine_level, _dt(x_f), _ptr(x_c), _ptr(x_f),
                               _stream(stream)))

    def coarse_solve(self, b, x, stream=None):
        check(lib().mg_coarse_solve(self._h, _dt(x), _ptr(b), _ptr(x), _stream(stream)))

    def autotune(self, reps=10):
        """Tune the single-problem fused passes' tiles of this hierarchy's
        levels (mg_hierarchy_autotune); returns the choices as dicts."""
        out = (TileChoice * 16)()
        got = _i()
        check(lib().mg_hierarchy_autotune(self._h, reps, out, 16, ctypes.byref(got)))
        return [_choice(out[i]) for i in range(min(got.value, 16))]

    def vcycle(self, level, b, x, nu_pre=2, nu_post=2, omega=0.7, fused=None, stream=None):
        if fused is None:
            fused = nu_pre == 2 and nu_post == 2
        check(lib().mg_vcycle(self._h, level, _dt(x), _ptr(b), _ptr(x), nu_pre, nu_post, omega,
                              int(fused), _stream(stream)))


def _choice(c):
    return {"level": c.level, "problems": c.problems, "tile_rows": c.tile_rows,
            "row_waves": c.row_waves, "tile_cols": c.tile_cols, "us": c.us}


def batch_autotune(hierarchies, opts=None, reps=10):
    """Tune the batched solver's tiles (marching tiles: rows and wavefronts
    per row; block tiles: rows and columns) for this composition; returns the
    choices as dicts (level, problems, tile_rows, row_waves, tile_cols, us)."""
    n = len(hierarchies)
    hs = (_vp * n)(*[h.handle for h in hierarchies])
    out = (TileChoice * 16)()
    got = _i()
    check(lib().mg_batch_autotune(hs, n, ctypes.byref(opts) if opts is not None else None, reps,
                                  out, 16, ctypes.byref(got)))
    return [_choice(out[i]) for i in range(min(got.value, 16))]


def batch_set_tiles(rows):
    """Install tile choices (the rows batch_autotune returns, e.g. from JSON;
    a missing row_waves keeps the width rule, a missing tile_cols means a
    marching tile)."""
    for r in rows:
        check(lib().mg_batch_set_tile(int(r["level"]), int(r["problems"]), int(r["tile_rows"]),
                                      int(r.get("row_waves", 0)), int(r.get("tile_cols", 0))))


def batch_clear_tiles():
    check(lib().mg_batch_clear_tiles())


def save_tiles(rows, path):
    import json
    with open(path, "w") as f:
        json.dump({"tiles": rows}, f, indent=1)


def load_tiles(path):
    """Read a tile file written by save_tiles and install it."""
    import json
    with open(path) as f:
        rows = json.load(f)["tiles"]
    batch_set_tiles(rows)
    return rows


def solve_batch(hierarchies, bs, xs, opts=None, stream=None, raise_on_error=True):
    """mg_solve_batch over lists of Hierarchy objects and device tensors;
    opts: None, one SolveOpts for all, or a list.  Returns the Stats list."""
    n = len(hierarchies)
    H = (_vp * n)(*[h.handle for h in hierarchies])
    B = _ptr_array(bs)
    X = _ptr_array(xs)
    O = None
    if isinstance(opts, (list, tuple)):
        O = (SolveOpts * n)(*opts)
    elif opts is not None:  # one struct for all: n copies in one buffer copy
        O = (SolveOpts * n).from_buffer_copy(bytes(opts) * n)
    S = (Stats * n)()
    rc = lib().mg_solve_batch(H, B, X, n, O, _stream(stream), S)
    if raise_on_error:
        check(rc)
    return list(S)


class Server:
    """mg_server_*: continuous-batching solve service on one device."""

    def __init__(self, ctx: Context, slots: int, budget_bytes: int, max_level: int,
                 coarse_level: int = 1, opts: SolveOpts | None = None):
        h = _vp()
        check(lib().mg_server_create(ctx.handle, slots, budget_bytes, max_level, coarse_level,
                                     ctypes.byref(opts) if opts is not None else None,
                                     ctypes.byref(h)))
        self._h = h
        self.ctx = ctx

    def submit(self, L, rel_tol, jitter, geom_seed, rhs_seed, keep_x=False) -> int:
        t = _u64()
        check(lib().mg_server_submit(self._h, L, rel_tol, jitter, geom_seed, rhs_seed,
                                     int(keep_x), ctypes.byref(t)))
        return t.value

    def poll(self, ticket, n=None):
        """(status, stats, x or None); status MG_ERR_BUSY while pending."""
        import numpy as np
        st = Stats()
        x = np.zeros(n) if n else None
        rc = lib().mg_server_poll(self._h, ticket, x.ctypes.data_as(_vp) if n else None,
                                  ctypes.byref(st))
        if rc not in (MG_OK, MG_ERR_BUSY, MG_ERR_NOCONV, MG_ERR_NUMERIC, MG_ERR_NOMEM):
            check(rc)
        return rc, st, x

    def next(self, timeout=1.0):
        """(ticket, status, stats) of the oldest finished request, or None."""
        st = Stats()
        t = _u64()
        rc = lib().mg_server_next(self._h, timeout, ctypes.byref(t), None, ctypes.byref(st))
        if rc == MG_ERR_BUSY:
            return None
        if rc not in (MG_OK, MG_ERR_NOCONV, MG_ERR_NUMERIC, MG_ERR_NOMEM):
            check(rc)
        return t.value, rc, st

    def info(self) -> ServerInfo:
        i = ServerInfo()
        check(lib().mg_server_info(self._h, ctypes.byref(i)))
        return i

    def close(self):
        if self._h:
            check(lib().mg_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
