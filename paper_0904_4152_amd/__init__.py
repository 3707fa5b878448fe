"""MI355X multigrid Poisson solver (Q1 finite elements, HONEI arXiv 0904.4152).

Thin ctypes binding of ``libmgfem.so`` (C ABI in ``include/mgfem.h``): every
function has the C name and only marshals arguments; all computation runs in
the library's HIP kernels.  Torch supplies device memory and streams.  The
module refuses to load when the built library is missing -- there is no
fallback path.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    MG_OK, MG_ERR_INVALID, MG_ERR_NOMEM, MG_ERR_NOCONV, MG_ERR_NUMERIC, MG_ERR_DEVICE,
    MG_ERR_BUSY, MG_PREC_FP64, MG_PREC_MIXED, MG_F64, MG_F32, SIDE_X0, SIDE_X1, SIDE_Y0, SIDE_Y1,
    ALL_DIRICHLET, MG_COARSE_CHOLESKY, MG_COARSE_CG, MgError, SolveOpts, Stats,
    lib, library_path, default_opts, Context, Hierarchy, check, solve_batch, Server,
    TileChoice, batch_autotune, batch_set_tiles, batch_clear_tiles, save_tiles, load_tiles,
    ServerInfo,
)
