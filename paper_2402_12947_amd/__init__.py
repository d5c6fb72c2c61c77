"""Global-local multigrid-preconditioned CG for FE Poisson problems on MI355X.

The numerical work runs in the gfx950 HIP library libmgpcg.so (C ABI in
include/mgpcg.h); this package is its ctypes binding.  See `binding.Solver`.
"""
from .binding import (MG_ERR_ARG, MG_ERR_BREAKDOWN, MG_ERR_HIP, MG_ERR_LIMIT, MG_ERR_LOCATE, MG_ERR_MESH,
                      MG_ERR_NOT_SPD, MG_ERR_OOM, MG_NOT_CONVERGED, MG_OK, MgError, Solver, lib, load_library,
                      pcg_solve_batch, setup_status)

__all__ = ["Solver", "MgError", "pcg_solve_batch", "lib", "load_library", "setup_status", "MG_OK", "MG_NOT_CONVERGED",
           "MG_ERR_ARG", "MG_ERR_MESH", "MG_ERR_LOCATE", "MG_ERR_NOT_SPD", "MG_ERR_BREAKDOWN", "MG_ERR_HIP",
           "MG_ERR_OOM", "MG_ERR_LIMIT"]
