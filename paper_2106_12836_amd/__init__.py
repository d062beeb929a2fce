"""SAIT on MI355X: sparse approximate inverses of triangular ILU factors
(Lu, arXiv 2106.12836) built and applied with HIP kernels for gfx950.

The library (libsait.so, C ABI in include/sait.h) is loaded lazily on the
first call; importing the package needs no GPU.
"""

from .sait import (  # noqa: F401
    EXPORTED,
    PRECISIONS,
    SaitError,
    SaitPreconditioner,
    SolveResult,
    default_build_opts,
    default_eig_opts,
    default_solve_opts,
    lib,
    library_path,
    sait_apply,
    sait_autotune,
    sait_build,
    sait_copy,
    sait_debug_step,
    sait_destroy,
    sait_export,
    sait_get_apply_lanes,
    sait_grad_values,
    sait_last_error,
    sait_matvec,
    sait_query,
    sait_set_apply_lanes,
    sait_lobpcg,
    sait_set_preconditioner,
    sait_set_values,
    sait_solve,
    sait_time_apply,
)
from .autograd import SaitSolve, sait_solve_autograd  # noqa: F401
