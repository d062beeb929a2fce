"""Seeded synthetic workloads for the SAIT hot path.

This package only *builds inputs*: sparse test matrices in CSR form
(int32 row pointers and column indices, float64 values) and right-hand
sides.  It contains none of the method's arithmetic (no ILU, no SAIT
series, no Krylov solver), so both the CPU oracle and the GPU library can
consume it without sharing any implementation of the method.
"""

from .generators import (  # noqa: F401
    Csr,
    poisson2d,
    poisson3d,
    convdiff2d_upwind,
    aniso2d,
    batched_aniso2d,
    grf_diffusion2d,
    gaussian_random_field,
    random_diag_dominant,
    random_triangular,
    uniform_vector,
    spmv_rhs,
    block_diag,
    config,
)
