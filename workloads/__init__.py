"""Seeded synthetic inputs for the TA / CTA solvers.

This package builds matrices and right-hand sides only.  It holds none of the
solvers' arithmetic, so both the CPU oracle and the GPU library can take their
inputs from it.
"""
from .gen import (  # noqa: F401
    Csr,
    Problem,
    csr_from_coo,
    csr_from_dense,
    dense_gaussian,
    convection_diffusion,
    kac_clement,
    lp_shaped,
    poisson5,
    random_diag_dominant,
    skewed_rows,
    batched_uneven,
    perturbed_stencil,
    ladder,
)
