"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates inputs*: the convection-diffusion coefficient
matrix in CSR form, manufactured solutions and right-hand sides, and the
seeded workload families.  It contains none of the solver's arithmetic (no
splitting, no Krylov step, no refinement), so the CPU oracle and the GPU path
can both consume it without sharing any method code.
"""
from .convdiff import (  # noqa: F401
    Csr,
    convdiff,
    convdiff_nnz,
    convdiff_skew_perturbed,
    csr_matvec,
    rhs_for,
    workload,
    batched_family,
    train_family,
    test_family,
    ALPHA_GRID,
    OMEGA_GRID,
)
from .sylvester import paper_tridiag, random_tridiag, sylvester_rhs  # noqa: F401
