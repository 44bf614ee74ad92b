"""CPU FP64 oracle for the multi-RHS BiCGStab solvers.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow reference that the
GPU library is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library itself never calls it,
and it shares no code with the library (no kernels, headers, helpers or
constants). It depends on NumPy/SciPy only.

Contents
--------
bicgstab   per-column BiCGStab in the classical (Alg. 1, 2, 5), Reordered
           (Alg. 6) and Pipelined (Alg. 4, 7) forms of the paper's Appendix B,
           basic and merged, with an optional Jacobi preconditioner.
adjoint    gradient of a linear solve with respect to b and the matrix values.
refine     FP32 inner solve with FP64 iterative refinement.
model      the paper's data-transfer execution-time model (Section 3.1).
"""
from .bicgstab import (  # noqa: F401
    RUNNING,
    CONVERGED,
    MAXIT,
    BREAKDOWN,
    NONFINITE,
    ColumnResult,
    jacobi_preconditioner,
    identity_preconditioner,
    solve_column,
    solve,
)
