"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This package builds matrices and right-hand sides only. It holds none of the
solver's arithmetic: no Krylov step, no preconditioner, no reduction.
"""
from .generators import (  # noqa: F401
    CSR,
    conv_diff,
    conv_diff_2d,
    conv_diff_3d,
    poisson_3d,
    random_27pt,
    random_sparse,
    diffusion_varcoef,
    batched_systems,
    manufactured_rhs,
    config_problem,
)
