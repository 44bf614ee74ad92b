"""Gradient of a sparse linear solve (the differentiation tier).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Not a method of the paper. For X = A^{-1} B (columns solved independently,
A shared) and a loss L(X) with G = dL/dX, differentiating A X = B gives

    Lambda = A^{-T} G,    dL/dB = Lambda,    dL/dA = -Lambda X^T,

and for the stored entries e = (i, j) of a sparse A only the pattern matters:
dL/dvalues[e] = -sum_c Lambda[i, c] X[j, c]. The solves use the oracle's
BiCGStab (on A^T for Lambda) at a tight tolerance.
"""
from __future__ import annotations

import numpy as np

from .bicgstab import CONVERGED, solve


def pattern_grad(A, lam, X):
    """-sum_c lam[i_e, c] X[j_e, c] for every stored entry e of CSR A."""
    import scipy.sparse as sp

    A = sp.csr_matrix(A)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    lam = np.asarray(lam).reshape(A.shape[0], -1)
    X = np.asarray(X).reshape(A.shape[0], -1)
    return -np.einsum("ec,ec->e", lam[rows], X[A.indices])


def solve_and_grad(A, B, G, tol=1e-13, maxit=5000, variant="classical", precond="none"):
    """Returns (X, Lambda, grad_values) with the solves done by the oracle
    BiCGStab; raises if a column does not converge."""
    import scipy.sparse as sp

    A = sp.csr_matrix(A)
    fx = solve(A, B, variant=variant, formulation="merged", precond=precond, tol=tol, maxit=maxit)
    fl = solve(A.T.tocsr(), G, variant=variant, formulation="merged", precond=precond, tol=tol, maxit=maxit)
    if not (np.all(fx.status == CONVERGED) and np.all(fl.status == CONVERGED)):
        raise RuntimeError("adjoint oracle: a solve did not converge")
    return fx.x, fl.x, pattern_grad(A, fl.x, fx.x)
