"""FP32 inner BiCGStab with FP64 iterative refinement (the precision tier).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Not a method of the paper: the paper's methods are FP64 throughout. The tier
keeps the matrix and the Krylov vectors in FP32 and wins the accuracy back by
classical iterative refinement (Wilkinson / Moler): with x the FP64 iterate,

    r = b - A x                     (FP64 matrix and arithmetic)
    solve A d = r / ||r||           (inner BiCGStab in FP32 storage, to a loose tolerance)
    x = x + ||r|| d                 (FP64)

until ||b - A x|| < tol ||b||. The inner solve is the merged classical method
(Alg. 2, or Alg. 5 with Jacobi) with FP32 vectors and an FP32 matrix: every
vector update is evaluated in FP64 from FP32 operands and rounded once to
FP32 when stored, the sparse product accumulates in FP32, dot products
accumulate in FP64, scalars are FP64, and the inner solution d is FP64.
"""
from __future__ import annotations

import numpy as np

from .bicgstab import BREAKDOWN, CONVERGED, MAXIT, NONFINITE


def _f32(v):
    return np.asarray(v, dtype=np.float64).astype(np.float32)


def _dot(u, w) -> float:
    return float(np.dot(np.asarray(u, np.float64), np.asarray(w, np.float64)))


def inner_merged_fp32(A32, diag32, b32, tol, maxit):
    """Alg. 2 / Alg. 5 on float32 storage from d_0 = 0. A32: float32 CSR;
    diag32: float32 diagonal for Jacobi or None. Returns (d float64, passes,
    status)."""
    n = b32.shape[0]
    d = np.zeros(n)
    M = (lambda u: (u / diag32).astype(np.float32)) if diag32 is not None else (lambda u: u)
    bb = _dot(b32, b32)
    if bb == 0.0:
        return d, 0, CONVERGED
    eps2 = tol * tol * bb
    r = b32.copy()  # r_0 = b - A d_0 with d_0 = 0
    r0 = r.copy()
    rho = _dot(r, r)
    if rho < eps2:
        return d, 0, CONVERGED
    p = r.copy()
    for j in range(maxit):
        ph = M(p)
        v = (A32 @ ph).astype(np.float32)
        delta = _dot(v, r0)
        if delta == 0.0:
            return d, j + 1, BREAKDOWN
        alpha = rho / delta
        s = _f32(r.astype(np.float64) - alpha * v.astype(np.float64))
        sh = M(s)
        t = (A32 @ sh).astype(np.float32)
        phi, psi, theta = _dot(t, s), _dot(t, t), _dot(s, s)
        omega = phi / psi if psi != 0.0 else 0.0
        est = theta - omega * phi
        if not (np.isfinite(omega) and np.isfinite(est)):
            return d, j + 1, NONFINITE
        d = d + alpha * ph.astype(np.float64) + omega * sh.astype(np.float64)
        r = _f32(s.astype(np.float64) - omega * t.astype(np.float64))
        if est < eps2:
            return d, j + 1, CONVERGED
        rho_next = _dot(r, r0)
        if omega == 0.0 or rho_next == 0.0:
            return d, j + 1, BREAKDOWN
        beta = (rho_next / rho) * (alpha / omega)
        p = _f32(r.astype(np.float64) + beta * (p.astype(np.float64) - omega * v.astype(np.float64)))
        rho = rho_next
    return d, maxit, MAXIT


def refine_solve(A, b, tol=1e-10, inner_tol=1e-5, maxit=5000, max_outer=30, precond="none"):
    """One right-hand side. Returns dict(x, outer, inner_iters, status,
    relres_history)."""
    import scipy.sparse as sp

    A = sp.csr_matrix(A)
    A32 = A.astype(np.float32)
    diag32 = A.diagonal().astype(np.float32) if precond == "jacobi" else None
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    hist = []
    inner_total = 0
    if not np.isfinite(bn):
        return {"x": x, "outer": 0, "inner_iters": 0, "status": NONFINITE, "relres_history": hist}
    if bn == 0.0:
        return {"x": x, "outer": 0, "inner_iters": 0, "status": CONVERGED, "relres_history": [0.0]}
    for outer in range(max_outer + 1):
        r = b - A @ x
        rn = np.linalg.norm(r)
        hist.append(rn / bn)
        if rn * rn < tol * tol * (bn * bn):
            return {"x": x, "outer": outer, "inner_iters": inner_total, "status": CONVERGED, "relres_history": hist}
        if outer == max_outer or inner_total >= maxit:
            break
        d, its, st = inner_merged_fp32(A32, diag32, _f32(r / rn), inner_tol, maxit)
        inner_total += its
        x = x + rn * d
    return {"x": x, "outer": max_outer, "inner_iters": inner_total, "status": MAXIT, "relres_history": hist}
