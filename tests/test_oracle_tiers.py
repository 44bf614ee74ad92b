"""Pins for the oracle's precision tier (FP32 inner solves with FP64
refinement) and adjoint (gradient of a linear solve): against LAPACK dense
solves, exact-arithmetic facts of refinement, torch autograd of a dense solve,
and central finite differences."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import CONVERGED
from oracle import refine as orf
from workloads import conv_diff, random_27pt


def test_refine_reaches_fp64_accuracy():
    """FP32 inner solves + FP64 refinement reach a 1e-12 relative residual
    (far below FP32's 6e-8) and the dense solution within kappa * tol."""
    A = random_27pt(10, seed=1)
    S = A.to_scipy()
    rng = np.random.default_rng(3)
    b = rng.uniform(-1, 1, A.n)
    res = orf.refine_solve(S, b, tol=1e-12, inner_tol=1e-5)
    assert res["status"] == CONVERGED
    xd = np.linalg.solve(S.toarray(), b)
    kappa = np.linalg.cond(S.toarray())
    assert np.linalg.norm(b - S @ res["x"]) / np.linalg.norm(b) < 1e-12
    assert np.linalg.norm(res["x"] - xd) / np.linalg.norm(xd) <= 2 * kappa * 1e-12
    # an FP32 solve alone cannot get there
    assert res["outer"] >= 2


def test_refine_contraction_per_outer_step():
    """Each correction reduces the FP64 residual by about the inner tolerance
    (plus FP32 rounding of order kappa u_32): the history contracts by >= 1e3
    per step for tau = 1e-5 on a well-conditioned matrix."""
    A = random_27pt(10, seed=2)
    S = A.to_scipy()
    b = np.random.default_rng(4).uniform(-1, 1, A.n)
    res = orf.refine_solve(S, b, tol=1e-13, inner_tol=1e-5)
    h = res["relres_history"]
    assert res["status"] == CONVERGED and len(h) >= 3
    for a, c in zip(h[:-1], h[1:]):
        assert c < a * 1e-3, h
    assert res["outer"] <= 4


def test_refine_inner_solve_meets_tolerance():
    """The FP32 inner solve reaches its own tolerance on the scaled residual."""
    A = conv_diff(12, 3, (1.0, 0.7, 0.3))
    S = A.to_scipy()
    b = np.random.default_rng(5).uniform(-1, 1, A.n)
    rs = (b / np.linalg.norm(b)).astype(np.float32)
    d, its, st = orf.inner_merged_fp32(S.astype(np.float32), None, rs, 1e-5, 1000)
    assert st == CONVERGED
    assert np.linalg.norm(rs.astype(np.float64) - S @ d) < 2e-5


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_refine_matches_dense_solve(precond):
    A = conv_diff(8, 3, (1.0, 0.7, 0.3))
    S = A.to_scipy()
    b = np.random.default_rng(6).uniform(-1, 1, A.n)
    res = orf.refine_solve(S, b, tol=1e-11, inner_tol=1e-4, precond=precond)
    xd = np.linalg.solve(S.toarray(), b)
    assert res["status"] == CONVERGED
    assert np.linalg.norm(res["x"] - xd) / np.linalg.norm(xd) < 1e-9


def test_refine_zero_rhs():
    A = conv_diff(6, 2, (1.0, 0.5)).to_scipy()
    res = orf.refine_solve(A, np.zeros(A.shape[0]))
    assert res["status"] == CONVERGED and np.all(res["x"] == 0) and res["outer"] == 0


# --------------------------------------------------------------- adjoint ---

from oracle import adjoint as oad  # noqa: E402
from workloads import generators as wg  # noqa: E402


def _dense_autograd_grad(A, B):
    """d/dvalues of sum ||A^{-1} B||^2 by torch autograd through a dense FP64
    solve (CPU)."""
    import torch

    rows = torch.as_tensor(A.row_of_entry())
    cols = torch.as_tensor(A.col_idx.astype(np.int64))
    vals = torch.tensor(A.values, dtype=torch.float64, requires_grad=True)
    Ad = torch.zeros(A.n, A.n, dtype=torch.float64).index_put((rows, cols), vals)
    X = torch.linalg.solve(Ad, torch.as_tensor(B))
    (X * X).sum().backward()
    return vals.grad.numpy()


@pytest.mark.parametrize("case", ["diffusion_spd", "convdiff_nonsym"])
def test_adjoint_matches_dense_autograd(case):
    """The pattern-restricted -Lambda X^T equals torch autograd of a dense
    solve; the nonsymmetric case catches an A vs A^T mix-up that a symmetric
    matrix would hide."""
    if case == "diffusion_spd":
        A, _ = wg.diffusion_varcoef(6, seed=1)
    else:
        A = conv_diff(5, 3, (3.0, -2.0, 1.5))
    B = np.random.default_rng(7).uniform(-1, 1, (A.n, 3))
    Xd = np.linalg.solve(A.to_scipy().toarray(), B)
    X, lam, g = oad.solve_and_grad(A.to_scipy(), B, 2 * Xd)  # dL/dX of sum ||X||^2
    ref = _dense_autograd_grad(A, B)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-9


def test_pattern_grad_definition():
    """Brute force: grad[e] = -sum_c lam[i, c] x[j, c], entry by entry."""
    A = conv_diff(3, 2, (1.0, 0.5))
    rng = np.random.default_rng(8)
    lam = rng.uniform(-1, 1, (A.n, 2))
    X = rng.uniform(-1, 1, (A.n, 2))
    g = oad.pattern_grad(A.to_scipy(), lam, X)
    rows = A.row_of_entry()
    for e in range(A.nnz):
        i, j = rows[e], A.col_idx[e]
        assert g[e] == pytest.approx(-(lam[i, 0] * X[j, 0] + lam[i, 1] * X[j, 1]), rel=1e-15, abs=1e-15)


def test_adjoint_finite_differences_through_assembly():
    """dL/dfield for L = sum ||x(field)||^2, with the conductivity assembly
    differentiated by torch and the solve by the adjoint, matches central
    differences along random directions (solves by SciPy's direct solver)."""
    import scipy.sparse.linalg as spla
    import torch

    g0 = 6
    A, field = wg.diffusion_varcoef(g0, seed=2)
    assemble = wg.diffusion_values_torch(A, g0)
    B = np.random.default_rng(9).uniform(-1, 1, (A.n, 2))

    def loss(fld):
        vals = wg.diffusion_values_numpy(A, fld, g0)
        M = wg.CSR(A.n, A.row_ptr, A.col_idx, vals).to_scipy().tocsc()
        Xs = spla.spsolve(M, B)
        return float((Xs * Xs).sum())

    S = A.to_scipy()
    Xs = spla.spsolve(S.tocsc(), B)
    _, lam, gvals = oad.solve_and_grad(S, B, 2 * Xs)
    ft = torch.tensor(field, dtype=torch.float64, requires_grad=True)
    (assemble(ft) * torch.as_tensor(gvals)).sum().backward()
    grad_field = ft.grad.numpy()
    rng = np.random.default_rng(10)
    h = 1e-6
    for _ in range(3):
        d = rng.standard_normal(A.n)
        fd = (loss(field + h * d) - loss(field - h * d)) / (2 * h)
        an = grad_field @ d
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
