"""Pins for the CPU oracle: each checks it against something other than itself
(a LAPACK dense solve, a manufactured solution, identities that hold in exact
arithmetic, special cases with known answers, and numbers the paper prints).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import BREAKDOWN, CONVERGED, MAXIT, NONFINITE, solve, solve_column
from oracle import bicgstab as ob
from oracle import model as om
from workloads import conv_diff, manufactured_rhs, random_sparse

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")
METHODS = [(v, f, p) for v in ("classical", "reordered", "pipelined") for f in ("merged", "basic") for p in ("none", "jacobi")]
# the fused forms with Jacobi fold M^{-1} into the products (A M^{-1} as a
# matrix), a rounding-level change of Alg. 5, 6 and 7; without a
# preconditioner the fused forms run the merged listing
METHODS += [("classical", "fused", "jacobi"), ("reordered", "fused", "jacobi"), ("pipelined", "fused", "jacobi")]


def _tiny_systems():
    out = []
    A = conv_diff(8, 2, (1.0, 0.5))
    out.append(("cd2d_8", A.to_scipy()))
    A = conv_diff(6, 3, (1.0, 0.7, 0.3))
    out.append(("cd3d_6", A.to_scipy()))
    A = random_sparse(50, 10, seed=3)
    out.append(("rand50", A.to_scipy()))
    return out


@pytest.mark.parametrize("name,A", _tiny_systems(), ids=lambda v: v if isinstance(v, str) else "")
@pytest.mark.parametrize("variant,formulation,precond", METHODS)
def test_dense_solve(name, A, variant, formulation, precond):
    """Converged oracle solutions agree with numpy.linalg.solve within the
    bound kappa_2 * tol that the stop test implies."""
    rng = np.random.default_rng(11)
    B = rng.uniform(-1, 1, (A.shape[0], 3))
    Ad = A.toarray()
    Xd = np.linalg.solve(Ad, B)
    kappa = np.linalg.cond(Ad)
    tol = 1e-10
    res = solve(A, B, variant=variant, formulation=formulation, precond=precond, tol=tol, maxit=2000)
    assert np.all(res.status == CONVERGED)
    for c in range(B.shape[1]):
        err = np.linalg.norm(res.x[:, c] - Xd[:, c]) / np.linalg.norm(Xd[:, c])
        assert err <= 2 * kappa * tol, (c, err, kappa)
    assert np.all(res.relres_true <= 1.1 * tol)


def test_manufactured_solution():
    A = conv_diff(16, 2, (1.0, 0.5))
    S = A.to_scipy()
    b, xs = manufactured_rhs(A, 4, seed=5)
    kappa = np.linalg.cond(S.toarray())
    for variant, formulation, precond in METHODS:
        res = solve(S, b, variant=variant, formulation=formulation, precond=precond, tol=1e-10, maxit=2000)
        err = np.linalg.norm(res.x - xs, axis=0) / np.linalg.norm(xs, axis=0)
        assert np.all(res.status == CONVERGED)
        assert np.all(err <= kappa * 1e-10), (variant, formulation, precond, err)


@pytest.mark.parametrize("variant,formulation,precond", METHODS)
def test_residual_gap(variant, formulation, precond):
    """The recursively updated residual stays equal to b - A x_j (up to
    rounding) along the whole run."""
    A = conv_diff(10, 3, (1.0, 0.7, 0.3)).to_scipy()
    rng = np.random.default_rng(2)
    b = rng.uniform(-1, 1, A.shape[0])
    tr = []
    res = solve_column(A, b, None, variant, formulation, precond, 1e-12, 500, trace=tr, trace_vectors=True)
    assert res.status == CONVERGED
    nb = np.linalg.norm(b)
    for rec in tr:
        gap = np.linalg.norm((b - A @ rec["vec"]["x"]) - rec["vec"]["r"]) / nb
        assert gap <= 1e-11, (rec["j"], gap)


def test_classical_merged_estimate_is_residual_norm():
    """theta - omega*phi = (r_{j+1}, r_{j+1}) in exact arithmetic (footnote of
    Section 1): the merged estimate tracks the explicit norm while the residual
    is well above rounding level."""
    A = conv_diff(12, 3, (1.0, 0.7, 0.3)).to_scipy()
    b = np.random.default_rng(4).uniform(-1, 1, A.shape[0])
    for precond in ("none", "jacobi"):
        tr = []
        solve_column(A, b, None, "classical", "merged", precond, 1e-12, 400, trace=tr, trace_vectors=True)
        rr0 = b @ b
        checked = 0
        for rec in tr:
            rr = rec["vec"]["r"] @ rec["vec"]["r"]
            if rr > 1e-8 * rr0:
                assert abs(rec["est"] - rr) <= 1e-7 * rr, (rec["j"], rec["est"], rr)
                checked += 1
        assert checked > 5


def test_reordered_orthogonality():
    """(r-tilde_j, r_0) = 0 in exact arithmetic, which is why Alg. 6 may take
    rho_{j+1} = -omega_j psi_j."""
    A = conv_diff(12, 3, (1.0, 0.7, 0.3)).to_scipy()
    b = np.random.default_rng(6).uniform(-1, 1, A.shape[0])
    tr = []
    solve_column(A, b, None, "reordered", "merged", "jacobi", 1e-12, 30, trace=tr, trace_vectors=True)
    for rec in tr[:15]:
        rt, r0 = rec["vec"]["rt"], rec["vec"]["r0"]
        assert abs(rt @ r0) <= 1e-10 * np.linalg.norm(rt) * np.linalg.norm(r0)


def _reordered_trace(kappa, monkeypatch, g=24, col=19, tol=1e-8):
    """Alg. 6 on the 3D convection-diffusion system with Jacobi, one column,
    with the restart factor set to kappa; returns the trace and the result."""
    monkeypatch.setattr(ob, "RESTART_KAPPA", kappa)
    A = conv_diff(g, 3, (1.0, 0.7, 0.3))
    S = A.to_scipy()
    b = manufactured_rhs(A, 32, seed=0)[0][:, col].copy()
    tr = []
    res = solve_column(S, b, None, "reordered", "merged", "jacobi", tol, 2000, trace=tr, trace_vectors=True)
    return S, b, tr, res


def _true_rho_next(tr):
    """(r_{j+1}, r_0) of every pass, summed exactly (math.fsum) from the stored
    vectors, beside the recurrence's rho_{j+1} (the next record's rho)."""
    import math

    out = []
    for i in range(len(tr) - 1):
        r, r0 = tr[i]["vec"]["r"], tr[i]["vec"]["r0"]
        out.append((tr[i + 1]["rho"], math.fsum(r * r0), tr[i]["restart"]))
    return out


def test_reordered_printed_listing_loses_rho(monkeypatch):
    """Without the restart (factor 0: only an exact zero rho restarts) the
    listing's rho_{j+1} = -omega_j psi_j drifts from the true (r_{j+1}, r_0)
    by an offset that does not shrink with the residual, until the
    recurrence is noise: some pass's rho is off by more than its own size."""
    _, _, tr, res = _reordered_trace(0.0, monkeypatch)
    pairs = _true_rho_next(tr)
    assert not any(rs for _, _, rs in pairs)
    assert any(abs(rho - true) > abs(rho) for rho, true, _ in pairs)


def test_reordered_restart_keeps_rho_informative(monkeypatch):
    """With the restart test, every pass that carries the recurrence on has
    rho_{j+1} within 25% of the exactly summed (r_{j+1}, r_0); a restart takes
    r_{j+1} as the new shadow vector with rho_{j+1} its squared norm (the stop
    estimate) and beta = 0; the solve converges and agrees with a direct
    solve."""
    import math

    S, b, tr, res = _reordered_trace(ob.RESTART_KAPPA, monkeypatch)
    pairs = _true_rho_next(tr)
    restarts = [i for i, (_, _, rs) in enumerate(pairs) if rs]
    assert restarts, "the case is meant to hit the restart test"
    for rho, true, rs in pairs:
        if not rs:
            assert abs(rho - true) <= 0.25 * abs(rho)
    for i in restarts:
        r = tr[i]["vec"]["r"]
        assert np.array_equal(tr[i + 1]["vec"]["r0"], r)
        assert tr[i + 1]["rho"] == tr[i]["est"]
        assert abs(tr[i]["est"] - math.fsum(r * r)) <= 1e-6 * tr[i]["est"]
    assert res.status == CONVERGED
    assert np.linalg.norm(b - S @ res.x) <= 1.1e-8 * np.linalg.norm(b)
    x_ref = sp.linalg.spsolve(S.tocsc(), b)
    assert np.linalg.norm(res.x - x_ref) <= 1e-5 * np.linalg.norm(x_ref)


def test_reordered_restart_test_bounds_the_drift(monkeypatch):
    """The bound E of the restart test covers the drift it is built for: on
    the passes before the first restart, |rho_{j+1} - (r_{j+1}, r_0)| stays
    below 4 u E_{j+1}."""
    _, _, tr, _ = _reordered_trace(ob.RESTART_KAPPA, monkeypatch)
    for i, (rho, true, rs) in enumerate(_true_rho_next(tr)):
        if rs:
            break
        assert abs(rho - true) <= 4 * ob.U64 * tr[i]["err"]


def test_jacobi_folded_operator():
    """A M^{-1} with M = diag(A): entry (i, j) is a_ij / a_jj, and the
    product with p equals A (M^{-1} p) up to one rounding per term."""
    A = conv_diff(9, 3, (1.0, -0.7, 0.3)).to_scipy()
    A.data = A.data * np.random.default_rng(3).uniform(0.5, 2.0, A.nnz)
    Ah = ob.jacobi_folded_operator(A)
    d = A.diagonal()
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    for e in np.random.default_rng(4).choice(A.nnz, 50, replace=False):
        i, j = rows[e], A.indices[e]
        assert Ah[i, j] == A[i, j] / d[j]
    p = np.random.default_rng(5).uniform(-1, 1, A.shape[0])
    ref = A @ (p / d)
    bound = 4 * np.finfo(float).eps * (abs(A) @ abs(p / d))
    assert np.all(np.abs(Ah @ p - ref) <= bound)


def test_pipelined_folded_jacobi_tracks_alg7():
    """The folded form (Alg. 4 on A M^{-1}, x += alpha M^{-1} p + omega
    M^{-1} q) takes Alg. 7's steps: over the first passes its x, r and
    scalars agree with Alg. 7's to rounding (r and w against their
    starting size), it keeps w = A M^{-1} r, and
    both stop at 1e-10 within two passes of each other. A product with A
    instead of A M^{-1}, or an update with p in place of M^{-1} p, fails
    from the first pass."""
    A = conv_diff(10, 3, (1.0, 0.7, 0.3)).to_scipy()
    A.data = A.data * np.random.default_rng(6).uniform(0.5, 2.0, A.nnz)
    A = A + sp.diags(np.random.default_rng(7).uniform(2.0, 9.0, A.shape[0]) * abs(A).sum(axis=1).A1 / 4)
    A = sp.csr_matrix(A)
    b = np.random.default_rng(8).uniform(-1, 1, A.shape[0])
    d = A.diagonal()
    tf, t7 = [], []
    solve_column(A, b, None, "pipelined", "fused", "jacobi", 0.0, 8, trace=tf, trace_vectors=True)
    solve_column(A, b, None, "pipelined", "merged", "jacobi", 0.0, 8, trace=t7, trace_vectors=True)

    def rel(u, w):
        return np.linalg.norm(u - w) / max(np.linalg.norm(w), 1e-300)

    for f, m in zip(tf, t7):
        assert rel(f["vec"]["x"], m["vec"]["x"]) < 1e-10
        # r falls by orders of magnitude over the passes: measure its
        # difference against ||b||
        assert np.linalg.norm(f["vec"]["r"] - m["vec"]["r"]) <= 1e-12 * np.linalg.norm(b)
    for f, m in zip(tf[:4], t7[:4]):  # later scalars come from vectors near rounding level
        assert abs(f["alpha"] - m["alpha"]) <= 1e-10 * abs(m["alpha"])
        assert abs(f["omega"] - m["omega"]) <= 1e-10 * abs(m["omega"])
    for prev, f in zip(tf, tf[1:]):  # w_{j+1} (recorded in the next pass) = A M^{-1} r_{j+1}
        w_true = A @ (prev["vec"]["r"] / d)
        assert np.linalg.norm(f["vec"]["w"] - w_true) <= 1e-12 * np.linalg.norm(A @ (b / d))
    rf = solve_column(A, b, None, "pipelined", "fused", "jacobi", 1e-10, 500)
    r7 = solve_column(A, b, None, "pipelined", "merged", "jacobi", 1e-10, 500)
    assert rf.status == r7.status == CONVERGED and abs(rf.iters - r7.iters) <= 2
    assert np.linalg.norm(b - A @ rf.x) <= 1.1e-10 * np.linalg.norm(b)


def test_reordered_folded_jacobi_tracks_alg6():
    """The folded Reordered form (Alg. 6 on A M^{-1} with no preconditioner,
    x += alpha M^{-1} p + omega M^{-1} r-tilde) takes Alg. 6's steps: over
    the first passes its x, r and scalars agree with the preconditioned
    listing's to rounding (r-tilde too, against ||b||), and both
    stop at 1e-10 within three passes of each other. A product with A instead
    of A M^{-1}, or an update with p in place of M^{-1} p, fails from the
    first pass."""
    A = conv_diff(10, 3, (1.0, 0.7, 0.3)).to_scipy()
    A.data = A.data * np.random.default_rng(6).uniform(0.5, 2.0, A.nnz)
    A = A + sp.diags(np.random.default_rng(7).uniform(2.0, 9.0, A.shape[0]) * abs(A).sum(axis=1).A1 / 4)
    A = sp.csr_matrix(A)
    b = np.random.default_rng(8).uniform(-1, 1, A.shape[0])
    tf, t6 = [], []
    solve_column(A, b, None, "reordered", "fused", "jacobi", 0.0, 6, trace=tf, trace_vectors=True)
    solve_column(A, b, None, "reordered", "merged", "jacobi", 0.0, 6, trace=t6, trace_vectors=True)
    nb = np.linalg.norm(b)
    for f, m in zip(tf, t6):
        assert np.linalg.norm(f["vec"]["x"] - m["vec"]["x"]) <= 1e-10 * np.linalg.norm(m["vec"]["x"])
        assert np.linalg.norm(f["vec"]["r"] - m["vec"]["r"]) <= 1e-12 * nb
        assert np.linalg.norm(f["vec"]["rt"] - m["vec"]["rt"]) <= 1e-12 * nb
    for f, m in zip(tf[:4], t6[:4]):
        assert abs(f["alpha"] - m["alpha"]) <= 1e-10 * abs(m["alpha"])
        assert abs(f["omega"] - m["omega"]) <= 1e-10 * abs(m["omega"])
    rf = solve_column(A, b, None, "reordered", "fused", "jacobi", 1e-10, 500)
    r6 = solve_column(A, b, None, "reordered", "merged", "jacobi", 1e-10, 500)
    assert rf.status == r6.status == CONVERGED and abs(rf.iters - r6.iters) <= 3
    assert np.linalg.norm(b - A @ rf.x) <= 1.1e-10 * nb


def test_pipelined_auxiliary_vectors():
    """Alg. 4 keeps s = A p, z = A s, y = A q, v = A z, w = A r, t = A w;
    Alg. 7 keeps the same with hat vectors on the right (s = A p-hat, ...) and
    p-hat = M^{-1} p-like relations for the hats."""
    A = conv_diff(10, 3, (1.0, 0.7, 0.3)).to_scipy()
    b = np.random.default_rng(8).uniform(-1, 1, A.shape[0])
    tr = []
    solve_column(A, b, None, "pipelined", "merged", "none", 1e-14, 25, trace=tr, trace_vectors=True)

    def rel(u, w):
        return np.linalg.norm(u - w) / max(np.linalg.norm(w), 1e-300)

    for rec in tr[:15]:
        V = rec["vec"]
        assert rel(V["s"], A @ V["p"]) < 1e-9
        assert rel(V["z"], A @ V["s"]) < 1e-9
        assert rel(V["y"], A @ V["q"]) < 1e-9
        assert rel(V["v"], A @ V["z"]) < 1e-14
        assert rel(V["t"], A @ V["w"]) < 1e-9
    d = A.diagonal()
    tr = []
    solve_column(A, b, None, "pipelined", "merged", "jacobi", 1e-14, 25, trace=tr, trace_vectors=True)
    prev_r = None
    for rec in tr[:15]:
        V = rec["vec"]
        assert rel(V["s"], A @ V["ph"]) < 1e-9
        assert rel(V["z"], A @ V["sh"]) < 1e-9
        assert rel(V["y"], A @ V["qh"]) < 1e-9
        assert rel(V["v"], A @ V["zh"]) < 1e-14
        assert rel(V["t"], A @ V["wh"]) < 1e-9
        assert rel(V["wh"], V["w"] / d) < 1e-9
        assert rel(V["sh"], V["s"] / d) < 1e-9
        assert rel(V["qh"], V["q"] / d) < 1e-9
        if prev_r is not None:
            assert rel(V["rh"], prev_r / d) < 1e-9
        prev_r = V["r"]


def test_cross_variant_equivalence():
    """All forms are reformulations of one method: the first iterates agree."""
    A = conv_diff(12, 3, (1.0, 0.7, 0.3)).to_scipy()
    b = np.random.default_rng(9).uniform(-1, 1, A.shape[0])
    ref = solve_column(A, b, None, "classical", "merged", "none", 0.0, 10).x
    for variant, formulation, precond in METHODS:
        x = solve_column(A, b, None, variant, formulation, precond, 0.0, 10).x
        assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-10, (variant, formulation, precond)
    full = {m: solve_column(A, b, None, *m, 1e-10, 1000) for m in METHODS}
    ref_its = solve_column(A, b, None, "classical", "merged", "none", 1e-10, 1000).iters
    # the tail of BiCGStab convergence is irregular, so the rounding of each
    # form moves the stopping pass by a few from the classical listing's
    assert all(abs(r.iters - ref_its) <= 5 for r in full.values()), {m: r.iters for m, r in full.items()}
    assert all(r.status == CONVERGED for r in full.values())


def test_identity_preconditioner_reduces_exactly():
    """With M = I the preconditioned listings compute exactly the
    unpreconditioned iterates: Alg. 5 with M = I equals Alg. 2, Alg. 7 with
    M = I equals Alg. 4, Alg. 1 with M = I equals Alg. 1 without M."""
    A = conv_diff(10, 3, (1.0, 0.7, 0.3)).to_scipy()
    b = np.random.default_rng(10).uniform(-1, 1, A.shape[0])
    x0 = np.zeros_like(b)
    eye = ob.identity_preconditioner(A)
    pairs = [
        (ob.alg5_merged_pbicgstab(A, b, x0, 1e-10, 500, eye), ob.alg2_merged_bicgstab(A, b, x0, 1e-10, 500)),
        (ob.alg7_merged_ppipebicgstab(A, b, x0, 1e-10, 500, eye), ob.alg4_merged_pipebicgstab(A, b, x0, 1e-10, 500)),
        (ob.alg1_bicgstab(A, b, x0, 1e-10, 500, eye), ob.alg1_bicgstab(A, b, x0, 1e-10, 500, None)),
    ]
    for a, c in pairs:
        assert a.iters == c.iters and a.status == c.status == CONVERGED
        assert np.array_equal(a.x, c.x)


def test_jacobi_on_constant_diagonal():
    """Jacobi on a constant diagonal is a uniform scaling: same iterates as the
    unpreconditioned method up to rounding."""
    A = conv_diff(10, 3, (1.0, 0.7, 0.3)).to_scipy()  # diagonal 6 everywhere
    b = np.random.default_rng(12).uniform(-1, 1, A.shape[0])
    for variant in ("classical", "reordered", "pipelined"):
        a = solve_column(A, b, None, variant, "merged", "none", 1e-10, 500)
        j = solve_column(A, b, None, variant, "merged", "jacobi", 1e-10, 500)
        assert abs(a.iters - j.iters) <= 2
        assert np.linalg.norm(a.x - j.x) / np.linalg.norm(a.x) < 1e-8


@pytest.mark.parametrize("c", [2.0, 3.0])
@pytest.mark.parametrize("variant,formulation,precond", METHODS)
def test_scaled_identity(c, variant, formulation, precond):
    """A = cI is solved in the first pass with x = b / c."""
    n = 17
    A = sp.csr_matrix(c * np.eye(n))
    b = np.random.default_rng(13).uniform(-1, 1, n)
    res = solve_column(A, b, None, variant, formulation, precond, 1e-12, 10)
    assert res.status == CONVERGED and res.iters == 1
    assert np.allclose(res.x, b / c, rtol=1e-15, atol=0)


@pytest.mark.parametrize("variant,formulation,precond", METHODS)
def test_diagonal_matrix_finite_termination(variant, formulation, precond):
    """For a diagonal matrix with d distinct eigenvalues the BiCG polynomial
    vanishes on the spectrum after d steps, so BiCGStab stops within d passes
    (one more is allowed for rounding)."""
    d = 4
    eig = np.array([1.0, 2.5, 4.0, 7.0])
    diag = np.repeat(eig, 10)
    A = sp.diags(diag).tocsr()
    b = np.random.default_rng(14).uniform(-1, 1, diag.size)
    res = solve_column(A, b, None, variant, formulation, "none", 1e-10, 50)
    assert res.status == CONVERGED and res.iters <= d + 1, res.iters
    assert np.allclose(res.x, b / diag, rtol=1e-8)


@pytest.mark.parametrize("variant,formulation,precond", METHODS)
def test_breakdown_skew(variant, formulation, precond):
    """A = [[0,1],[-1,0]] is skew, so (A r_0, r_0) = 0: delta_0 = 0 for the
    classical and Reordered forms and (r_0, w_0) = 0 for the Pipelined ones."""
    if precond == "jacobi":
        pytest.skip("zero diagonal: Jacobi is undefined")
    A = sp.csr_matrix(np.array([[0.0, 1.0], [-1.0, 0.0]]))
    b = np.array([1.0, 2.0])
    res = solve_column(A, b, None, variant, formulation, precond, 1e-10, 10)
    assert res.status == BREAKDOWN
    assert res.iters == (0 if variant == "pipelined" else 1)
    assert np.array_equal(res.x, np.zeros(2))


def test_jacobi_zero_diagonal_is_error():
    A = sp.csr_matrix(np.array([[0.0, 1.0], [-1.0, 0.0]]))
    with pytest.raises(ValueError):
        solve_column(A, np.ones(2), None, "classical", "merged", "jacobi", 1e-10, 10)


@pytest.mark.parametrize("variant,formulation,precond", METHODS)
def test_edge_columns(variant, formulation, precond):
    """Zero column: x = 0 after 0 passes. NaN: NONFINITE. maxit = 1: MAXIT.
    Exact initial guess: converged after 0 passes."""
    A = conv_diff(6, 2, (1.0, 0.5)).to_scipy()
    n = A.shape[0]
    rng = np.random.default_rng(15)
    xs = rng.uniform(-1, 1, n)
    B = np.stack([np.zeros(n), A @ xs, A @ xs, A @ xs], axis=1)
    B[3, 1] = np.nan
    X0 = np.zeros_like(B)
    X0[:, 3] = xs
    X0[:, 0] = 1.0  # ignored for a zero right-hand side
    res = solve(A, B, X0, variant, formulation, precond, 1e-10, 1)
    assert res.status[0] == CONVERGED and res.iters[0] == 0 and np.all(res.x[:, 0] == 0)
    assert res.status[1] == NONFINITE and res.iters[1] == 0
    assert res.status[2] == MAXIT and res.iters[2] == 1
    assert res.status[3] == CONVERGED and res.iters[3] == 0 and np.array_equal(res.x[:, 3], xs)


def test_stop_test_is_strict_and_first():
    """The count is the first pass whose estimate is below eps^2."""
    A = conv_diff(12, 2, (1.0, 0.5)).to_scipy()
    b = np.random.default_rng(16).uniform(-1, 1, A.shape[0])
    tol = 1e-9
    eps2 = tol * tol * (b @ b)
    for variant, formulation, precond in METHODS:
        tr = []
        res = solve_column(A, b, None, variant, formulation, precond, tol, 500, trace=tr)
        ests = [rec["est"] for rec in tr]
        assert res.iters == len(ests)
        assert ests[-1] < eps2 and all(e >= eps2 for e in ests[:-1])


def test_multi_rhs_columns_are_independent():
    A = conv_diff(8, 3, (1.0, 0.7, 0.3)).to_scipy()
    rng = np.random.default_rng(17)
    u = rng.uniform(-1, 1, A.shape[0])
    w = rng.uniform(-1, 1, A.shape[0])
    B = np.stack([u, w, u], axis=1)
    r1 = solve(A, B, tol=1e-10, maxit=500)
    r2 = solve(A, B[:, [1, 2, 0]], tol=1e-10, maxit=500)
    assert np.array_equal(r1.x[:, 0], r1.x[:, 2])
    assert np.array_equal(r1.x[:, [1, 2, 0]], r2.x)


def test_paper_model_tables():
    """The traffic model reproduces the 'Model' columns of Tables 5 and 6."""
    g = json.load(open(GOLDEN))["model_single_node"]
    N = g["grid"] ** 3
    C = (7 * N - 6 * g["grid"] ** 2) / N
    for mach in g["machines"].values():
        B = mach["node_GBps"] * 1000 * 2**20
        for meth, vals in mach["model"].items():
            for m, v in zip(mach["m"], vals):
                t = om.iteration_time(meth, N, m, C, B)
                assert abs(t - v) / v < 0.03, (meth, m, t, v)


# ------------------------------------------------- Improved BiCGStab (Alg. 3) ---

def _ib_problem(seed=1, g=10):
    A = conv_diff(g, 3, (1.0, -0.6, 0.4))
    b, xs = manufactured_rhs(A, 1, seed=seed)
    return A.to_scipy(), b[:, 0], xs[:, 0]


def test_improved_equals_classical_in_exact_arithmetic():
    """Alg. 3 is an algebraic rearrangement of BiCGStab: pass by pass, its
    alpha_{j+1}, omega_{j+1}, rho_{j+1} and iterate equal the classical
    method's alpha_j, omega_j, rho_j and iterate up to rounding. A dropped
    term or wrong index in any of its scalar recurrences breaks this at once."""
    S, b, _ = _ib_problem()
    ib = oracle.solve_column(S, b, variant="improved", tol=0.0, maxit=12, trace=[], trace_vectors=True)
    cl = oracle.solve_column(S, b, variant="classical", tol=0.0, maxit=12, trace=[], trace_vectors=True)
    for j in range(12):
        for key in ("alpha", "omega", "rho"):
            a, c = ib.trace[j][key], cl.trace[j][key]
            assert abs(a - c) <= 1e-9 * abs(c), (j, key, a, c)
        xi, xc = ib.trace[j]["vec"]["x"], cl.trace[j]["vec"]["x"]
        assert np.linalg.norm(xi - xc) <= 1e-9 * np.linalg.norm(xc), j


def test_improved_invariants():
    """rho_{j+1} = (r_0, r_j), sigma_{j+1} = (r_0, A r_{j+1}) and the stop
    estimate nu - omega theta = (r_{j+1}, r_{j+1}) hold along the run (they
    are what the recurrences replace)."""
    S, b, _ = _ib_problem(seed=2)
    res = oracle.solve_column(S, b, variant="improved", tol=0.0, maxit=15, trace=[], trace_vectors=True)
    r0 = b.copy()  # x0 = 0
    prev_r = r0
    for j, t in enumerate(res.trace):
        r = t["vec"]["r"]
        assert abs(t["rho"] - r0 @ prev_r) <= 1e-8 * abs(r0 @ r0), (j, t["rho"], r0 @ prev_r)
        ar = S @ r
        assert abs(t["sigma"] - r0 @ ar) <= 1e-8 * np.linalg.norm(r0) * np.linalg.norm(ar), j
        assert abs(t["est"] - r @ r) <= 1e-8 * (r0 @ r0), (j, t["est"], r @ r)
        prev_r = r


def test_improved_dense_solve_and_edges():
    S, b, xs = _ib_problem(seed=3, g=6)
    res = oracle.solve_column(S, b, variant="improved", tol=1e-12, maxit=500)
    assert res.status == oracle.CONVERGED
    xd = np.linalg.solve(S.toarray(), b)
    assert np.linalg.norm(res.x - xd) <= 1e-9 * np.linalg.norm(xd)
    # b = 0: x = 0 after 0 passes; maxit = 0: MAXIT, x unchanged
    z = oracle.solve_column(S, np.zeros_like(b), np.ones_like(b), variant="improved")
    assert z.status == oracle.CONVERGED and z.iters == 0 and np.all(z.x == 0)
    m = oracle.solve_column(S, b, variant="improved", tol=1e-12, maxit=0)
    assert m.status == oracle.MAXIT and m.iters == 0 and np.all(m.x == 0)
    with pytest.raises(ValueError):
        oracle.solve_column(S, b, variant="improved", precond="jacobi")


def test_improved_scaled_identity_one_pass():
    """A = 2I: alpha_1 = 1/2 makes s = 0 and t = 0, so kappa = 0 (omega = 0)
    and the estimate nu - omega theta = 0: converged in one pass with the
    exact solution x = b / 2."""
    import scipy.sparse as sp

    n = 40
    S = sp.identity(n, format="csr") * 2.0
    b = np.random.default_rng(4).uniform(-1, 1, n)
    res = oracle.solve_column(S, b, variant="improved", tol=1e-10, maxit=10)
    assert res.status == oracle.CONVERGED and res.iters == 1
    assert np.array_equal(res.x, b * 0.5)
