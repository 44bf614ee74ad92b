"""Plain FP64 BiCGStab, one right-hand side at a time.

TEST INFRASTRUCTURE ONLY (see the package docstring): the library never calls
this module.

Each function below takes the steps of one listing of the paper's Appendix B in
the listing's order and notation, for ONE column b of the right-hand-side block
(1-D NumPy arrays, SciPy CSR for the matrix-vector product). Multi-RHS solves
treat the columns as independent systems that share A: every dot product of
the paper yields one scalar per right-hand side (the message of a grouped
reduction holds 8*m*k bytes, Section 3.1.2), so the scalars alpha, omega, rho,
... are per column and the method is not a block-Krylov method.

Readings where the paper is silent (the paper sets convergence issues aside,
Section 1):

* Stop test. The listings break when the squared residual estimate drops below
  eps^2; here eps = tol * ||b||_2 per column, with a strict '<'. Classical
  basic (Alg. 1) uses the explicit (r_{j+1}, r_{j+1}); the merged forms use the
  estimate the listing prints (theta - omega*phi for Alg. 2/5, eta - omega*theta
  for Alg. 6, pi - omega*theta for Alg. 4/7). tol <= 0 disables the test (fixed
  iteration count). The iteration count is the number of loop passes entered,
  including the one that terminates.
* Before the loop: a non-finite ||b||^2 or (r_0, r_0) gives NONFINITE after 0
  iterations; b = 0 gives x = 0, CONVERGED after 0 iterations; (r_0, r_0) <
  eps^2 gives CONVERGED after 0 iterations with x = x_0.
* Zero divisors. delta = 0 (Alg. 1, 2, 5, 6) and (r_0, w_0) = 0 (Alg. 4, 7)
  stop the column as BREAKDOWN before any update of that pass. psi = 0 (phi = 0
  in Alg. 4, 6, 7) sets omega = 0 instead of dividing; if the stop test then
  fails, the pass's x and r updates are still applied and the column stops as
  BREAKDOWN. rho_{j+1} = 0 (Alg. 1, 2, 4, 5, 7) and a zero denominator for
  alpha_{j+1} (Alg. 4, 7) stop the column as BREAKDOWN after that pass's x and
  r updates; in Alg. 6 a zero rho_{j+1} is a loss of the recurrence (below).
* A non-finite alpha, omega, stop estimate, beta or alpha_{j+1} stops the
  column as NONFINITE at the point where that scalar is formed.
* Alg. 6 forms rho_{j+1} = -omega_j psi_j from the exact-arithmetic
  orthogonality (r-tilde_j, r_0) = 0. Rounding leaves the stored vectors off
  that relation by an amount that adds up pass by pass and does not shrink with
  the residual, so once |rho_{j+1}| falls to that level the recurrence carries
  no information and alpha is formed from noise (the paper sets such
  convergence issues of the reordering aside). Reading: a running bound E of
  the accumulated terms, E_0 = rho_0 and
  E_{j+1} = E_j + sqrt(rho^) (||r_j|| + 2 sqrt(eta_j) + 2 |omega_j| sqrt(phi_j)),
  with rho^ = (r_0, r_0) of the current shadow vector and ||r_j|| taken from
  the previous pass's stop estimate (rho_0 at the first pass). When
  |rho_{j+1}| <= RESTART_KAPPA * u * E_{j+1} (u = 2^-53; this includes
  rho_{j+1} = 0) the method restarts after the pass's updates: the shadow
  vector becomes r_{j+1}, rho_{j+1} = eta_j - omega_j theta_j (the pass's stop
  estimate, which is (r_{j+1}, r_{j+1}) in exact arithmetic), beta_j = 0 (so
  v-hat_{j+1} = z_{j+1}), rho^ = rho_{j+1} and E = eta_j. A restart with a
  stop estimate that is not positive stops the column as BREAKDOWN instead.
* Alg. 7 typos: the initial line reads w-hat_0 = M^{-1} w_0, and the line after
  the last grouped update reads w-hat_{j+1} = M^{-1} w_{j+1},
  t_{j+1} = A w-hat_{j+1}.
* Pipelined "previous" vectors are zero before the first pass, with
  beta_{-1} = 0 and omega_{-1} = 1.
* Improved BiCGStab (Alg. 3) is taken as printed (the paper notes two
  corrections it took from another code base; the printed listing includes
  them). Its scalars rho_{j+1}, delta_{j+1}, beta_{j+1}, tau_{j+1} and
  alpha_{j+1} are formed at the start of pass j: rho_{j+1} = 0 or
  tau_{j+1} = 0 stops the column as BREAKDOWN, and a non-finite delta, beta,
  tau or alpha as NONFINITE, both before any update of that pass (the pass
  counts as entered). kappa = 0 sets omega = 0; a non-finite omega, sigma or
  stop estimate nu - omega*theta stops the column as NONFINITE before the x
  and r updates; otherwise the updates are applied, then the stop test, then
  omega = 0 gives BREAKDOWN. Alg. 3 has no preconditioned form in the paper.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RUNNING = -1
CONVERGED = 0
MAXIT = 1
BREAKDOWN = 2
NONFINITE = 3

# Unit roundoff of FP64 and the factor of the Reordered method's restart test.
U64 = 2.0**-53
RESTART_KAPPA = 16.0

STATUS_NAMES = {RUNNING: "running", CONVERGED: "converged", MAXIT: "maxit", BREAKDOWN: "breakdown", NONFINITE: "nonfinite"}


@dataclass
class ColumnResult:
    x: np.ndarray
    r: np.ndarray  # the recursively updated residual at exit
    iters: int
    status: int
    trace: list = field(default_factory=list)


def dot(u, w) -> float:
    """Euclidean inner product (u, w)."""
    return float(np.dot(u, w))


def identity_preconditioner(A):
    """M = I: M^{-1} u is a copy of u (the preconditioner of Section 2.3)."""
    return lambda u: u.copy()


def jacobi_preconditioner(A):
    """M = diag(A): M^{-1} u = u / a_ii. A zero diagonal entry is an error."""
    d = np.asarray(A.diagonal(), dtype=np.float64)
    if np.any(d == 0.0):
        raise ValueError("Jacobi preconditioner: zero diagonal entry")
    return lambda u: u / d


def jacobi_folded_operator(A):
    """A M^{-1} with M = diag(A), as a CSR matrix: entry (i, j) is
    a_ij / a_jj (one division per stored entry)."""
    import scipy.sparse as sp

    A = sp.csr_matrix(A)
    d = np.asarray(A.diagonal(), dtype=np.float64)
    if np.any(d == 0.0):
        raise ValueError("Jacobi preconditioner: zero diagonal entry")
    Ah = A.copy()
    Ah.data = A.data / d[A.indices]
    return Ah


class _Recorder:
    def __init__(self, trace, vectors: bool):
        self.trace = trace
        self.vectors = vectors

    def __call__(self, j, scal: dict, **vecs):
        if self.trace is None:
            return
        rec = {"j": j}
        rec.update(scal)
        if self.vectors:
            rec["vec"] = {k: v.copy() for k, v in vecs.items()}
        self.trace.append(rec)


def _begin(A, b, x0, tol):
    """Shared start: norms, eps^2 and the initial residual r_0 = b - A x_0.
    Returns (early ColumnResult or None, x, r, rho0, eps2)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    bb = dot(b, b)
    if not np.isfinite(bb):
        return ColumnResult(x, b - A @ x, 0, NONFINITE), None, None, None, None
    if bb == 0.0:
        z = np.zeros_like(x)
        return ColumnResult(z, np.zeros_like(x), 0, CONVERGED), None, None, None, None
    eps2 = tol * tol * bb if tol > 0 else -np.inf
    r = b - A @ x
    rho0 = dot(r, r)
    if not np.isfinite(rho0):
        return ColumnResult(x, r, 0, NONFINITE), None, None, None, None
    if rho0 < eps2:
        return ColumnResult(x, r, 0, CONVERGED), None, None, None, None
    return None, x, r, rho0, eps2


# ------------------------------------------------------------- classical ---

def alg1_bicgstab(A, b, x0, tol, maxit, Minv=None, trace=None, trace_vectors=False):
    """Alg. 1 (Van der Vorst's BiCGStab), one operation per statement. With a
    preconditioner the two products become v = A M^{-1} p and t = A M^{-1} s and
    the solution update uses the preconditioned vectors (right preconditioning,
    as in Alg. 5). Stop test: explicit (r_{j+1}, r_{j+1}) < eps^2."""
    rec = _Recorder(trace, trace_vectors)
    early, x, r, rho, eps2 = _begin(A, b, x0, tol)
    if early is not None:
        return early
    M = Minv if Minv is not None else (lambda u: u)
    r0 = r.copy()
    p = r.copy()
    for j in range(maxit):
        ph = M(p)
        v = A @ ph
        delta = dot(v, r0)
        if delta == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        alpha = rho / delta
        if not np.isfinite(alpha):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        s = r - alpha * v
        sh = M(s)
        t = A @ sh
        phi = dot(t, s)
        psi = dot(t, t)
        omega = phi / psi if psi != 0.0 else 0.0
        if not np.isfinite(omega):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rr = dot(r, r)
        rec(j, {"alpha": alpha, "omega": omega, "rho": rho, "est": rr}, x=x, r=r)
        if not np.isfinite(rr):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        if rr < eps2:
            return ColumnResult(x, r, j + 1, CONVERGED, trace)
        if omega == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        rho_next = dot(r, r0)
        if rho_next == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        beta = (rho_next / rho) * (alpha / omega)
        if not np.isfinite(beta):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        p = r + beta * (p - omega * v)
        rho = rho_next
    return ColumnResult(x, r, maxit, MAXIT, trace)


def alg2_merged_bicgstab(A, b, x0, tol, maxit, trace=None, trace_vectors=False):
    """Alg. 2: merged BiCGStab. theta = (s, s) is formed with phi and psi, and
    the stop test uses theta - omega*phi, which equals (r_{j+1}, r_{j+1}) in
    exact arithmetic (footnote in Section 1)."""
    rec = _Recorder(trace, trace_vectors)
    early, x, r, rho, eps2 = _begin(A, b, x0, tol)
    if early is not None:
        return early
    r0 = r.copy()
    p = r.copy()
    for j in range(maxit):
        v = A @ p
        delta = dot(v, r0)
        if delta == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        alpha = rho / delta
        if not np.isfinite(alpha):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        s = r - alpha * v
        t = A @ s
        phi, psi, theta = dot(t, s), dot(t, t), dot(s, s)
        omega = phi / psi if psi != 0.0 else 0.0
        est = theta - omega * phi
        if not (np.isfinite(omega) and np.isfinite(est)):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rec(j, {"alpha": alpha, "omega": omega, "rho": rho, "est": est}, x=x, r=r)
        if est < eps2:
            return ColumnResult(x, r, j + 1, CONVERGED, trace)
        if omega == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        rho_next = dot(r, r0)
        if rho_next == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        beta = (rho_next / rho) * (alpha / omega)
        if not np.isfinite(beta):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        p = r + beta * (p - omega * v)
        rho = rho_next
    return ColumnResult(x, r, maxit, MAXIT, trace)


def alg5_merged_pbicgstab(A, b, x0, tol, maxit, Minv, trace=None, trace_vectors=False, A_prec=None):
    """Alg. 5: merged preconditioned BiCGStab (p-hat = M^{-1} p, s-hat =
    M^{-1} s). The solution update x += alpha p-hat + omega s-hat does not
    depend on beta; it is formed before the breakdown checks on rho_{j+1} so a
    column that stops there keeps the pass's x and r updates.

    A_prec, if given, is the operator A M^{-1} stored as a matrix (possible
    for a diagonal M): the two products read v = A_prec p and t = A_prec s
    instead of A (M^{-1} p) and A (M^{-1} s). Alg. 5 preconditions from the
    right, so the iterates are the same in exact arithmetic; only the
    rounding of the products differs. p-hat and s-hat are then formed for the
    solution update alone."""
    rec = _Recorder(trace, trace_vectors)
    early, x, r, rho, eps2 = _begin(A, b, x0, tol)
    if early is not None:
        return early
    r0 = r.copy()
    p = r.copy()
    for j in range(maxit):
        ph = Minv(p)
        v = A @ ph if A_prec is None else A_prec @ p
        delta = dot(v, r0)
        if delta == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        alpha = rho / delta
        if not np.isfinite(alpha):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        s = r - alpha * v
        sh = Minv(s)
        t = A @ sh if A_prec is None else A_prec @ s
        phi, psi, theta = dot(t, s), dot(t, t), dot(s, s)
        omega = phi / psi if psi != 0.0 else 0.0
        est = theta - omega * phi
        if not (np.isfinite(omega) and np.isfinite(est)):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        if est < eps2:
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            rec(j, {"alpha": alpha, "omega": omega, "rho": rho, "est": est}, x=x, r=r)
            return ColumnResult(x, r, j + 1, CONVERGED, trace)
        r = s - omega * t
        rho_next = dot(r, r0)
        x = x + alpha * ph + omega * sh
        rec(j, {"alpha": alpha, "omega": omega, "rho": rho, "est": est}, x=x, r=r)
        if omega == 0.0 or rho_next == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        beta = (rho_next / rho) * (alpha / omega)
        if not np.isfinite(beta):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        p = r + beta * (p - omega * v)
        rho = rho_next
    return ColumnResult(x, r, maxit, MAXIT, trace)


# -------------------------------------------------------------- improved ---

def alg3_merged_ibicgstab(A, b, x0, tol, maxit, trace=None, trace_vectors=False):
    """Alg. 3: merged Improved BiCGStab, one grouped reduction of seven dot
    products per pass. f_0 = A^T r_0 is formed once; sigma_j equals
    (r_0, A r_j) and rho_{j+1} equals (r_0, r_j) in exact arithmetic, and the
    stop estimate nu - omega*theta equals (r_{j+1}, r_{j+1})."""
    rec = _Recorder(trace, trace_vectors)
    early, x, r, _, eps2 = _begin(A, b, x0, tol)
    if early is not None:
        return early
    r0 = r.copy()
    u = A @ r
    f0 = A.T @ r0
    q = np.zeros_like(r)
    v = np.zeros_like(r)
    z = np.zeros_like(r)
    sigma_prev, pi, tau = 0.0, 0.0, 0.0
    sigma = dot(r0, u)
    rho = alpha = omega = 1.0
    phi = dot(r0, r0)
    for j in range(maxit):
        rho1 = phi - omega * sigma_prev + omega * alpha * pi
        delta = (rho1 / rho) * alpha
        beta = delta / omega
        tau = sigma + beta * tau - delta * pi
        if rho1 == 0.0 or tau == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        alpha1 = rho1 / tau
        if not (np.isfinite(delta) and np.isfinite(beta) and np.isfinite(tau) and np.isfinite(alpha1)):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        z = alpha1 * r + (beta * (alpha1 / alpha)) * z - (alpha1 * delta) * v
        v = u + beta * v - delta * q
        s = r - alpha1 * v
        q = A @ v
        t = u - alpha1 * q
        phi, pi = dot(r0, s), dot(r0, q)
        gamma, eta = dot(f0, s), dot(f0, t)
        theta, kappa, nu = dot(s, t), dot(t, t), dot(s, s)
        omega = theta / kappa if kappa != 0.0 else 0.0
        sigma_new = gamma - omega * eta
        est = nu - omega * theta
        if not (np.isfinite(omega) and np.isfinite(sigma_new) and np.isfinite(est)):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        r = s - omega * t
        x = x + z + omega * s
        rec(j, {"alpha": alpha1, "omega": omega, "rho": rho1, "est": est, "sigma": sigma_new, "tau": tau},
            x=x, r=r)
        if est < eps2:
            return ColumnResult(x, r, j + 1, CONVERGED, trace)
        if omega == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        u = A @ r
        sigma_prev, sigma = sigma, sigma_new
        alpha, rho = alpha1, rho1
    return ColumnResult(x, r, maxit, MAXIT, trace)


# ------------------------------------------------------------- reordered ---

def alg6_merged_rbicgstab(A, b, x0, tol, maxit, Minv, trace=None, trace_vectors=False, A_prec=None, Minv_x=None):
    """Alg. 6: merged Reordered BiCGStab. The preconditioner is applied to
    v_j and t_j (s_j = M^{-1} v_j, q_j = M^{-1} t_j) so that z_{j+1} = M^{-1}
    r_{j+1} comes from a vector update; rho_{j+1} = -omega_j psi_j uses the
    exact-arithmetic orthogonality (r-tilde_j, r_0) = 0. The z_{j+1} line is
    taken as printed (it already carries the paper's fix of the original).
    When rounding has used up what that relation carries (the restart test of
    the module docstring), the method restarts with r_{j+1} as the shadow
    vector.

    A_prec, if given, is A M^{-1} stored as a matrix (a diagonal M, with
    Minv_x applying M^{-1}); Minv is then the identity. Alg. 6 preconditions
    from the right: with p_j defined by v-hat_j = M^{-1} p_j, its vectors obey
    v = (A M^{-1}) p, t-hat = M^{-1} r-tilde, t = (A M^{-1}) r-tilde, z =
    M^{-1} r, so the listing run on A M^{-1} without a preconditioner carries
    p and r-tilde where it carried v-hat and t-hat, and the solution update
    becomes x += alpha M^{-1} p + omega M^{-1} r-tilde: Alg. 6's iterates in
    exact arithmetic, with no preconditioned block kept."""
    rec = _Recorder(trace, trace_vectors)
    early, x, r, rho, eps2 = _begin(A, b, x0, tol)
    if early is not None:
        return early
    op = A if A_prec is None else A_prec
    r0 = r.copy()
    z = Minv(r)
    vh = z.copy()
    rho_sh = rho      # (r_0, r_0) of the shadow vector
    err = rho         # E_0
    est_prev = rho    # ||r_0||^2
    for j in range(maxit):
        v = op @ vh
        delta = dot(v, r0)
        if delta == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        s = Minv(v)
        alpha = rho / delta
        if not np.isfinite(alpha):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        th = z - alpha * s
        t = op @ th
        rt = r - alpha * v
        theta, phi, psi, eta = dot(t, rt), dot(t, t), dot(t, r0), dot(rt, rt)
        q = Minv(t)
        omega = theta / phi if phi != 0.0 else 0.0
        est = eta - omega * theta
        if not (np.isfinite(omega) and np.isfinite(est)):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        stop = est < eps2
        stop_breakdown = False
        restart = False
        if not stop:
            rho_next = -omega * psi
            stop_breakdown = omega == 0.0
            if not stop_breakdown:
                rn = math.sqrt(est_prev) if est_prev > 0.0 else 0.0
                err = err + math.sqrt(rho_sh) * (rn + 2.0 * math.sqrt(eta) + 2.0 * abs(omega) * math.sqrt(phi))
                restart = abs(rho_next) <= RESTART_KAPPA * U64 * err
                if restart:
                    stop_breakdown = not est > 0.0
                    rho_next = est
                    beta = 0.0
                    rho_sh = est
                    err = eta
                else:
                    beta = (rho_next / rho) * (alpha / omega)
                    if not np.isfinite(beta):
                        return ColumnResult(x, r, j + 1, NONFINITE, trace)
        r = rt - omega * t
        if Minv_x is None:
            x = x + alpha * vh + omega * th
        else:
            x = x + alpha * Minv_x(vh) + omega * Minv_x(th)
        rec(j, {"alpha": alpha, "omega": omega, "rho": rho, "est": est, "theta": theta, "phi": phi, "psi": psi,
                "eta": eta, "err": err, "restart": restart}, x=x, r=r, rt=rt, r0=r0)
        if stop:
            return ColumnResult(x, r, j + 1, CONVERGED, trace)
        if stop_breakdown:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        if restart:
            r0 = r.copy()
        z = th - omega * q
        vh = z + beta * (vh - omega * s)
        rho = rho_next
        est_prev = est
    return ColumnResult(x, r, maxit, MAXIT, trace)


# ------------------------------------------------------------- pipelined ---

def _pipelined_scalars(alpha, omega, rho, rho_next, sigma, delta, psi):
    """beta_j and alpha_{j+1} of Alg. 4/7; returns (status or None, beta, alpha')."""
    if rho_next == 0.0:
        return BREAKDOWN, None, None
    beta = (alpha / omega) * (rho_next / rho)
    denom = sigma + beta * delta - beta * omega * psi
    if denom == 0.0:
        return BREAKDOWN, None, None
    alpha_next = rho_next / denom
    if not (np.isfinite(beta) and np.isfinite(alpha_next)):
        return NONFINITE, None, None
    return None, beta, alpha_next


def alg4_merged_pipebicgstab(A, b, x0, tol, maxit, trace=None, trace_vectors=False, A_prec=None, Minv=None):
    """Alg. 4: merged Pipelined BiCGStab (Cools and Vanroose). The auxiliary
    vectors satisfy s = A p, z = A s, w = A r, t = A w, y = A q, v = A z in
    exact arithmetic; the stop test is pi - omega*theta.

    A_prec, if given, is A M^{-1} stored as a matrix (a diagonal M, with Minv
    applying M^{-1}). Alg. 7 preconditions from the right: its plain vectors
    (r, w, t, s, z, q, y, v) obey Alg. 4's recurrences with the operator
    A M^{-1}, and each hat vector is M^{-1} times its plain one (p-hat =
    M^{-1} p, q-hat = M^{-1} q, ...). So the products take A_prec and the
    solution update is x += alpha M^{-1} p + omega M^{-1} q: Alg. 7's iterates
    in exact arithmetic, with no hat vector kept."""
    rec = _Recorder(trace, trace_vectors)
    early, x, r, rho, eps2 = _begin(A, b, x0, tol)
    if early is not None:
        return early
    op = A if A_prec is None else A_prec
    r0 = r.copy()
    w = op @ r
    t = op @ w
    rw = dot(r, w)
    if rw == 0.0:
        return ColumnResult(x, r, 0, BREAKDOWN)
    alpha = rho / rw
    if not np.isfinite(alpha):
        return ColumnResult(x, r, 0, NONFINITE)
    beta, omega = 0.0, 1.0
    p = np.zeros_like(r)
    s = np.zeros_like(r)
    z = np.zeros_like(r)
    v = np.zeros_like(r)
    for j in range(maxit):
        p = r + beta * (p - omega * s)
        s = w + beta * (s - omega * z)
        z = t + beta * (z - omega * v)
        q = r - alpha * s
        y = w - alpha * z
        theta, phi, pi = dot(q, y), dot(y, y), dot(q, q)
        v = op @ z
        omega = theta / phi if phi != 0.0 else 0.0
        est = pi - omega * theta
        if not (np.isfinite(omega) and np.isfinite(est)):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        if Minv is None:
            x = x + alpha * p + omega * q
        else:
            x = x + alpha * Minv(p) + omega * Minv(q)
        r = q - omega * y
        rec(j, {"alpha": alpha, "omega": omega, "rho": rho, "est": est}, x=x, r=r, p=p, s=s, z=z, q=q, y=y, v=v, w=w, t=t)
        if est < eps2:
            return ColumnResult(x, r, j + 1, CONVERGED, trace)
        if omega == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        w = y - omega * (t - alpha * v)
        rho_next, psi, sigma, delta = dot(r0, r), dot(r0, z), dot(r0, w), dot(r0, s)
        t = op @ w
        st, beta, alpha_next = _pipelined_scalars(alpha, omega, rho, rho_next, sigma, delta, psi)
        if st is not None:
            return ColumnResult(x, r, j + 1, st, trace)
        alpha, rho = alpha_next, rho_next
    return ColumnResult(x, r, maxit, MAXIT, trace)


def alg7_merged_ppipebicgstab(A, b, x0, tol, maxit, Minv, trace=None, trace_vectors=False):
    """Alg. 7: merged preconditioned Pipelined BiCGStab. Hat vectors are the
    preconditioned ones (r-hat = M^{-1} r, ...); the shadow residual is r_0."""
    rec = _Recorder(trace, trace_vectors)
    early, x, r, rho, eps2 = _begin(A, b, x0, tol)
    if early is not None:
        return early
    r0 = r.copy()
    rh = Minv(r)
    w = A @ rh
    wh = Minv(w)
    t = A @ wh
    rw = dot(r, w)
    if rw == 0.0:
        return ColumnResult(x, r, 0, BREAKDOWN)
    alpha = rho / rw
    if not np.isfinite(alpha):
        return ColumnResult(x, r, 0, NONFINITE)
    beta, omega = 0.0, 1.0
    ph = np.zeros_like(r)
    sh = np.zeros_like(r)
    zh = np.zeros_like(r)
    s = np.zeros_like(r)
    z = np.zeros_like(r)
    v = np.zeros_like(r)
    for j in range(maxit):
        ph = rh + beta * (ph - omega * sh)
        sh = wh + beta * (sh - omega * zh)
        qh = rh - alpha * sh
        s = w + beta * (s - omega * z)
        z = t + beta * (z - omega * v)
        q = r - alpha * s
        y = w - alpha * z
        theta, phi, pi = dot(q, y), dot(y, y), dot(q, q)
        zh = Minv(z)
        v = A @ zh
        omega = theta / phi if phi != 0.0 else 0.0
        est = pi - omega * theta
        if not (np.isfinite(omega) and np.isfinite(est)):
            return ColumnResult(x, r, j + 1, NONFINITE, trace)
        x = x + alpha * ph + omega * qh
        r = q - omega * y
        rec(j, {"alpha": alpha, "omega": omega, "rho": rho, "est": est}, x=x, r=r, ph=ph, sh=sh, qh=qh, s=s, z=z, zh=zh,
            q=q, y=y, v=v, w=w, wh=wh, t=t, rh=rh)
        if est < eps2:
            return ColumnResult(x, r, j + 1, CONVERGED, trace)
        if omega == 0.0:
            return ColumnResult(x, r, j + 1, BREAKDOWN, trace)
        rh = qh - omega * (wh - alpha * zh)
        w = y - omega * (t - alpha * v)
        rho_next, psi, sigma, delta = dot(r0, r), dot(r0, z), dot(r0, w), dot(r0, s)
        wh = Minv(w)
        t = A @ wh
        st, beta, alpha_next = _pipelined_scalars(alpha, omega, rho, rho_next, sigma, delta, psi)
        if st is not None:
            return ColumnResult(x, r, j + 1, st, trace)
        alpha, rho = alpha_next, rho_next
    return ColumnResult(x, r, maxit, MAXIT, trace)


# -------------------------------------------------------------- dispatch ---

VARIANTS = ("classical", "reordered", "pipelined", "improved")
FORMULATIONS = ("merged", "basic", "fused")
PRECONDS = ("none", "jacobi")


def solve_column(A, b, x0=None, variant="classical", formulation="merged", precond="none", tol=1e-8, maxit=1000,
                 trace=None, trace_vectors=False) -> ColumnResult:
    """One column. The basic and merged forms of the Reordered and Pipelined
    methods run the same statements (merging changes which statements share a
    pass over memory, Table 2, not what they compute), so both map to the
    listing; for the classical method the basic form is Alg. 1 with its
    explicit residual-norm stop test. The fused form (a single-device
    regrouping of the merged statements: dots formed in the sparse products'
    epilogues, the Jacobi division done by the pass that produces the vector)
    computes the merged listing's statements, so it maps to that listing;
    with Jacobi it folds M^{-1} into the products (Alg. 5, Alg. 6, and Alg. 4
    standing for Alg. 7, with A M^{-1} stored as a matrix)."""
    import scipy.sparse as sp

    A = sp.csr_matrix(A)
    b = np.asarray(b, dtype=np.float64)
    x0 = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64)
    if variant not in VARIANTS or formulation not in FORMULATIONS or precond not in PRECONDS:
        raise ValueError(f"unknown method {variant}/{formulation}/{precond}")
    fused = formulation == "fused"
    if fused:
        formulation = "merged"
    if variant == "improved":
        # Alg. 3; its basic form runs the same statements one per pass
        if precond != "none":
            raise ValueError("Improved BiCGStab has no preconditioned form in the paper")
        return alg3_merged_ibicgstab(A, b, x0, tol, maxit, trace=trace, trace_vectors=trace_vectors)
    if precond == "jacobi":
        Minv = jacobi_preconditioner(A)
    else:
        Minv = identity_preconditioner(A)
    kw = dict(trace=trace, trace_vectors=trace_vectors)
    if variant == "classical":
        if formulation == "basic":
            return alg1_bicgstab(A, b, x0, tol, maxit, Minv if precond == "jacobi" else None, **kw)
        if precond == "none":
            return alg2_merged_bicgstab(A, b, x0, tol, maxit, **kw)
        if fused:
            # the fused form folds Jacobi into the products: A M^{-1} as a matrix
            return alg5_merged_pbicgstab(A, b, x0, tol, maxit, Minv, A_prec=jacobi_folded_operator(A), **kw)
        return alg5_merged_pbicgstab(A, b, x0, tol, maxit, Minv, **kw)
    if variant == "reordered":
        if fused and precond == "jacobi":
            # Alg. 6 with Jacobi folded into the products: the listing on A M^{-1}
            return alg6_merged_rbicgstab(A, b, x0, tol, maxit, identity_preconditioner(A),
                                         A_prec=jacobi_folded_operator(A), Minv_x=Minv, **kw)
        return alg6_merged_rbicgstab(A, b, x0, tol, maxit, Minv, **kw)
    if precond == "none":
        return alg4_merged_pipebicgstab(A, b, x0, tol, maxit, **kw)
    if fused:
        # Alg. 7 with Jacobi folded into the products: Alg. 4 on A M^{-1}
        return alg4_merged_pipebicgstab(A, b, x0, tol, maxit, A_prec=jacobi_folded_operator(A), Minv=Minv, **kw)
    return alg7_merged_ppipebicgstab(A, b, x0, tol, maxit, Minv, **kw)


@dataclass
class BlockResult:
    x: np.ndarray  # n x k
    r: np.ndarray  # n x k, recursive residual
    iters: np.ndarray  # k
    status: np.ndarray  # k
    relres_true: np.ndarray  # k, ||b - A x|| / ||b||
    relres_recursive: np.ndarray  # k, ||r|| / ||b||
    traces: list


def solve(A, B, X0=None, variant="classical", formulation="merged", precond="none", tol=1e-8, maxit=1000,
          columns=None, trace=False, trace_vectors=False) -> BlockResult:
    """Solve A X = B for an n x k block, column by column (independent
    recurrences). `columns` restricts the work to a subset of columns; the
    other columns of the result are NaN."""
    import scipy.sparse as sp

    A = sp.csr_matrix(A)
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    n, k = B.shape
    X0 = np.zeros_like(B) if X0 is None else np.asarray(X0, dtype=np.float64).reshape(n, k)
    cols = range(k) if columns is None else columns
    X = np.full((n, k), np.nan)
    R = np.full((n, k), np.nan)
    iters = np.full(k, -1, dtype=np.int64)
    status = np.full(k, RUNNING, dtype=np.int64)
    rt = np.full(k, np.nan)
    rr = np.full(k, np.nan)
    traces = [None] * k
    for c in cols:
        tr = [] if trace else None
        res = solve_column(A, B[:, c], X0[:, c], variant, formulation, precond, tol, maxit, tr, trace_vectors)
        X[:, c], R[:, c], iters[c], status[c], traces[c] = res.x, res.r, res.iters, res.status, tr
        nb = np.linalg.norm(B[:, c])
        if nb > 0:
            rt[c] = np.linalg.norm(B[:, c] - A @ res.x) / nb
            rr[c] = np.linalg.norm(res.r) / nb
        else:
            rt[c] = rr[c] = 0.0
    return BlockResult(X, R, iters, status, rt, rr, traces)
