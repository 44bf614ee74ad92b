"""Seeded generators for the synthetic workloads.

Every matrix is returned in canonical CSR form (int32 row pointers and column
indices, float64 values, columns ascending within each row). Unknowns on a grid
are numbered lexicographically with the x coordinate fastest. Multi-vectors are
n x k arrays in row-major order, so element (i, c) lives at i*k + c.

The workloads follow the paper's benchmark setting (a 7-point stencil on a
uniform cube, Section 2.3 and Section 3.2) and the derived configurations:

* 2D / 3D convection-diffusion -Lap(u) + beta . grad(u) with central
  differences on the unit square / cube, homogeneous Dirichlet boundary
  eliminated, the whole operator scaled by h^2 (h = 1/(g+1)): diagonal 2d,
  neighbour in direction +e_d gets -1 + beta_d h/2, in -e_d gets -1 - beta_d h/2.
* a 27-point stencil with random nonsymmetric off-diagonals
  a_ij = u_ij (1 + 0.3 xi_ij), u ~ U[-1,0], xi ~ U[-1,1], diagonal
  1.05 * sum_j |a_ij| (strictly diagonally dominant).
* a random sparse matrix: diagonal plus a fixed number of distinct uniformly
  random columns per row, values as for the 27-point matrix.
* cell-centred finite-volume diffusion with conductivity exp(g) on a cube,
  harmonic-mean face transmissibilities, Dirichlet faces 2*kappa (SPD).
* a batch of independent 2D / 3D convection-diffusion systems of log-uniform
  size.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSR:
    """A square sparse matrix in CSR form (host arrays)."""

    n: int
    row_ptr: np.ndarray  # int32, n+1
    col_idx: np.ndarray  # int32, nnz
    values: np.ndarray  # float64, nnz
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.values, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def row_of_entry(self) -> np.ndarray:
        """Row index of every stored entry (int64, length nnz)."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))


def _assemble_rows(cols: np.ndarray, vals: np.ndarray, valid: np.ndarray, n: int, meta: dict) -> CSR:
    """Pack per-row candidate entries (n x m arrays, columns already ascending
    along axis 1) into CSR, dropping the invalid ones."""
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    col_idx = cols[valid].astype(np.int32)
    values = vals[valid].astype(np.float64)
    return CSR(n, row_ptr.astype(np.int32), col_idx, values, meta)


def _grid_coords(g: int, dim: int):
    idx = np.arange(g**dim, dtype=np.int64)
    return idx, [(idx // (g**d)) % g for d in range(dim)]


def conv_diff(g: int, dim: int, beta) -> CSR:
    """h^2-scaled central-difference -Lap(u) + beta.grad(u) on a g^dim grid."""
    beta = [float(b) for b in beta][:dim]
    n = g**dim
    h = 1.0 / (g + 1)
    idx, coords = _grid_coords(g, dim)
    # candidate neighbours in ascending linear offset: -e_{dim-1} .. -e_0, 0, +e_0 .. +e_{dim-1}
    plan = [(d, -1) for d in reversed(range(dim))] + [None] + [(d, +1) for d in range(dim)]
    m = len(plan)
    cols = np.empty((n, m), dtype=np.int64)
    vals = np.empty((n, m), dtype=np.float64)
    valid = np.empty((n, m), dtype=bool)
    for j, p in enumerate(plan):
        if p is None:
            cols[:, j] = idx
            vals[:, j] = 2.0 * dim
            valid[:, j] = True
        else:
            d, s = p
            cols[:, j] = idx + s * g**d
            vals[:, j] = -1.0 + s * beta[d] * h / 2.0
            valid[:, j] = (coords[d] + s >= 0) & (coords[d] + s < g)
    return _assemble_rows(cols, vals, valid, n, {"kind": f"convdiff{dim}d", "g": g, "beta": beta})


def conv_diff_2d(g: int = 64, beta=(1.0, 0.5)) -> CSR:
    return conv_diff(g, 2, beta)


def conv_diff_3d(g: int = 128, beta=(1.0, 0.7, 0.3)) -> CSR:
    return conv_diff(g, 3, beta)


def poisson_3d(g: int = 200) -> CSR:
    """7-point Poisson matrix on a g^3 grid (the paper's benchmark matrix)."""
    A = conv_diff(g, 3, (0.0, 0.0, 0.0))
    A.meta["kind"] = "poisson3d"
    return A


def _random_offdiag_values(rng, count: int, factor_noise: float = 0.3):
    u = rng.uniform(-1.0, 0.0, count)
    xi = rng.uniform(-1.0, 1.0, count)
    return u * (1.0 + factor_noise * xi)


def _set_dominant_diagonal(A: CSR, factor: float = 1.05) -> None:
    rows = A.row_of_entry()
    diag = A.col_idx.astype(np.int64) == rows
    absrow = np.zeros(A.n)
    np.add.at(absrow, rows[~diag], np.abs(A.values[~diag]))
    A.values[diag] = factor * absrow[rows[diag]]


def random_27pt(g: int = 100, seed: int = 0) -> CSR:
    """27-point stencil pattern (Dirichlet truncation) with random
    nonsymmetric off-diagonals and a 1.05x dominant diagonal."""
    n = g**3
    idx, (cx, cy, cz) = _grid_coords(g, 3)
    offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    m = len(offs)
    cols = np.empty((n, m), dtype=np.int64)
    valid = np.empty((n, m), dtype=bool)
    for j, (dz, dy, dx) in enumerate(offs):
        cols[:, j] = idx + dz * g * g + dy * g + dx
        valid[:, j] = (
            (cx + dx >= 0) & (cx + dx < g) & (cy + dy >= 0) & (cy + dy < g) & (cz + dz >= 0) & (cz + dz < g)
        )
    vals = np.zeros((n, m))
    A = _assemble_rows(cols, vals, valid, n, {"kind": "random27", "g": g, "seed": seed})
    del cols, vals, valid
    rng = np.random.default_rng(seed)
    rows = A.row_of_entry()
    off = A.col_idx.astype(np.int64) != rows
    A.values[off] = _random_offdiag_values(rng, int(off.sum()))
    _set_dominant_diagonal(A)
    return A


def random_sparse(n: int = 2**21, per_row: int = 15, seed: int = 0) -> CSR:
    """Diagonal plus `per_row` distinct uniformly random off-diagonal columns
    per row, 27-point-style random values, 1.05x dominant diagonal."""
    rng = np.random.default_rng(seed)
    c = rng.integers(0, n - 1, size=(n, per_row), dtype=np.int64)
    rows = np.arange(n, dtype=np.int64)[:, None]
    c = c + (c >= rows)  # skip the diagonal
    c.sort(axis=1)
    dup = np.any(c[:, 1:] == c[:, :-1], axis=1)
    while dup.any():  # redraw rows that drew a column twice
        bad = np.nonzero(dup)[0]
        cc = rng.integers(0, n - 1, size=(bad.size, per_row), dtype=np.int64)
        cc = cc + (cc >= bad[:, None])
        cc.sort(axis=1)
        c[bad] = cc
        dup = np.any(c[:, 1:] == c[:, :-1], axis=1)
    cols = np.concatenate([c, rows], axis=1)
    cols.sort(axis=1)
    valid = np.ones_like(cols, dtype=bool)
    A = _assemble_rows(cols, np.zeros(cols.shape), valid, n, {"kind": "random_sparse", "per_row": per_row, "seed": seed})
    rr = A.row_of_entry()
    off = A.col_idx.astype(np.int64) != rr
    A.values[off] = _random_offdiag_values(rng, int(off.sum()))
    _set_dominant_diagonal(A)
    return A


# ---------------------------------------------------------------- diffusion ---

def gaussian_random_field(g: int, seed: int, sigma: float = 0.5, ell: float = 3.0) -> np.ndarray:
    """White noise smoothed by a separable Gaussian of `ell` cells, rescaled to
    mean 0 and standard deviation `sigma`. Shape (g, g, g) indexed [z, y, x]."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    w = rng.standard_normal((g, g, g))
    f = gaussian_filter(w, sigma=ell, mode="wrap")
    f = (f - f.mean()) / f.std()
    return sigma * f


def diffusion_faces(g: int):
    """Interior faces (P, Q) of a g^3 cell grid, and per-cell counts of
    boundary faces. Returns (P, Q, nbound) with P < Q."""
    idx, coords = _grid_coords(g, 3)
    Ps, Qs = [], []
    nb = np.zeros(g**3, dtype=np.int64)
    for d in range(3):
        inner = coords[d] + 1 < g
        Ps.append(idx[inner])
        Qs.append(idx[inner] + g**d)
        nb += (coords[d] == 0).astype(np.int64) + (coords[d] == g - 1).astype(np.int64)
    return np.concatenate(Ps), np.concatenate(Qs), nb


def diffusion_varcoef(g: int = 64, seed: int = 0, sigma: float = 0.5, ell: float = 3.0):
    """Finite-volume diffusion with conductivity exp(field). Returns (A, field)
    where field has shape (g^3,) in lexicographic cell order."""
    field_ = gaussian_random_field(g, seed, sigma, ell).reshape(-1)
    A = conv_diff(g, 3, (0.0, 0.0, 0.0))  # same 7-point pattern
    A.values[:] = diffusion_values_numpy(A, field_, g)
    A.meta = {"kind": "diffusion_varcoef", "g": g, "seed": seed}
    return A, field_


def _diffusion_entry_map(A: CSR, g: int):
    """For every stored entry: the face it belongs to (or -1 for diagonals)."""
    P, Q, nb = diffusion_faces(g)
    rows = A.row_of_entry()
    cols = A.col_idx.astype(np.int64)
    # face id lookup keyed by (min, max) pair
    key_face = np.minimum(P, Q) * (g**3) + np.maximum(P, Q)
    order = np.argsort(key_face)
    key_sorted = key_face[order]
    key_e = np.minimum(rows, cols) * (g**3) + np.maximum(rows, cols)
    off = rows != cols
    face_of = np.full(A.nnz, -1, dtype=np.int64)
    pos = np.searchsorted(key_sorted, key_e[off])
    face_of[off] = order[pos]
    return P, Q, nb, rows, face_of


def diffusion_values_numpy(A: CSR, field_: np.ndarray, g: int) -> np.ndarray:
    P, Q, nb, rows, face_of = _diffusion_entry_map(A, g)
    kap = np.exp(field_)
    T = 2.0 * kap[P] * kap[Q] / (kap[P] + kap[Q])
    diag = 2.0 * kap * nb
    np.add.at(diag, P, T)
    np.add.at(diag, Q, T)
    vals = np.empty(A.nnz)
    off = face_of >= 0
    vals[off] = -T[face_of[off]]
    vals[~off] = diag[rows[~off]]
    return vals


def diffusion_values_torch(A: CSR, g: int):
    """Return a function field (torch tensor, n) -> CSR values (torch tensor,
    nnz): the same assembly as `diffusion_values_numpy`, written with
    differentiable torch operations so autograd can chain through it."""
    import torch

    P, Q, nb, rows, face_of = _diffusion_entry_map(A, g)
    off = face_of >= 0
    P_t = torch.as_tensor(P)
    Q_t = torch.as_tensor(Q)
    nb_t = torch.as_tensor(nb, dtype=torch.float64)
    off_idx = torch.as_tensor(np.nonzero(off)[0])
    off_face = torch.as_tensor(face_of[off])
    diag_idx = torch.as_tensor(np.nonzero(~off)[0])
    diag_row = torch.as_tensor(rows[~off])
    nnz = A.nnz

    def assemble(field_t):
        dev = field_t.device
        kap = torch.exp(field_t)
        kP, kQ = kap[P_t.to(dev)], kap[Q_t.to(dev)]
        T = 2.0 * kP * kQ / (kP + kQ)
        diag = 2.0 * kap * nb_t.to(dev)
        diag = diag.index_add(0, P_t.to(dev), T).index_add(0, Q_t.to(dev), T)
        vals = torch.zeros(nnz, dtype=field_t.dtype, device=dev)
        vals = vals.index_put((off_idx.to(dev),), -T[off_face.to(dev)])
        vals = vals.index_put((diag_idx.to(dev),), diag[diag_row.to(dev)])
        return vals

    return assemble


# ------------------------------------------------------------------ batches ---

def batched_systems(nsys: int = 64, seed: int = 0, nmin: float = 1e3, nmax: float = 2e5, kmax: int = 8):
    """Independent convection-diffusion systems of log-uniform size.
    Returns a list of (A, k) pairs; one RNG is drawn in a fixed order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nsys):
        n_target = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        dim = 2 if rng.uniform() < 0.5 else 3
        beta = rng.uniform(-1.0, 1.0, 3)
        k = int(rng.integers(1, kmax + 1))
        g = max(3, int(round(n_target ** (1.0 / dim))))
        A = conv_diff(g, dim, beta[:dim])
        out.append((A, k))
    return out


# --------------------------------------------------------------------- RHS ---

def manufactured_rhs(A: CSR, k: int, seed: int):
    """x* ~ U[-1,1]^{n x k} (row-major) and b = A x* in float64."""
    rng = np.random.default_rng(seed)
    xs = rng.uniform(-1.0, 1.0, size=(A.n, k))
    b = np.ascontiguousarray(A.to_scipy() @ xs)
    return b, xs


def uniform_rhs(n: int, k: int, seed: int):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(n, k))


def config_problem(i: int, seed: int = 0, k: int | None = None, scale: int | None = None):
    """The five workload configurations. `scale` overrides the grid size g so
    tests can build the same recipe at a size the CPU oracle finishes fast.

    0: 2D 5-point conv-diff g=64, beta=(1,0.5), k=1, no preconditioner, tol 1e-10
    1: 3D 7-point conv-diff g=128, beta=(1,0.7,0.3), Jacobi, k in 1..32, tol 1e-8
    2: 27-point random g=100, k=32, tol 1e-10 (precision tier)
    3: 64 systems (batched tier), tol 1e-8
    4: 3D variable-coefficient diffusion g=64, k=8 (differentiation tier)
    """
    if i == 0:
        g = scale or 64
        A = conv_diff_2d(g)
        k = k or 1
        b, xs = manufactured_rhs(A, k, seed)
        return {"A": A, "b": b, "x_star": xs, "k": k, "tol": 1e-10, "precond": "none"}
    if i == 1:
        g = scale or 128
        A = conv_diff_3d(g)
        k = k or 32
        b, xs = manufactured_rhs(A, k, seed)
        return {"A": A, "b": b, "x_star": xs, "k": k, "tol": 1e-8, "precond": "jacobi"}
    if i == 2:
        g = scale or 100
        A = random_27pt(g, seed)
        k = k or 32
        b, xs = manufactured_rhs(A, k, seed + 1000)
        return {"A": A, "b": b, "x_star": xs, "k": k, "tol": 1e-10, "precond": "none"}
    if i == 3:
        systems = batched_systems(64 if scale is None else scale, seed)
        rhs = [manufactured_rhs(A, k, seed * 1000 + s) for s, (A, k) in enumerate(systems)]
        return {"systems": systems, "rhs": rhs, "tol": 1e-8, "precond": "none"}
    if i == 4:
        g = scale or 64
        A, fld = diffusion_varcoef(g, seed)
        k = k or 8
        b = uniform_rhs(A.n, k, seed + 7)
        return {"A": A, "field": fld, "g": g, "b": b, "k": k, "tol": 1e-8, "precond": "none"}
    raise ValueError(f"no configuration {i}")
