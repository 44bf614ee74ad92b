"""The paper's data-transfer execution-time model (Section 3.1), single node.

TEST INFRASTRUCTURE ONLY (see the package docstring).

On one node the global and local communication terms are negligible (Section
3.2.1), so an iteration costs its memory traffic divided by the node bandwidth
(eq. exec_time): vector operations 8 N m bytes per vector read or write
(Sigma_vec), each SpMV N (8 m (C+1) + 4 (3C+1)) bytes (eq. SpMV_mem), and each
preconditioner application, here the identity (a copy), one vector read and one
write.
"""
from __future__ import annotations

# Merged read+write vector counts per iteration that multiply T_vec in the
# per-method estimates est:bicgstab ... est:ppipebicgstab.
MERGED_VECTOR_OPS = {
    "BiCGStab": 18,
    "IBiCGStab": 20,
    "PipeBiCGStab": 26,
    "PBiCGStab": 19,
    "RBiCGStab": 21,
    "PPipeBiCGStab": 34,
}
# Preconditioner applications per iteration (the three preconditioned methods).
PRECOND_OPS = {"BiCGStab": 0, "IBiCGStab": 0, "PipeBiCGStab": 0, "PBiCGStab": 2, "RBiCGStab": 2, "PPipeBiCGStab": 2}


def spmv_bytes(N: float, m: int, C: float) -> float:
    """eq. SpMV_mem: CRS with 4-byte indices and 8-byte values, m RHS."""
    return N * (8 * m * (C + 1) + 4 * (3 * C + 1))


def vec_bytes(N: float, m: int) -> float:
    """Sigma_vec: one read or one write of an N x m block."""
    return 8 * N * m


def iteration_bytes(method: str, N: float, m: int, C: float) -> float:
    """Bytes one iteration moves: V vector operations, two SpMVs and the
    identity preconditioner (a copy: one read plus one write) P times."""
    V = MERGED_VECTOR_OPS[method]
    P = PRECOND_OPS[method]
    return V * vec_bytes(N, m) + 2 * spmv_bytes(N, m, C) + P * 2 * vec_bytes(N, m)


def iteration_time(method: str, N: float, m: int, C: float, b_bytes_per_s: float) -> float:
    """T = Sigma / B with B = b p and p = 1 (eq. exec_time)."""
    return iteration_bytes(method, N, m, C) / b_bytes_per_s
