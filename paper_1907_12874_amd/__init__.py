"""MI355X multi-right-hand-side BiCGStab (classical, Reordered, Pipelined,
Improved; basic, merged and fused forms), a HIP library for gfx950 behind a
C ABI.

The compute path is the in-tree libbicgstab.so; there is no CPU fallback.
"""
from ._lib import BicgstabError, lib  # noqa: F401
from .solver import Solver, SolveInfo, axpby_tab1, plan_traffic  # noqa: F401
from . import batched  # noqa: F401
from .batched import BatchedSolver  # noqa: F401


def load():
    """Load the native library (raises if it is not built)."""
    return lib()
