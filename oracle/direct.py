"""Exact references for the pinned pressure system.

Test infrastructure only (see the package docstring).  The pinned operator
is symmetric positive definite, so a dense Cholesky factorisation solves it
exactly up to rounding; SuperLU covers larger meshes.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .assembly import MaskedSystem, pinned_rhs, scatter


def solve_dense(system: MaskedSystem, b) -> np.ndarray:
    """Dense Cholesky solve (small meshes).  Returns the full-length p."""
    bp = pinned_rhs(system, b)
    if system.n_active == 0:
        return np.zeros(system.n_cells)
    c = sla.cho_factor(system.A.toarray(), lower=True)
    return scatter(system, sla.cho_solve(c, bp))


def solve_sparse(system: MaskedSystem, b) -> np.ndarray:
    """SuperLU solve.  Returns the full-length p."""
    bp = pinned_rhs(system, b)
    if system.n_active == 0:
        return np.zeros(system.n_cells)
    lu = spla.splu(system.A.tocsc())
    return scatter(system, lu.solve(bp))
