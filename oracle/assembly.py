"""Masked pressure system: active set, open faces, components, pins, matrix.

Test infrastructure only (see the package docstring).

The pressure Poisson equation (paper Eq. 9) is discretised on the collocated
finite-volume mesh with the direct term of the diffusion split (Eq. 11,
first term), so face f between cells o and n contributes
    c_f * (p_n - p_o),   c_f = |S_f| / (rho * n.d)    (given as input)
to the balance of cell o and the negative to that of n.  Section 2.4.2 then
changes the system for solidification:
  * rows of fully solid cells are deleted (tag S, here f_l == 0);
  * a face with at least one solid owner is blocked: its flux is zero, which
    is a Neumann condition, so the face's coefficient leaves the diagonal as
    well as the off-diagonal (case 3; modification step 2);
  * the remaining rows are re-assembled from their open faces (step 3).
Wall faces carry no flux (Neumann walls).  The resulting operator is
singular on each connected set of active cells; this implementation fixes
the reference level by pinning one cell per component (its lowest original
index) to zero, the reading used throughout this project.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclass
class MaskedSystem:
    n_cells: int
    active: np.ndarray      # bool [n_cells]
    cid: np.ndarray         # int64 [n_cells], compact id or -1
    perm: np.ndarray        # int64 [n_active], compact -> original
    open_face: np.ndarray   # bool [n_faces]
    comp: np.ndarray        # int64 [n_active], component label = pin's original index
    pins: np.ndarray        # int64 [n_components], original indices, ascending
    pinned: np.ndarray      # bool [n_active]
    diag_L: np.ndarray      # float64 [n_active], unpinned diagonal
    L: sp.csr_matrix        # unpinned operator on the active cells
    A: sp.csr_matrix        # pinned operator (what is solved)

    @property
    def n_active(self) -> int:
        return int(self.perm.shape[0])


def validate(n_cells, owner, neigh, coeff, fl):
    """Argument rules of the solver's boundary; raises ValueError."""
    owner = np.asarray(owner)
    neigh = np.asarray(neigh)
    if n_cells <= 0:
        raise ValueError("n_cells must be positive")
    if owner.shape != neigh.shape:
        raise ValueError("owner/neigh size mismatch")
    if owner.size and (owner.min() < 0 or owner.max() >= n_cells):
        raise ValueError("owner out of range")
    if neigh.size and (neigh.min() < -1 or neigh.max() >= n_cells):
        raise ValueError("neigh out of range")
    if np.any(owner == neigh):
        raise ValueError("face with equal owners")
    inner = neigh >= 0
    c = np.asarray(coeff)[inner]
    if not np.all(np.isfinite(c)) or np.any(c <= 0):
        raise ValueError("face coefficient must be finite and > 0 on interior faces")
    fl = np.asarray(fl)
    if not np.all(np.isfinite(fl)) or np.any(fl < 0) or np.any(fl > 1):
        raise ValueError("liquid fraction must be finite and in [0, 1]")


def masked_system(n_cells, owner, neigh, coeff, fl) -> MaskedSystem:
    validate(n_cells, owner, neigh, coeff, fl)
    owner = np.asarray(owner, dtype=np.int64)
    neigh = np.asarray(neigh, dtype=np.int64)
    coeff = np.asarray(coeff, dtype=np.float64)
    fl = np.asarray(fl, dtype=np.float64)

    # 1. active set: LM cells (liquid or mushy), i.e. f_l > 0
    active = fl > 0.0
    n_a = int(active.sum())
    cid = np.full(n_cells, -1, dtype=np.int64)
    cid[active] = np.arange(n_a)
    perm = np.nonzero(active)[0]

    # 2. a face is open iff it is interior and both owners are active
    inner = neigh >= 0
    open_face = np.zeros(owner.shape[0], dtype=bool)
    open_face[inner] = active[owner[inner]] & active[neigh[inner]]
    f = np.nonzero(open_face)[0]
    o, nb, c = owner[f], neigh[f], coeff[f]

    # 3. unpinned operator.  Both half-edges of every open face:
    rows = np.concatenate([o, nb])
    cols = np.concatenate([nb, o])
    vals = np.concatenate([c, c])
    fids = np.concatenate([f, f])
    # Diagonal: sum of the row's open-face coefficients, added one at a time
    # in ascending (neighbour index, face index) order.
    order = np.lexsort((fids, cols, rows))
    rows_s, vals_s = rows[order], vals[order]
    counts = np.bincount(cid[rows_s], minlength=n_a) if n_a else np.zeros(0, np.int64)
    width = int(counts.max()) if counts.size else 0
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]]) if n_a else np.zeros(0, np.int64)
    pos = np.arange(rows_s.shape[0]) - starts[cid[rows_s]]
    table = np.zeros((n_a, max(width, 1)))
    table[cid[rows_s], pos] = vals_s
    diag = table[:, 0].copy()
    for k in range(1, width):
        diag = diag + table[:, k]
    L = sp.coo_matrix((-vals, (cid[rows], cid[cols])), shape=(n_a, n_a)).tocsr()
    L = (L + sp.diags(diag, format="csr")).tocsr()
    L.sort_indices()

    # 4. connected components of the open-face graph; pin = lowest index
    if n_a:
        G = sp.coo_matrix((np.ones(f.shape[0]), (cid[o], cid[nb])), shape=(n_a, n_a))
        n_comp, labels = connected_components(G, directed=False)
        pin_of = np.full(n_comp, np.iinfo(np.int64).max)
        np.minimum.at(pin_of, labels, perm)
        comp = pin_of[labels]
        pins = np.sort(pin_of)
    else:
        comp = np.zeros(0, np.int64)
        pins = np.zeros(0, np.int64)
    pinned = np.zeros(n_a, dtype=bool)
    pinned[cid[pins]] = True

    # 5. pinned operator: zero the pin's row and column, keep its diagonal
    # (1 for a singleton, whose diagonal is 0)
    Lc = L.tocoo()
    keep = (Lc.row == Lc.col) | (~pinned[Lc.row] & ~pinned[Lc.col])
    A = sp.coo_matrix((Lc.data[keep], (Lc.row[keep], Lc.col[keep])), shape=(n_a, n_a)).tocsr()
    A.sort_indices()
    d = A.diagonal()
    fix = pinned & (d == 0.0)
    if fix.any():
        A = (A + sp.diags(np.where(fix, 1.0, 0.0), format="csr")).tocsr()
        A.sort_indices()

    return MaskedSystem(n_cells=n_cells, active=active, cid=cid, perm=perm,
                        open_face=open_face, comp=comp, pins=pins, pinned=pinned,
                        diag_L=diag, L=L, A=A)


def pinned_rhs(system: MaskedSystem, b) -> np.ndarray:
    """b' on the active cells: b restricted to active rows, 0 at every pin."""
    bp = np.asarray(b, dtype=np.float64)[system.perm].copy()
    bp[system.pinned] = 0.0
    return bp


def scatter(system: MaskedSystem, p_active) -> np.ndarray:
    """Full-length pressure: 0 on masked cells and at pins."""
    p = np.zeros(system.n_cells)
    p[system.perm] = p_active
    p[system.pins] = 0.0
    return p


def relative_residual(system: MaskedSystem, b, p_full) -> float:
    """||b' - A p|| / ||b'|| on the compact pinned system (0 if b' = 0)."""
    bp = pinned_rhs(system, b)
    r = bp - system.A @ np.asarray(p_full)[system.perm]
    nb = np.linalg.norm(bp)
    return float(np.linalg.norm(r) / nb) if nb > 0 else float(np.linalg.norm(r))
