"""The pressure-correction step with the cross-diffusion term and the
solidification changes to the face gradient (test infrastructure only: the
tests, the smoke check and the benchmark's CPU leg use it; the product path
never does).

What is computed, and where the paper defines it:

* Face gradient (section 2.3, Eq. 12).  At an interior face with owner C1,
  neighbour C2 and vertices V1..V4, a local frame has xi along C1->C2, eta
  along V1->V3 and zeta along V2->V4.  The chain rule gives
      [phi_xi, phi_eta, phi_zeta]^T = J grad(phi),
      J = rows (C2 - C1, V3 - V1, V4 - V2),
  with phi_xi = phi_C2 - phi_C1, phi_eta = phi_V3 - phi_V1,
  phi_zeta = phi_V4 - phi_V2, and each vertex value the mean over the cells
  that share the vertex.  So grad(phi)_f = J^-1 (...) is a linear stencil
  over the face's neighbour cells (every cell sharing a vertex with it).
* Diffusion split (Eq. 11).  n.grad(phi) |S| = c_f (phi_C2 - phi_C1)
  + t_f . grad(phi)_f, with c_f = |S_f|^2 / (rho S_f.d) the direct term
  (given, as in the direct system) and t_f = S_f / rho - c_f d the cross
  vector (n - d/(n.d)) |S| / rho.  t_f = 0 when S_f is parallel to d.
* Solidification (section 2.4.2).  Case 2, an open face with solid cells
  in its stencil: their columns are deleted and their coefficients spread
  equally over the remaining cells (Eq. 15-16).  Case 3, a face with a solid
  owner: all its coefficients are zero, and it carries no flux.
* Pressure equation (Eq. 9 integrated over a cell).  For an active cell i,
      sum_{open f of i} s_if [c_f (p_C2 - p_C1) + t_f . grad(p)_f]
          = (1/dt) sum_{open f of i} s_if F*_f,
  with s_if = +1 if i owns f and -1 otherwise, and F*_f = u*_f . S_f where
  u*_f is the mean of the owners' values (section 2.4.3).  With L the masked
  direct operator (positive semi-definite, as in `assembly`):
      (L - X) p = b,   (X p)_i = sum s_if t_f . grad(p)_f,
      b_i = -(1/dt) sum s_if F*_f.
  The same pins fix the reference level (one per component, p_pin = 0).
* Face flux and velocity correction (Eq. 17 and Eq. 8).
      F_f = F*_f - dt [c_f (p_C2 - p_C1) + t_f . grad(p)_f] on open faces,
      0 on blocked and wall faces;
      u_i = u*_i - (dt/rho) grad(p)_i, with grad(p)_i the mean of the face
      gradients over the cell's open faces.
  At the solution of the pressure equation, every active cell's fluxes sum
  to zero: F is discretely divergence-free.

The exact solution of (L - X) p = b is taken with a sparse LU (the operator
is not symmetric); no deferred correction is involved here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import assembly


@dataclass
class FaceStencil:
    """Per-face gradient stencils in CSR form: face f uses
    cells[ptr[f]:ptr[f+1]] (ascending) with 3-vector coefficients coef[...];
    wall faces have empty rows."""
    ptr: np.ndarray     # int64 [n_faces + 1]
    cells: np.ndarray   # int64 [nnz]
    coef: np.ndarray    # float64 [nnz, 3]

    def row(self, f):
        a, b = self.ptr[f], self.ptr[f + 1]
        return self.cells[a:b], self.coef[a:b]


def vertex_cells(n_nodes, cell_nodes):
    """For each vertex, the ascending ids of the cells that have it as a
    corner."""
    cell_nodes = np.asarray(cell_nodes)
    out = [[] for _ in range(n_nodes)]
    for c in range(cell_nodes.shape[0]):
        for v in cell_nodes[c]:
            out[int(v)].append(c)
    return [np.array(sorted(set(lst)), dtype=np.int64) for lst in out]


def face_stencils(mesh) -> FaceStencil:
    """Eq. 12 stencil of every interior face over its neighbour cells."""
    fn = mesh.extra["face_nodes"]
    vc = vertex_cells(mesh.nodes.shape[0], mesh.extra["cell_nodes"])
    X = mesh.nodes
    C = mesh.cell_centre
    ptr = [0]
    cells, coef = [], []
    for f in range(mesh.n_faces):
        o, n = int(mesh.owner[f]), int(mesh.neigh[f])
        if n < 0:
            ptr.append(ptr[-1])
            continue
        v1, v2, v3, v4 = (int(v) for v in fn[f])
        J = np.array([C[n] - C[o], X[v3] - X[v1], X[v4] - X[v2]])
        G = np.linalg.inv(J)  # column k multiplies the k-th local derivative
        acc = {}

        def add(c, vec):
            acc[c] = acc.get(c, np.zeros(3)) + vec

        add(o, -G[:, 0])
        add(n, G[:, 0])
        for v, col, sgn in ((v3, 1, 1.0), (v1, 1, -1.0), (v4, 2, 1.0), (v2, 2, -1.0)):
            for c in vc[v]:
                add(int(c), sgn * G[:, col] / len(vc[v]))
        ids = sorted(set(int(c) for v in (v1, v2, v3, v4) for c in vc[v]) | {o, n})
        cells.extend(ids)
        coef.extend(acc.get(c, np.zeros(3)) for c in ids)
        ptr.append(ptr[-1] + len(ids))
    return FaceStencil(np.array(ptr, dtype=np.int64), np.array(cells, dtype=np.int64),
                       np.array(coef, dtype=np.float64).reshape(-1, 3))


def smear(cells, coef, active):
    """Case 2 of section 2.4.2 on one stencil row: drop the solid cells and
    add their summed coefficients, divided by the number of remaining cells,
    to each remaining one (Eq. 15 -> Eq. 16)."""
    keep = active[cells]
    if keep.all():
        return cells, coef
    spread = coef[~keep].sum(axis=0) / int(keep.sum())
    return cells[keep], coef[keep] + spread


def masked_stencils(st: FaceStencil, owner, neigh, active) -> FaceStencil:
    """Case 3 (a solid owner: the row is emptied) and case 2 (smearing) on
    every face; rows of faces with both owners active and no solid neighbour
    are unchanged (case 1)."""
    ptr = [0]
    cells, coef = [], []
    for f in range(len(owner)):
        o, n = int(owner[f]), int(neigh[f])
        if n < 0 or not (active[o] and active[n]):
            ptr.append(ptr[-1])
            continue
        c, k = smear(*st.row(f), active)
        cells.extend(c)
        coef.extend(k)
        ptr.append(ptr[-1] + len(c))
    return FaceStencil(np.array(ptr, dtype=np.int64), np.array(cells, dtype=np.int64),
                       np.array(coef, dtype=np.float64).reshape(-1, 3))


def gradient_matrices(st: FaceStencil, n_cells):
    """The three (n_faces x n_cells) matrices that give grad(p)_f."""
    n_faces = len(st.ptr) - 1
    return [sp.csr_matrix((st.coef[:, d], st.cells, st.ptr), shape=(n_faces, n_cells))
            for d in range(3)]


def cross_vectors(mesh, coeff, rho):
    """t_f = S_f / rho - c_f d_f on interior faces (0 on walls)."""
    t = np.zeros((mesh.n_faces, 3))
    inner = mesh.neigh >= 0
    d = mesh.cell_centre[mesh.neigh[inner]] - mesh.cell_centre[mesh.owner[inner]]
    t[inner] = mesh.face_area[inner] / rho - np.asarray(coeff)[inner, None] * d
    return t


def incidence(mesh, open_face):
    """E (n_faces x n_cells): +1 at (f, owner), -1 at (f, neighbour) for open
    faces, so (E^T F)_i is the net outflow of cell i."""
    f = np.nonzero(open_face)[0]
    rows = np.concatenate([f, f])
    cols = np.concatenate([mesh.owner[f], mesh.neigh[f]]).astype(np.int64)
    vals = np.concatenate([np.ones(len(f)), -np.ones(len(f))])
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.n_faces, mesh.n_cells))


def cross_operator(mesh, Gm, t, open_face):
    """X = E^T (sum_d diag(t_d) G_d): (X p)_i = sum s_if t_f . grad(p)_f."""
    E = incidence(mesh, open_face)
    TG = sum(sp.diags(t[:, d] * open_face) @ Gm[d] for d in range(3))
    return (E.T @ TG).tocsr()


def star_flux(mesh, ustar, open_face):
    """F*_f = u*_f . S_f with u*_f the mean of the owners' values; 0 on
    blocked and wall faces."""
    F = np.zeros(mesh.n_faces)
    f = np.nonzero(open_face)[0]
    uf = 0.5 * (ustar[mesh.owner[f]] + ustar[mesh.neigh[f]])
    F[f] = np.einsum("fd,fd->f", uf, mesh.face_area[f])
    return F


@dataclass
class Projection:
    system: assembly.MaskedSystem
    stencil: FaceStencil     # masked (Eq. 16) stencils
    b: np.ndarray            # [n_cells] right-hand side from u* (0 on masked cells)
    p: np.ndarray            # [n_cells] pressure (0 on masked cells and pins)
    grad_f: np.ndarray       # [n_faces, 3] face gradients of p
    flux: np.ndarray         # [n_faces] corrected volume fluxes F_f
    u: np.ndarray            # [n_cells, 3] corrected cell velocities
    full: sp.csr_matrix      # pinned L - X on the active cells


def pinned_full_operator(sy: assembly.MaskedSystem, X):
    """L - X on the active cells, pinned as the direct system is: pin rows
    keep only the direct diagonal, pin columns are removed."""
    Xa = X[sy.perm][:, sy.perm]
    M = (sy.L - Xa).tolil()
    pins = np.nonzero(sy.pinned)[0]
    keep = np.ones(sy.n_active)
    keep[pins] = 0.0
    D = sp.diags(keep)
    M = (D @ M.tocsr() @ D).tolil()
    dA = sy.A.diagonal()
    for k in pins:
        M[k, k] = dA[k]
    return M.tocsr()


def correct(mesh, coeff, stencil: FaceStencil, p, ustar, open_face, rho, dt):
    """Eq. 17 fluxes and Eq. 8 cell velocities for a given pressure."""
    n = mesh.n_cells
    Gm = gradient_matrices(stencil, n)
    grad_f = np.stack([G @ p for G in Gm], axis=1)
    t = cross_vectors(mesh, coeff, rho)
    F = star_flux(mesh, ustar, open_face)
    f = np.nonzero(open_face)[0]
    o, nb = mesh.owner[f], mesh.neigh[f]
    F[f] -= dt * (np.asarray(coeff)[f] * (p[nb] - p[o]) + np.einsum("fd,fd->f", t[f], grad_f[f]))
    # cell gradient: mean of the face gradients over the cell's open faces
    cnt = np.bincount(o, minlength=n) + np.bincount(nb, minlength=n)
    gsum = np.zeros((n, 3))
    for d in range(3):
        gsum[:, d] = (np.bincount(o, weights=grad_f[f, d], minlength=n)
                      + np.bincount(nb, weights=grad_f[f, d], minlength=n))
    u = np.asarray(ustar, dtype=np.float64).copy()
    has = cnt > 0
    u[has] -= (dt / rho) * gsum[has] / cnt[has, None]
    return grad_f, F, u


def project(mesh, coeff, fl, ustar, rho, dt) -> Projection:
    """One pressure-correction step on the masked mesh, solved exactly."""
    ustar = np.asarray(ustar, dtype=np.float64)
    sy = assembly.masked_system(mesh.n_cells, mesh.owner, mesh.neigh, coeff, fl)
    st = masked_stencils(face_stencils(mesh), mesh.owner, mesh.neigh, sy.active)
    Gm = gradient_matrices(st, mesh.n_cells)
    t = cross_vectors(mesh, coeff, rho)
    X = cross_operator(mesh, Gm, t, sy.open_face)
    E = incidence(mesh, sy.open_face)
    b = -(E.T @ star_flux(mesh, ustar, sy.open_face)) / dt
    b[~sy.active] = 0.0
    M = pinned_full_operator(sy, X)
    bp = assembly.pinned_rhs(sy, b)
    pa = spla.spsolve(M.tocsc(), bp) if sy.n_active else np.zeros(0)
    p = assembly.scatter(sy, pa)
    grad_f, F, u = correct(mesh, coeff, st, p, ustar, sy.open_face, rho, dt)
    u[~sy.active] = 0.0
    return Projection(sy, st, b, p, grad_f, F, u, M)


def divergence(mesh, F, open_face):
    """Net outflow E^T F of every cell."""
    return incidence(mesh, open_face).T @ F
