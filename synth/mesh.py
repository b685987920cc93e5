"""Jittered hexahedral meshes stored as unstructured face lists.

A mesh is a set of hexahedral cells taken from a logical ``mx x my x mz``
block (optionally with cells removed), with every cell face listed once.
An interior face has two owners, ``owner < neigh``; a wall face has
``neigh == -1``.  This matches the collocated cell-centred finite-volume
layout of the paper's section 2.3 (two cells C1, C2 share a face f with
vertices V1..V4; n is the unit normal pointing out of C1, d the vector from
C1 to C2).

Geometry definitions, chosen where the paper is silent:
  * cell centre  = mean of the 8 vertices;
  * face centre  = mean of the 4 vertices;
  * face vector area S_f = (V3 - V1) x (V4 - V2) / 2, i.e. built from the two
    face diagonals that the paper uses as the eta and zeta axes; it points
    from ``owner`` to ``neigh`` (outward of the owner);
  * cell volume  = (1/3) sum_f x_f . S_f(outward)  (divergence theorem).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class HexMesh:
    n_cells: int
    owner: np.ndarray          # int32 [n_faces]
    neigh: np.ndarray          # int32 [n_faces], -1 on walls
    face_area: np.ndarray      # float64 [n_faces, 3], owner -> neigh
    face_centre: np.ndarray    # float64 [n_faces, 3]
    cell_centre: np.ndarray    # float64 [n_cells, 3]
    cell_volume: np.ndarray    # float64 [n_cells]
    nodes: np.ndarray          # float64 [n_nodes, 3]
    grid_index: np.ndarray     # int32 [n_cells, 3], (i, j, k) in the logical block
    shape: tuple               # logical block (mx, my, mz)
    spacing: tuple             # unjittered (hx, hy, hz)
    extra: dict = field(default_factory=dict)

    @property
    def n_faces(self) -> int:
        return int(self.owner.shape[0])

    @property
    def n_interior(self) -> int:
        return int(np.count_nonzero(self.neigh >= 0))


# (axis, first in-plane axis, second in-plane axis), cyclic so that the
# vertex order below gives a normal along +axis.
_AXES = ((0, 1, 2), (1, 2, 0), (2, 0, 1))
_QUAD = ((0, 0), (1, 0), (1, 1), (0, 1))


def _node_id(idx, nshape):
    nx, ny, _ = nshape
    return idx[0] + nx * (idx[1] + ny * idx[2])


def _face_nodes(cells_ijk, axis, plane_offset, nshape, reverse):
    """Node ids [k, 4] of the face of each cell that lies on node plane
    ``i_axis + plane_offset``, ordered for a normal along +axis (or -axis
    when ``reverse``)."""
    a, b, c = _AXES[axis]
    out = np.empty((cells_ijk.shape[0], 4), dtype=np.int64)
    for q, (ob, oc) in enumerate(_QUAD):
        idx = [None, None, None]
        idx[a] = cells_ijk[:, a] + plane_offset
        idx[b] = cells_ijk[:, b] + ob
        idx[c] = cells_ijk[:, c] + oc
        out[:, q] = _node_id(idx, nshape)
    if reverse:
        out = out[:, [0, 3, 2, 1]]
    return out


def box_mesh(shape, lengths=(1.0, 1.0, 1.0), jitter=0.1, seed=0, mode="node",
             keep=None, origin=(0.0, 0.0, 0.0), affine=None) -> HexMesh:
    """Hex mesh of a logical block, stored as an unstructured face list.

    shape   : (mx, my, mz) cells of the logical block.
    lengths : physical size of the block.
    jitter  : displacement bound as a fraction of the local spacing.
    mode    : "node"  - every node strictly inside the block moves by an
                        independent U(-jitter*h, +jitter*h) per coordinate;
              "plane" - each interior node plane moves as a whole
                        (rectilinear mesh, faces stay axis-aligned);
              None    - no jitter.
    keep    : optional bool [mx, my, mz]; cells left out are not meshed and
              their faces towards kept cells become walls.
    affine  : optional 3x3 matrix applied to every node after the jitter
              (x -> affine @ x), e.g. a shear that makes a uniform mesh
              non-orthogonal while keeping its cells affine images of cubes.
    Cells are numbered in the order c = i + mx*(j + my*k) among kept cells.
    """
    mx, my, mz = (int(s) for s in shape)
    lx, ly, lz = (float(v) for v in lengths)
    h = np.array([lx / mx, ly / my, lz / mz])
    nshape = (mx + 1, my + 1, mz + 1)
    rng = np.random.default_rng(seed)

    axes = [origin[d] + h[d] * np.arange(nshape[d], dtype=np.float64) for d in range(3)]
    if mode == "plane" and jitter:
        for d in range(3):
            disp = rng.uniform(-1.0, 1.0, size=nshape[d]) * (jitter * h[d])
            disp[0] = disp[-1] = 0.0
            axes[d] = axes[d] + disp
    X, Y, Z = np.meshgrid(axes[0], axes[1], axes[2], indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)  # [nx, ny, nz, 3]
    if mode == "node" and jitter:
        disp = rng.uniform(-1.0, 1.0, size=P.shape) * (jitter * h)
        inner = np.zeros(nshape, dtype=bool)
        inner[1:-1, 1:-1, 1:-1] = True
        P = P + disp * inner[..., None]
    elif mode not in ("node", "plane", None):
        raise ValueError(f"unknown jitter mode {mode!r}")
    nodes = P.reshape(-1, 3, order="F")  # node id = i + nx*(j + ny*k)
    if affine is not None:
        nodes = nodes @ np.asarray(affine, dtype=np.float64).T

    if keep is None:
        keep = np.ones((mx, my, mz), dtype=bool)
    keep = np.asarray(keep, dtype=bool)
    assert keep.shape == (mx, my, mz)
    keep_flat = keep.ravel(order="F")
    cell_id = np.full(mx * my * mz, -1, dtype=np.int64)
    cell_id[keep_flat] = np.arange(int(keep_flat.sum()))
    cell_id = cell_id.reshape((mx, my, mz), order="F")
    n_cells = int(keep_flat.sum())
    ii, jj, kk = np.meshgrid(np.arange(mx), np.arange(my), np.arange(mz), indexing="ij")
    ijk_all = np.stack([ii.ravel(order="F"), jj.ravel(order="F"), kk.ravel(order="F")], axis=1)
    cells_ijk = ijk_all[keep_flat]

    owners, neighs, fnodes = [], [], []
    # interior faces, x then y then z
    for axis in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        both = keep[tuple(lo)] & keep[tuple(hi)]
        o = cell_id[tuple(lo)][both]
        n = cell_id[tuple(hi)][both]
        # reorder by owner id so faces follow cell order
        order = np.argsort(o, kind="stable")
        o, n = o[order], n[order]
        owners.append(o)
        neighs.append(n)
        fnodes.append(_face_nodes(cells_ijk[o], axis, 1, nshape, reverse=False))
    # wall faces: +axis side then -axis side of each kept cell
    for axis in range(3):
        for side in (+1, -1):
            ijk = cells_ijk
            nb = ijk[:, axis] + side
            inside = (nb >= 0) & (nb < shape[axis])
            has_nb = np.zeros(n_cells, dtype=bool)
            idx = ijk[inside].copy()
            idx[:, axis] = nb[inside]
            has_nb[inside] = keep[idx[:, 0], idx[:, 1], idx[:, 2]]
            wall = np.nonzero(~has_nb)[0]
            owners.append(wall.astype(np.int64))
            neighs.append(np.full(wall.shape[0], -1, dtype=np.int64))
            fnodes.append(_face_nodes(ijk[wall], axis, 1 if side > 0 else 0, nshape,
                                      reverse=(side < 0)))
    owner = np.concatenate(owners).astype(np.int32)
    neigh = np.concatenate(neighs).astype(np.int32)
    fn = np.concatenate(fnodes)

    V = nodes[fn]  # [n_faces, 4, 3]
    face_area = 0.5 * np.cross(V[:, 2] - V[:, 0], V[:, 3] - V[:, 1])
    face_centre = V.mean(axis=1)

    corner = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                       [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]])
    cn = np.stack([_node_id([cells_ijk[:, 0] + c[0], cells_ijk[:, 1] + c[1],
                             cells_ijk[:, 2] + c[2]], nshape) for c in corner], axis=1)
    cell_centre = nodes[cn].mean(axis=1)

    flux = np.einsum("fd,fd->f", face_centre, face_area) / 3.0
    vol = np.bincount(owner, weights=flux, minlength=n_cells)
    inner = neigh >= 0
    vol -= np.bincount(neigh[inner], weights=flux[inner], minlength=n_cells)

    out = HexMesh(n_cells=n_cells, owner=owner, neigh=neigh, face_area=face_area,
                  face_centre=face_centre, cell_centre=cell_centre, cell_volume=vol,
                  nodes=nodes, grid_index=cells_ijk.astype(np.int32),
                  shape=(mx, my, mz), spacing=tuple(h.tolist()))
    # vertex lists: a face's V1..V4 (V1->V3 and V2->V4 are its diagonals) and
    # a cell's eight corners
    out.extra["face_nodes"] = fn.astype(np.int32)
    out.extra["cell_nodes"] = cn.astype(np.int32)
    return out


def plate_with_ribs_mesh(h=2.0e-3 / 3.0, plate=(240, 144, 36), rib_cells=8,
                         rib_height=56, n_ribs=4, jitter=0.05, seed=0) -> HexMesh:
    """Plate with ribs: a plate of ``plate`` cells at spacing ``h`` (default
    160 x 96 x 24 mm at 2/3 mm) carrying ``n_ribs`` ribs, each ``rib_cells``
    cells thick along x, spanning the plate in y and standing ``rib_height``
    cells on top, evenly spaced along x.  Default: 1,502,208 cells."""
    px, py, pz = plate
    mz = pz + rib_height
    keep = np.zeros((px, py, mz), dtype=bool)
    keep[:, :, :pz] = True
    for q in range(n_ribs):
        centre = (2 * q + 1) * px // (2 * n_ribs)
        keep[centre - rib_cells // 2: centre + rib_cells // 2, :, pz:] = True
    return box_mesh((px, py, mz), lengths=(px * h, py * h, mz * h), jitter=jitter,
                    seed=seed, mode="node", keep=keep)


def concat_meshes(meshes):
    """Block-diagonal union of independent meshes (cell ids offset).  Returns
    the union mesh; ``extra['cell_offsets']`` and ``extra['face_offsets']``
    give each sample's range."""
    cell_off = np.zeros(len(meshes) + 1, dtype=np.int64)
    face_off = np.zeros(len(meshes) + 1, dtype=np.int64)
    node_off = 0
    owners, neighs, fa, fc, cc, cv, nodes, gi = [], [], [], [], [], [], [], []
    fnodes, cnodes = [], []
    for s, m in enumerate(meshes):
        c0 = cell_off[s]
        owners.append(m.owner.astype(np.int64) + c0)
        nb = m.neigh.astype(np.int64)
        neighs.append(np.where(nb >= 0, nb + c0, -1))
        fa.append(m.face_area)
        fc.append(m.face_centre)
        cc.append(m.cell_centre)
        cv.append(m.cell_volume)
        nodes.append(m.nodes)
        gi.append(m.grid_index)
        if "face_nodes" in m.extra:
            fnodes.append(m.extra["face_nodes"].astype(np.int64) + node_off)
            cnodes.append(m.extra["cell_nodes"].astype(np.int64) + node_off)
        node_off += m.nodes.shape[0]
        cell_off[s + 1] = c0 + m.n_cells
        face_off[s + 1] = face_off[s] + m.n_faces
    if cell_off[-1] >= 2**31 - 1:
        raise ValueError("union mesh too large for int32 cell ids")
    out = HexMesh(n_cells=int(cell_off[-1]),
                  owner=np.concatenate(owners).astype(np.int32),
                  neigh=np.concatenate(neighs).astype(np.int32),
                  face_area=np.concatenate(fa), face_centre=np.concatenate(fc),
                  cell_centre=np.concatenate(cc), cell_volume=np.concatenate(cv),
                  nodes=np.concatenate(nodes), grid_index=np.concatenate(gi),
                  shape=None, spacing=None)
    out.extra["cell_offsets"] = cell_off
    out.extra["face_offsets"] = face_off
    if len(fnodes) == len(meshes):
        out.extra["face_nodes"] = np.concatenate(fnodes).astype(np.int32)
        out.extra["cell_nodes"] = np.concatenate(cnodes).astype(np.int32)
    return out


def face_coeff(mesh: HexMesh, rho: float) -> np.ndarray:
    """Direct-term face coefficient of the diffusion split (section 2.3,
    Eq. 11, first term): c_f = |S_f| / (rho * n.d) with n = S_f/|S_f| and d
    the owner-to-neighbour centre vector, i.e. |S_f|^2 / (rho * S_f.d).
    Walls get 0."""
    c = np.zeros(mesh.n_faces, dtype=np.float64)
    inner = mesh.neigh >= 0
    S = mesh.face_area[inner]
    d = mesh.cell_centre[mesh.neigh[inner]] - mesh.cell_centre[mesh.owner[inner]]
    c[inner] = np.einsum("fd,fd->f", S, S) / (rho * np.einsum("fd,fd->f", S, d))
    return c
