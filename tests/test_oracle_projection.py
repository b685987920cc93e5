"""Pins of the pressure-correction oracle (cross diffusion, smearing, flux
and velocity correction) against facts the paper and the mathematics fix:

- Eq. 12 on an affine image of a uniform mesh: vertex means of cell values
  are the vertex values for a linear field, so the face gradient of a linear
  field is exact, although the mesh is not orthogonal.
- Eq. 11: with that exact gradient, direct + cross term give the exact face
  flux g.S_f / rho of a linear pressure, whatever the split.
- Constant fields have zero gradient before and after the smearing of
  section 2.4.2 (coefficients sum to zero).
- The smearing rule is the one the paper spells out for its face F2.
- On a rectilinear mesh S_f is parallel to d, the cross term vanishes and the
  step reduces to the direct system.
- The corrected fluxes (Eq. 17) are discretely divergence-free, and zero on
  blocked and wall faces.
"""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import assembly, projection as pj
from synth import box_mesh, face_coeff, fl_planar_front

RHO, DT = 2400.0, 1e-3
SHEAR = np.array([[1.0, 0.3, 0.1], [0.0, 1.0, 0.25], [0.0, 0.0, 1.0]])
G = np.array([0.7, -1.3, 2.1])


def _sheared():
    m = box_mesh((6, 5, 4), jitter=0.0, affine=SHEAR)
    st = pj.face_stencils(m)
    vc = pj.vertex_cells(m.nodes.shape[0], m.extra["cell_nodes"])
    exact = np.array([m.neigh[f] >= 0 and all(len(vc[v]) == 8 for v in m.extra["face_nodes"][f])
                      for f in range(m.n_faces)])
    return m, st, exact


def test_linear_field_gradient_exact_on_sheared_mesh():
    m, st, exact = _sheared()
    assert exact.sum() > 50
    phi = m.cell_centre @ G
    for f in np.nonzero(exact)[0]:
        c, k = st.row(f)
        assert np.abs(k.T @ phi[c] - G).max() <= 1e-12 * np.abs(G).max(), f
    # the mesh really is non-orthogonal: the cross vectors do not vanish
    t = pj.cross_vectors(m, face_coeff(m, RHO), RHO)
    inner = m.neigh >= 0
    scale = np.linalg.norm(m.face_area[inner], axis=1) / RHO
    assert (np.linalg.norm(t[inner], axis=1) / scale).max() > 0.1


def test_split_gives_exact_flux_of_linear_pressure():
    m, st, exact = _sheared()
    c = face_coeff(m, RHO)
    t = pj.cross_vectors(m, c, RHO)
    p = m.cell_centre @ G
    Gm = pj.gradient_matrices(st, m.n_cells)
    grad = np.stack([M @ p for M in Gm], axis=1)
    f = np.nonzero(exact)[0]
    flux = c[f] * (p[m.neigh[f]] - p[m.owner[f]]) + np.einsum("fd,fd->f", t[f], grad[f])
    ref = m.face_area[f] @ G / RHO
    assert np.abs(flux - ref).max() <= 1e-12 * np.abs(ref).max()


def test_constant_fields_have_zero_gradient_with_and_without_smearing():
    m = box_mesh((7, 6, 5), jitter=0.1, seed=4)
    f = fl_planar_front(m.cell_centre, seed=2)
    st = pj.face_stencils(m)
    ms = pj.masked_stencils(st, m.owner, m.neigh, f > 0)
    for s in (st, ms):
        scale = np.abs(s.coef).max()
        for q in range(m.n_faces):
            _, k = s.row(q)
            if len(k):
                assert np.abs(k.sum(axis=0)).max() <= 1e-13 * scale
    # the front really smears some rows and blocks others
    sizes, msizes = np.diff(st.ptr), np.diff(ms.ptr)
    inner = m.neigh >= 0
    assert np.any((msizes < sizes) & (msizes > 0))
    assert np.any(inner & (msizes == 0))


def test_smearing_rule_of_the_papers_face_f2():
    # seven neighbour cells, the last two solid: each of the five remaining
    # coefficients gains (A6 + A7) / 5, and the solid columns are removed
    rng = np.random.default_rng(1)
    cells = np.arange(10, 17)
    coef = rng.normal(size=(7, 3))
    active = np.ones(20, dtype=bool)
    active[[15, 16]] = False
    c, k = pj.smear(cells, coef, active)
    assert np.array_equal(c, cells[:5])
    assert np.allclose(k, coef[:5] + (coef[5] + coef[6]) / 5, rtol=0, atol=1e-15)


def test_rectilinear_mesh_reduces_to_direct_system():
    m = box_mesh((6, 5, 4), jitter=0.15, seed=1, mode="plane")
    c = face_coeff(m, RHO)
    t = pj.cross_vectors(m, c, RHO)
    assert np.abs(t).max() <= 1e-12 * np.abs(m.face_area).max() / RHO
    f = fl_planar_front(m.cell_centre, seed=5)
    us = np.random.default_rng(2).normal(size=(m.n_cells, 3))
    pr = pj.project(m, c, f, us, RHO, DT)
    sy = pr.system
    pd = assembly.scatter(sy, spla.spsolve(sy.A.tocsc(), assembly.pinned_rhs(sy, pr.b)))
    assert np.abs(pr.p - pd).max() <= 1e-10 * np.abs(pd).max()


def test_velocity_correction_of_linear_pressure():
    m, st, exact = _sheared()
    c = face_coeff(m, RHO)
    us = np.random.default_rng(3).normal(size=(m.n_cells, 3))
    open_face = m.neigh >= 0
    _, _, u = pj.correct(m, c, st, m.cell_centre @ G, us, open_face, RHO, DT)
    # cells all of whose interior faces have exact stencils
    ok = np.ones(m.n_cells, dtype=bool)
    bad = np.nonzero(open_face & ~exact)[0]
    ok[m.owner[bad]] = False
    ok[m.neigh[bad]] = False
    assert ok.sum() > 5
    assert np.abs(u[ok] - (us[ok] - DT / RHO * G)).max() <= 1e-12 * np.abs(us).max()


def test_projection_is_divergence_free_and_respects_the_mask():
    m = box_mesh((8, 7, 6), jitter=0.1, seed=3)
    c = face_coeff(m, RHO)
    f = fl_planar_front(m.cell_centre, seed=2)
    us = np.random.default_rng(0).normal(size=(m.n_cells, 3))
    pr = pj.project(m, c, f, us, RHO, DT)
    sy = pr.system
    fs = pj.star_flux(m, us, sy.open_face)
    div = pj.divergence(m, pr.flux, sy.open_face)
    assert np.abs(div[sy.active]).max() <= 1e-12 * np.abs(fs).max()
    assert np.all(pr.flux[~sy.open_face] == 0)
    assert np.all(pr.u[~sy.active] == 0) and np.all(pr.p[~sy.active] == 0)
    assert np.all(pr.p[sy.pins] == 0)
    # the cross term matters on this mesh: the direct-only pressure differs
    pd = assembly.scatter(sy, spla.spsolve(sy.A.tocsc(), assembly.pinned_rhs(sy, pr.b)))
    assert np.abs(pr.p - pd).max() > 1e-4 * np.abs(pr.p).max()
