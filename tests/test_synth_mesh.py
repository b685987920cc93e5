"""Pins of the synthetic mesh generator: closure, volume, orientation,
counts, jitter bound and seeded determinism."""
import numpy as np
import pytest

from synth import box_mesh, plate_with_ribs_mesh, concat_meshes, face_coeff, fl_linear_x


def _closure(m):
    S = np.zeros((m.n_cells, 3))
    np.add.at(S, m.owner, m.face_area)
    inner = m.neigh >= 0
    np.add.at(S, m.neigh[inner], -m.face_area[inner])
    return np.abs(S).max()


@pytest.mark.parametrize("n", [1, 2, 3, 16])
@pytest.mark.parametrize("mode", ["node", "plane", None])
def test_closed_cells_and_unit_volume(n, mode):
    m = box_mesh((n, n, n), jitter=0.1, seed=0, mode=mode)
    h = 1.0 / n
    assert _closure(m) <= 1e-15 * 10 * h * h + 1e-18
    assert abs(m.cell_volume.sum() - 1.0) <= 1e-14
    assert m.cell_volume.min() > 0
    assert m.n_faces == 6 * n * n * n - 3 * n * n * (n - 1)  # each interior face once


def test_c1_counts_and_active_cells():
    m = box_mesh((16, 16, 16), jitter=0.1, seed=0)
    assert m.n_cells == 4096
    assert m.n_interior == 11520
    assert m.n_faces - m.n_interior == 1536
    fl = fl_linear_x(m.cell_centre)
    # jitter <= 0.1h cannot move a centre across x = 0.3
    assert int((fl > 0).sum()) == 2816


def test_orientation_and_coefficients_positive():
    m = box_mesh((8, 8, 8), jitter=0.1, seed=3)
    inner = m.neigh >= 0
    d = m.cell_centre[m.neigh[inner]] - m.cell_centre[m.owner[inner]]
    assert np.all(np.einsum("fd,fd->f", m.face_area[inner], d) > 0)
    assert np.all(m.owner[inner] < m.neigh[inner])
    c = face_coeff(m, 2400.0)
    assert np.all(c[inner] > 0) and np.all(c[~inner] == 0)
    # unjittered: c = h^2 / (rho h) = h / rho exactly up to rounding
    u = box_mesh((8, 8, 8), jitter=0.0, mode=None)
    cu = face_coeff(u, 2400.0)[u.neigh >= 0]
    assert np.allclose(cu, (1 / 8) / 2400.0, rtol=1e-13)


def test_jitter_bound_and_determinism():
    a = box_mesh((6, 5, 4), jitter=0.1, seed=7)
    b = box_mesh((6, 5, 4), jitter=0.1, seed=7)
    u = box_mesh((6, 5, 4), jitter=0.0, mode=None)
    assert np.array_equal(a.nodes, b.nodes)
    h = np.array([1 / 6, 1 / 5, 1 / 4])
    assert np.all(np.abs(a.nodes - u.nodes) <= 0.1 * h + 1e-15)
    # boundary nodes do not move
    on_wall = np.any((np.abs(u.nodes) < 1e-12) | (np.abs(u.nodes - 1) < 1e-12), axis=1)
    assert np.array_equal(a.nodes[on_wall], u.nodes[on_wall])


def test_plate_with_ribs_size():
    m = plate_with_ribs_mesh(plate=(24, 12, 4), rib_cells=2, rib_height=3, n_ribs=2)
    assert m.n_cells == 24 * 12 * 4 + 2 * 2 * 12 * 3
    assert _closure(m) < 1e-18


def test_concat_offsets():
    ms = [box_mesh((2, 2, 2), seed=1), box_mesh((3, 2, 2), seed=2)]
    u = concat_meshes(ms)
    assert u.n_cells == 8 + 12
    assert list(u.extra["cell_offsets"]) == [0, 8, 20]
    inner = u.neigh >= 0
    assert u.owner[inner].max() < 20
    # no face couples the two samples
    s_of = np.searchsorted(u.extra["cell_offsets"], np.arange(20), side="right") - 1
    assert np.all(s_of[u.owner[inner]] == s_of[u.neigh[inner]])
