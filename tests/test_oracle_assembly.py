"""Pins of the oracle's masked assembly against hand-derived chains, the
operator's invariants, and the closed-form Neumann box solution."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import assembly, closed_form, direct
from synth import box_mesh, face_coeff, fl_linear_x, rhs_uniform

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "chains.json")


def _chain(case):
    n = len(case["fl"])
    owner = np.arange(n - 1, dtype=np.int32)
    neigh = owner + 1
    return n, owner, neigh, np.array(case["c"]), np.array(case["fl"], dtype=float)


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_golden_chains(case):
    n, owner, neigh, c, fl = _chain(case)
    sy = assembly.masked_system(n, owner, neigh, c, fl)
    assert len(sy.pins) == case["n_components"]
    p = direct.solve_dense(sy, np.array(case["b"]))
    ref = np.array(case["p"])
    assert np.allclose(p, ref, rtol=1e-14, atol=1e-14 * max(1.0, np.abs(ref).max()))
    assert np.all(p[np.array(case["fl"]) == 0] == 0)


def _c1(jitter=0.1, mode="node"):
    m = box_mesh((16, 16, 16), jitter=jitter, seed=0, mode=mode)
    fl = fl_linear_x(m.cell_centre)
    return m, fl, face_coeff(m, 2400.0)


def test_c1_invariants():
    m, fl, c = _c1()
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, fl)
    A, L = sy.A, sy.L
    assert sy.n_active == 2816
    assert L.nnz == 2816 + 2 * 7840
    assert int(sy.open_face.sum()) == 7840
    inner = m.neigh >= 0
    # faces joining a solid and an active cell: the 16 x 16 front
    front = inner & (fl[m.owner] > 0) != (fl[np.maximum(m.neigh, 0)] > 0)
    assert int((front & inner).sum()) == 256
    assert (A != A.T).nnz == 0                       # bitwise symmetric
    d = A.diagonal()
    assert np.all(d > 0)
    off = A - np.diag(d)
    assert off.max() <= 0.0
    # Neumann walls AND Neumann front: zero row sums away from the pin
    rs = np.asarray(L.sum(axis=1)).ravel()
    assert np.all(np.abs(rs) <= 8 * np.finfo(float).eps * sy.diag_L)
    pin_c = sy.cid[sy.pins]
    near_pin = np.unique(np.concatenate([L[pin_c].indices, pin_c]))
    rsA = np.asarray(A.sum(axis=1)).ravel()
    far = np.setdiff1d(np.arange(sy.n_active), near_pin)
    assert np.all(np.abs(rsA[far]) <= 8 * np.finfo(float).eps * d[far])
    # rows next to the pin keep the pin's coefficient on the diagonal only
    nb = np.setdiff1d(near_pin, pin_c)
    assert np.all(rsA[nb] > 0)
    sla.cholesky(A.toarray(), lower=True)            # SPD
    # a Dirichlet front would leave a positive row sum at every front cell
    front_cells = np.unique(m.neigh[front & inner])
    assert np.all(np.abs(rs[sy.cid[front_cells]]) <= 8 * np.finfo(float).eps * sy.diag_L[sy.cid[front_cells]])


def test_diagonal_is_ordered_sum():
    """Diagonal = open-face coefficients added one by one in ascending
    neighbour order (the order the device assembly also uses)."""
    m, fl, c = _c1()
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, fl)
    rng = np.random.default_rng(0)
    for i in rng.choice(sy.n_active, 50, replace=False):
        cell = sy.perm[i]
        faces = np.nonzero(sy.open_face & ((m.owner == cell) | (m.neigh == cell)))[0]
        other = np.where(m.owner[faces] == cell, m.neigh[faces], m.owner[faces])
        acc = 0.0
        for f in faces[np.lexsort((faces, other))]:
            acc = acc + c[f]
        assert acc == sy.diag_L[i] == sy.A[i, i] or sy.pinned[i]


def test_closed_form_neumann_box():
    """Unjittered mesh + face-aligned front: the active set is a box and
    the pinned solution is the DCT solution shifted to 0 at the pin."""
    m, fl, c = _c1(jitter=0.0, mode=None)
    b = rhs_uniform(m.n_cells, seed=1, center_mask=fl > 0)
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, fl)
    p = direct.solve_dense(sy, b)
    gi = m.grid_index
    act = fl > 0
    lo = gi[act].min(axis=0)
    box = np.zeros(tuple(gi[act].max(axis=0) - lo + 1))
    bb = np.zeros_like(box)
    idx = tuple((gi[act] - lo).T)
    bb[idx] = b[act]
    pin = tuple(gi[sy.pins[0]] - lo)
    bb[pin] = 0.0
    bb[pin] = -bb.sum()          # the pinned row is dropped; restore balance
    h = 1.0 / 16
    ref = closed_form.neumann_box_solve(bb, (h / 2400.0,) * 3, pin)
    box[idx] = p[act]
    assert np.abs(box - ref).max() <= 1e-12 * np.abs(ref).max()


def test_sparse_and_dense_direct_agree():
    m, fl, c = _c1()
    b = rhs_uniform(m.n_cells, seed=1, center_mask=fl > 0)
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, fl)
    p1 = direct.solve_dense(sy, b)
    p2 = direct.solve_sparse(sy, b)
    assert np.linalg.norm(p1 - p2) <= 1e-12 * np.linalg.norm(p1)
    assert assembly.relative_residual(sy, b, p1) <= 1e-13
    assert np.all(p1[~(fl > 0)] == 0) and np.all(p1[sy.pins] == 0)


@pytest.mark.parametrize("bad", ["owner", "coef", "nan_fl", "fl_range", "equal"])
def test_validation(bad):
    n, owner, neigh = 3, np.array([0, 1]), np.array([1, 2])
    c, fl = np.array([1.0, 1.0]), np.array([1.0, 1.0, 1.0])
    if bad == "owner":
        owner = np.array([0, 3])
    elif bad == "coef":
        c = np.array([1.0, -1.0])
    elif bad == "nan_fl":
        fl = np.array([1.0, np.nan, 1.0])
    elif bad == "fl_range":
        fl = np.array([1.0, 1.5, 1.0])
    else:
        neigh = np.array([0, 2])
    with pytest.raises(ValueError):
        assembly.masked_system(n, owner, neigh, c, fl)
