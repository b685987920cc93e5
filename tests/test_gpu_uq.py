"""GPU parity of the collocation wrapper (section 3, Eq. 27-28) against the
oracle:

- least-squares coefficients, evaluation at Latin-hypercube points and the
  mean / variance / Sobol indices of many outputs at once, against numpy's
  least squares and the oracle's statistics (1e-12), with term counts,
  sample counts and output counts that cross the kernel's tiles;
- a collocation over batched pressure solves: the fields of 27 tensor
  samples of three inputs (melt and wall temperature normal, liquidus shift
  uniform) on one mesh, fitted on the GPU and by the oracle from the same
  solved fields;
- too few or repeated points are rejected.
"""
import numpy as np
import pytest

from oracle import uq
from synth import box_mesh, concat_meshes, face_coeff, latin_hypercube, rhs_smooth_series, uq_front_fl
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu
KINDS = ["normal", "normal", "uniform"]
OK = [uq.NORMAL, uq.NORMAL, uq.UNIFORM]


def test_fit_eval_stats_match_oracle():
    import torch

    import paper_1810_08572_amd as ppe

    q = ppe.PolynomialChaos(KINDS, 3)
    assert q.n_terms == 20
    X, _ = q.nodes("smolyak", 4)
    assert X.shape[0] == 69
    rng = np.random.default_rng(2)
    n_out = 5003
    Y = rng.normal(size=(X.shape[0], n_out))
    W = q.fit(X, to_dev(Y, torch.float64)).cpu().numpy()
    al = uq.total_degree_indices(3, 3)
    Wo = uq.fit(uq.vandermonde(OK, al, X), Y)
    assert np.abs(W - Wo).max() <= 1e-12 * np.abs(Wo).max()
    T, _ = latin_hypercube(KINDS, 60, seed=4)
    Ye = q.eval(T, to_dev(Wo, torch.float64)).cpu().numpy()
    Yo = uq.vandermonde(OK, al, T) @ Wo
    assert np.abs(Ye - Yo).max() <= 1e-12 * np.abs(Yo).max()
    mean, var, first, total = [t.cpu().numpy() for t in q.stats(to_dev(Wo, torch.float64))]
    mo, vo, fo, to = uq.statistics(al, Wo)
    assert np.abs(mean - mo).max() <= 1e-14 * np.abs(mo).max()
    assert np.abs(var - vo).max() <= 1e-12 * np.abs(vo).max()
    assert np.abs(first - fo).max() <= 1e-12 and np.abs(total - to).max() <= 1e-12


def test_collocation_of_batched_pressure_solves():
    import torch

    import paper_1810_08572_amd as ppe

    q = ppe.PolynomialChaos(KINDS, 2)
    X, _ = q.nodes("tensor", 3)  # 27 samples, as in the paper's three-input table
    m = box_mesh((16, 16, 16), lengths=(0.01,) * 3, jitter=0.1, seed=0)
    u = concat_meshes([m] * X.shape[0])
    fls, bs = [], []
    for x in X:
        sm = dict(t_melt=950.0 + 10.0 * x[0], t_wall=600.0 + 20.0 * x[1], d_liq=5.0 * x[2])
        f = uq_front_fl(m.cell_centre, sm, 0.03, 0.05, length=0.01)
        fls.append(f)
        bs.append(rhs_smooth_series(m.cell_centre, 0.03, seed=5, center_mask=f > 0))
    s = ppe.Solver()
    s.set_mesh(u.n_cells, to_dev(u.owner, torch.int32), to_dev(u.neigh, torch.int32))
    s.set_segments(u.extra["cell_offsets"])
    s.assemble(to_dev(face_coeff(u, 2400.0), torch.float64), to_dev(np.concatenate(fls), torch.float64))
    res = s.solve(to_dev(np.concatenate(bs), torch.float64))
    its, rr = s.segment_stats()
    assert max(rr) <= 1e-10
    Y = res.p.reshape(X.shape[0], m.n_cells)
    W = q.fit(X, Y).cpu().numpy()
    al = uq.total_degree_indices(3, 2)
    Wo = uq.fit(uq.vandermonde(OK, al, X), Y.cpu().numpy())
    assert np.abs(W - Wo).max() <= 1e-12 * np.abs(Wo).max()
    mean, var, first, total = [t.cpu().numpy() for t in q.stats(to_dev(Wo, torch.float64))]
    # the front depth depends on the wall and melt temperatures: the cells
    # whose pressure varies at all are sensitive to them
    varying = var > 1e-6 * var.max()
    assert varying.sum() > 100
    f, t = first[:, varying], total[:, varying]
    assert np.all(f >= 0) and np.all(f <= t + 1e-12) and np.all(t <= 1 + 1e-12)
    assert np.all(f.sum(axis=0) <= 1 + 1e-12)
    print(f"27 samples x {m.n_cells} cells: mean PCG iterations {np.mean(its):.1f}, "
          f"cells with varying pressure {varying.sum()}", flush=True)


def test_rejects_too_few_or_repeated_points():
    import torch

    import paper_1810_08572_amd as ppe

    q = ppe.PolynomialChaos(KINDS, 2)  # 10 terms
    Y = to_dev(np.ones((8, 4)), torch.float64)
    with pytest.raises(ppe.PpeError) as e:
        q.fit(np.zeros((8, 3)), Y)
    assert e.value.status == ppe.PPE_ERR_ARG
    X = np.repeat(np.random.default_rng(0).normal(size=(4, 3)), 3, axis=0)  # 12 points, 4 distinct
    with pytest.raises(ppe.PpeError) as e:
        q.fit(X, to_dev(np.ones((12, 4)), torch.float64))
    assert e.value.status == ppe.PPE_ERR_ARG


def test_smallest_expansions():
    """Degree 0 (the mean only) from one node; one input; the smallest
    Smolyak grid; a single output column."""
    import torch

    import paper_1810_08572_amd as ppe

    q = ppe.PolynomialChaos(["normal"], 0)
    X, w = q.nodes("smolyak", 1)
    assert X.shape == (1, 1) and X[0, 0] == 0.0 and w[0] == 1.0
    Y = to_dev(np.array([[3.5, -1.0]]), torch.float64)
    W = q.fit(X, Y).cpu().numpy()
    assert np.array_equal(W, np.array([[3.5, -1.0]]))
    mean, var, first, total = [t.cpu().numpy() for t in q.stats(to_dev(W, torch.float64))]
    assert np.array_equal(mean, [3.5, -1.0]) and np.all(var == 0) and np.all(total == 0)
    q = ppe.PolynomialChaos(["uniform"], 4)
    X, _ = q.nodes("tensor", 5)
    x = X[:, 0]
    y = 1.0 + 2.0 * x - 0.5 * x ** 4  # in the span of the basis
    W = q.fit(X, to_dev(y[:, None], torch.float64))
    T = np.linspace(-1, 1, 7)[:, None]
    Ye = q.eval(T, W).cpu().numpy()[:, 0]
    assert np.abs(Ye - (1.0 + 2.0 * T[:, 0] - 0.5 * T[:, 0] ** 4)).max() <= 1e-13
