"""Pins of the oracle's warm-start network: SiLU values, a forward pass
small enough to do by hand, gradients against central finite differences,
and Adam against its closed form on a quadratic."""
import numpy as np
import pytest

from oracle import mlp


def test_silu_values():
    assert mlp.silu(np.array([0.0]))[0] == 0.0
    assert mlp.dsilu(np.array([0.0]))[0] == 0.5
    z = np.array([2.0])
    s = 1 / (1 + np.exp(-2.0))
    assert np.isclose(mlp.silu(z)[0], 2.0 * s, rtol=1e-15)


def test_forward_by_hand():
    # 2 -> 1 -> 1: y = w2 * silu(w1 . x + b1) + b2
    shapes = mlp.layer_shapes(n_in=2, width=1, n_hidden=1)
    theta = np.array([0.5, -1.0, 0.25, 3.0, -2.0])
    x = np.array([[2.0, 1.0]])
    z = 0.5 * 2.0 - 1.0 * 1.0 + 0.25
    y_ref = 3.0 * z / (1 + np.exp(-z)) - 2.0
    y, _, _ = mlp.forward(theta, shapes, x)
    assert np.isclose(y[0], y_ref, rtol=1e-15)
    assert mlp.n_params(mlp.layer_shapes()) == 34561


@pytest.mark.parametrize("width,hidden", [(7, 2), (16, 3)])
def test_gradient_against_finite_differences(width, hidden):
    shapes = mlp.layer_shapes(n_in=10, width=width, n_hidden=hidden)
    theta = mlp.init_params(shapes, seed=1)
    rng = np.random.default_rng(2)
    X = rng.normal(size=(13, 10))
    T = rng.normal(size=13)
    _, g = mlp.loss_and_grad(theta, shapes, X, T)
    h = 1e-6
    for k in rng.choice(theta.size, 40, replace=False):
        e = np.zeros_like(theta)
        e[k] = h
        lp, _ = mlp.loss_and_grad(theta + e, shapes, X, T)
        lm, _ = mlp.loss_and_grad(theta - e, shapes, X, T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd)), (k, fd, g[k])


def test_adam_closed_form_and_descent():
    # first step of Adam moves every coordinate by lr * sign(g) (bias-corrected)
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = mlp.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(t1, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # training reduces the loss on a smooth regression
    shapes = mlp.layer_shapes(n_in=10, width=16, n_hidden=2)
    th = mlp.init_params(shapes, seed=0)
    rng = np.random.default_rng(0)
    X = rng.normal(size=(256, 10))
    T = np.tanh(X[:, 0]) - 0.5 * X[:, 1]
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0, _ = mlp.loss_and_grad(th, shapes, X, T)
    for t in range(1, 301):
        _, gr = mlp.loss_and_grad(th, shapes, X, T)
        th, m, v = mlp.adam_step(th, gr, m, v, t, lr=3e-3)
    l1, _ = mlp.loss_and_grad(th, shapes, X, T)
    assert l1 < 0.1 * l0


def test_warm_start_features_by_hand():
    """Eight cells, one removed (4), two pockets {0,1,2,3,5} (pin 0) and
    {6,7} (pin 6).  Every feature below is worked out by hand from the
    definitions: the previous increment re-referenced to the cell's own
    pocket pin over its RMS, the RHS over its RMS, f_l, the volume over the
    mean volume (RMS and mean over the seven active cells), and the open-face
    coefficients of the cell, largest first, over their sum.  Cell 1's open
    faces come in the face list with coefficients 1, 3, 2 and cell 3's with
    2, 7, so a missing sort or an ascending one shows; the blocked face
    (1, 4) and the wall face must not count."""
    owner = np.array([1, 1, 3, 1, 5, 3, 7])
    neigh = np.array([0, 2, 1, 4, -1, 5, 6])
    coeff = np.array([1.0, 3.0, 2.0, 5.0, 8.0, 7.0, 4.0])
    fl = np.array([1.0, 0.5, 1.0, 0.75, 0.0, 1.0, 1.0, 1.0])
    vol = np.array([1.0, 1.0, 2.0, 2.0, 9.0, 3.0, 4.0, 1.0])
    dp = np.array([2.0, 5.0, -1.0, 4.0, 99.0, 3.0, 10.0, 13.0])
    rhs = np.array([1.0, 2.0, -2.0, 0.0, 50.0, -1.0, 3.0, -3.0])
    pin_of = np.array([0, 0, 0, 0, -1, 0, 6, 6])
    F, s_dp = mlp.warm_start_features(8, owner, neigh, coeff, fl, vol, dp, rhs, pin_of)
    # re-referenced increments 0, 3, -3, 2, 1 | 0, 3: sum of squares 32 over 7 cells
    s = np.sqrt(32.0 / 7.0)
    assert s_dp == pytest.approx(s, rel=1e-15)
    expect = np.zeros((7, 10))
    expect[:, 0] = np.array([0.0, 3.0, -3.0, 2.0, 1.0, 0.0, 3.0]) / s
    # RHS over the active cells: 1, 2, -2, 0, -1, 3, -3 -> RMS sqrt(28 / 7) = 2
    expect[:, 1] = [0.5, 1.0, -1.0, 0.0, -0.5, 1.5, -1.5]
    expect[:, 2] = [1.0, 0.5, 1.0, 0.75, 1.0, 1.0, 1.0]
    # mean active volume 14 / 7 = 2
    expect[:, 3] = [0.5, 0.5, 1.0, 1.0, 1.5, 2.0, 0.5]
    expect[0, 4] = 1.0                              # cell 0: face to 1 only
    expect[1, 4:7] = [3.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0]  # cell 1: 3, 2, 1
    expect[2, 4] = 1.0                              # cell 2: face to 1
    expect[3, 4:6] = [7.0 / 9.0, 2.0 / 9.0]         # cell 3: 7, 2
    expect[4, 4] = 1.0                              # cell 5: face to 3 (wall ignored)
    expect[5, 4] = 1.0                              # cell 6: face to 7
    expect[6, 4] = 1.0                              # cell 7: face to 6
    assert np.allclose(F, expect, rtol=1e-15, atol=1e-15), F - expect
