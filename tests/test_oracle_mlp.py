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
