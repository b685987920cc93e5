"""Warm-start network: forward and backward pass and Adam (FP64 reference).

Test infrastructure only (see the package docstring).  Not in the paper:
the network predicts the next pressure increment of each cell from local
features, and conjugate gradients always finishes the solve, so it can only
change the iteration count.

Network: L dense layers, widths n_in -> w -> ... -> w -> 1; hidden layers
use SiLU, silu(z) = z / (1 + exp(-z)); the output layer is linear.  Loss:
mean squared error.  Parameters are packed flat, layer by layer, each layer
as W (row-major, [out][in]) followed by b.
"""
from __future__ import annotations

import numpy as np


def layer_shapes(n_in=10, width=128, n_hidden=3):
    dims = [n_in] + [width] * n_hidden + [1]
    return [(dims[k + 1], dims[k]) for k in range(len(dims) - 1)]


def n_params(shapes):
    return sum(o * i + o for o, i in shapes)


def unpack(theta, shapes):
    out, k = [], 0
    for o, i in shapes:
        W = theta[k:k + o * i].reshape(o, i)
        k += o * i
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    return out


def init_params(shapes, seed=0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (PCG64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in shapes:
        lim = 1.0 / np.sqrt(i)
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(rng.uniform(-lim, lim, size=o))
    return np.concatenate(parts)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s + z * s * (1.0 - s)


def forward(theta, shapes, X):
    """X: [n, n_in].  Returns y [n] and the pre-activations of every layer."""
    h = np.asarray(X, dtype=np.float64)
    zs, hs = [], [h]
    layers = unpack(theta, shapes)
    for k, (W, b) in enumerate(layers):
        z = h @ W.T + b
        zs.append(z)
        h = silu(z) if k < len(layers) - 1 else z
        hs.append(h)
    return h[:, 0], zs, hs


def loss_and_grad(theta, shapes, X, T):
    """Mean squared error over the rows and its gradient (packed)."""
    y, zs, hs = forward(theta, shapes, X)
    n = y.shape[0]
    err = y - T
    loss = float(np.mean(err * err))
    layers = unpack(theta, shapes)
    g = (2.0 / n) * err[:, None]            # dL/dz of the output layer
    grads = [None] * len(layers)
    for k in range(len(layers) - 1, -1, -1):
        W, _ = layers[k]
        grads[k] = (g.T @ hs[k], g.sum(axis=0))
        if k > 0:
            g = (g @ W) * dsilu(zs[k - 1])
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) at step t >= 1; returns the
    new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def warm_start_features(n_cells, owner, neigh, coeff, fl, volume, dp_prev, rhs, pin_of):
    """Raw (unstandardised) features of every active cell, in compact order:
    previous increment re-referenced to the cell's pin (dp_c - dp_pin(c)) /
    its RMS, rhs / its RMS, f_l, volume / mean volume, and the six largest
    open-face coefficients divided by their sum, descending.  RMS and mean
    are over the active cells; pin_of[c] is the pin of cell c's pocket."""
    active = np.asarray(fl) > 0
    cells = np.nonzero(active)[0]
    na = cells.size
    dp_prev = np.where(active, dp_prev - dp_prev[np.where(active, pin_of, 0)], 0.0)
    rms = lambda a: np.sqrt(np.mean(np.asarray(a)[cells] ** 2))
    s_dp, s_b = rms(dp_prev), rms(rhs)
    v_mean = np.mean(np.asarray(volume)[cells])
    F = np.zeros((na, 10))
    F[:, 0] = dp_prev[cells] / s_dp if s_dp > 0 else 0.0
    F[:, 1] = rhs[cells] / s_b if s_b > 0 else 0.0
    F[:, 2] = fl[cells]
    F[:, 3] = volume[cells] / v_mean
    inner = np.nonzero(neigh >= 0)[0]
    open_ = inner[active[owner[inner]] & active[neigh[inner]]]
    lists = {c: [] for c in cells}
    for f in open_:
        lists[owner[f]].append(coeff[f])
        lists[neigh[f]].append(coeff[f])
    for r, c in enumerate(cells):
        v = sorted(lists[c], reverse=True)
        tot = sum(v)
        for q in range(min(6, len(v))):
            F[r, 4 + q] = v[q] / tot
    return F, s_dp
