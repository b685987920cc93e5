"""Polynomial chaos by stochastic collocation (section 3): the oracle of the
uncertainty wrapper (test infrastructure only; the product path never uses it).

* Expansion (Eq. 27): w(x, xi) ~ sum_{i=0..n} w_i(x) Psi_i(xi), with Psi_i
  products of one-dimensional polynomials orthonormal under each input's
  distribution: probabilists' Hermite He_k / sqrt(k!) for a standard normal
  input, Legendre sqrt(2k+1) P_k for a uniform input on [-1, 1] (the
  Askey-scheme choice of section 3).  The basis holds every multi-index of
  total degree <= p.
* Collocation (Eq. 28): the Vandermonde system V w = w_sim at M > n + 1
  sample points is solved in the least-squares sense.
* Sample points: tensor products of one-dimensional Gauss rules, or
  Smolyak's sparse combination of them.  Accuracy level l uses the l-point
  Gauss rule in one dimension, which integrates degree 2l - 1 exactly; the
  Smolyak grid of level l in d dimensions is
      sum_{l <= |i| <= l + d - 1} (-1)^(l + d - 1 - |i|) C(d - 1, l + d - 1 - |i|)
          (Q_{i_1} x ... x Q_{i_d}),   i_k >= 1,
  with coincident nodes merged (their weights added).
* Statistics of the expansion: mean w_0, variance sum_{i>0} w_i^2; Sobol
  indices (first order: terms in that input alone; total: every term that
  involves it) as shares of the variance.
"""
from __future__ import annotations

import itertools
from math import comb, factorial, sqrt

import numpy as np
from numpy.polynomial.hermite_e import hermegauss, hermeval
from numpy.polynomial.legendre import leggauss, legval

NORMAL, UNIFORM = "normal", "uniform"


def gauss_rule(kind, n):
    """n-point Gauss rule for the standard input: nodes, probability weights
    (summing to 1)."""
    if kind == NORMAL:
        x, w = hermegauss(n)
        return x, w / np.sqrt(2.0 * np.pi)
    if kind == UNIFORM:
        x, w = leggauss(n)
        return x, w / 2.0
    raise ValueError(kind)


def _merge(points):
    """points: key -> [coordinates of the first node with that key, weight];
    nodes in key order."""
    keys = sorted(points)
    X = np.array([points[k][0] for k in keys], dtype=np.float64).reshape(len(keys), -1)
    return X, np.array([points[k][1] for k in keys])


def _key(x):
    # nodes of different rules coincide only where they are equal up to the
    # rounding of the 1-D rule; 1e-12 identifies those and nothing else (the
    # node keeps its own coordinates)
    return tuple(float(np.round(v, 12)) + 0.0 for v in x)


def _add(points, x, w):
    k = _key(x)
    if k in points:
        points[k][1] += w
    else:
        points[k] = [[float(v) for v in x], w]


def tensor_grid(kinds, level):
    """level-point Gauss rule in every input, full tensor product."""
    rules = [gauss_rule(k, level) for k in kinds]
    pts = {}
    for combo in itertools.product(*[range(level)] * len(kinds)):
        x = [rules[j][0][c] for j, c in enumerate(combo)]
        _add(pts, x, float(np.prod([rules[j][1][c] for j, c in enumerate(combo)])))
    return _merge(pts)


def smolyak_grid(kinds, level):
    """Smolyak's combination of Gauss rules (accuracy level `level`)."""
    d = len(kinds)
    q = level + d - 1
    pts = {}
    for idx in itertools.product(range(1, level + 1), repeat=d):
        s = sum(idx)
        if s < level or s > q:
            continue
        c = (-1) ** (q - s) * comb(d - 1, q - s)
        rules = [gauss_rule(kinds[j], idx[j]) for j in range(d)]
        for combo in itertools.product(*[range(i) for i in idx]):
            x = [rules[j][0][combo[j]] for j in range(d)]
            _add(pts, x, c * float(np.prod([rules[j][1][combo[j]] for j in range(d)])))
    return _merge(pts)


def total_degree_indices(d, p):
    """Multi-indices of total degree <= p: by degree, then lexicographically
    descending in the first input (graded order)."""
    out = []
    for deg in range(p + 1):
        level = [a for a in itertools.product(range(deg + 1), repeat=d) if sum(a) == deg]
        out.extend(sorted(level, reverse=True))
    return np.array(out, dtype=np.int64).reshape(-1, d)


def orthonormal_1d(kind, k, x):
    c = np.zeros(k + 1)
    c[k] = 1.0
    if kind == NORMAL:
        return hermeval(x, c) / sqrt(factorial(k))
    if kind == UNIFORM:
        return legval(x, c) * sqrt(2 * k + 1)
    raise ValueError(kind)


def vandermonde(kinds, alphas, X):
    """V[m, i] = Psi_i(xi^m) (Eq. 28)."""
    X = np.atleast_2d(X)
    V = np.ones((X.shape[0], alphas.shape[0]))
    for i, a in enumerate(alphas):
        for j, kind in enumerate(kinds):
            if a[j]:
                V[:, i] *= orthonormal_1d(kind, int(a[j]), X[:, j])
    return V


def fit(V, Y):
    """Least-squares coefficients W (n_terms x n_out) of V W = Y."""
    W, *_ = np.linalg.lstsq(V, Y, rcond=None)
    return W


def statistics(alphas, W):
    """Mean, variance, first-order and total Sobol indices (per output)."""
    W = np.atleast_2d(W.T).T if W.ndim == 1 else W
    mean = W[0]
    var = (W[1:] ** 2).sum(axis=0)
    d = alphas.shape[1]
    first = np.zeros((d,) + mean.shape)
    total = np.zeros((d,) + mean.shape)
    for i, a in enumerate(alphas):
        if i == 0:
            continue
        nz = np.nonzero(a)[0]
        for j in nz:
            total[j] += W[i] ** 2
        if len(nz) == 1:
            first[nz[0]] += W[i] ** 2
    with np.errstate(invalid="ignore", divide="ignore"):
        first = np.where(var > 0, first / var, 0.0)
        total = np.where(var > 0, total / var, 0.0)
    return mean, var, first, total
