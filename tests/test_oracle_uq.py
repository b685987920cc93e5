"""Pins of the collocation oracle (section 3) against facts fixed outside
the code: the node counts the paper prints, exact moments of the normal and
uniform distributions, recovery of a known expansion, Sobol indices computed
independently as conditional variances, and the strata of the Latin-hypercube
test points (an input generator)."""
import itertools
import json
import os
from math import prod

import numpy as np

from oracle import uq

HERE = os.path.dirname(__file__)


def _moment(kind, k):
    if k % 2:
        return 0.0
    if kind == uq.NORMAL:
        return float(prod(range(k - 1, 0, -2))) if k else 1.0  # (k-1)!!
    return 1.0 / (k + 1)  # uniform on [-1, 1]


def test_node_counts_match_the_papers_tables():
    g = json.load(open(os.path.join(HERE, "golden", "collocation_counts.json")))
    for lvl, n in g["smolyak_4_inputs"].items():
        X, w = uq.smolyak_grid([uq.NORMAL] * 4, int(lvl))
        assert X.shape[0] == n, (lvl, X.shape)
    for lvl, n in g["tensor_3_inputs"].items():
        X, w = uq.tensor_grid([uq.NORMAL] * 3, int(lvl))
        assert X.shape[0] == n


def test_gauss_rules_exact_to_degree_2l_minus_1():
    for kind in (uq.NORMAL, uq.UNIFORM):
        for lvl in range(1, 8):
            x, w = uq.gauss_rule(kind, lvl)
            for k in range(2 * lvl):
                scale = w @ np.abs(x) ** k  # the sum cancels for odd k
                assert abs(w @ x ** k - _moment(kind, k)) <= 1e-14 * scale + 1e-15, (kind, lvl, k)
            # one degree more is not integrated exactly (an even power)
            k = 2 * lvl
            assert abs(w @ x ** k - _moment(kind, k)) > 1e-8


def test_sparse_grids_exact_to_total_degree_2l_minus_1():
    kinds = [uq.NORMAL, uq.UNIFORM, uq.NORMAL]
    for lvl in (2, 3, 4, 5):
        X, w = uq.smolyak_grid(kinds, lvl)
        assert abs(w.sum() - 1.0) <= 1e-13
        for a in itertools.product(range(2 * lvl), repeat=3):
            if sum(a) > 2 * lvl - 1:
                continue
            ref = prod(_moment(kinds[j], a[j]) for j in range(3))
            mono = np.prod(X ** np.array(a), axis=1)
            got = w @ mono
            assert abs(got - ref) <= 1e-13 * (np.abs(w) @ np.abs(mono)) + 1e-15, (lvl, a)


def test_basis_is_orthonormal_under_the_quadrature():
    kinds = [uq.NORMAL, uq.UNIFORM]
    p = 4
    al = uq.total_degree_indices(2, p)
    assert al.shape[0] == 15 and tuple(al[0]) == (0, 0)
    X, w = uq.tensor_grid(kinds, p + 1)  # exact to degree 2p + 1
    V = uq.vandermonde(kinds, al, X)
    scale = np.abs(V).T @ (w[:, None] * np.abs(V))
    assert np.all(np.abs(V.T @ (w[:, None] * V) - np.eye(len(al))) <= 1e-14 * scale + 1e-15)


def test_fit_recovers_a_known_expansion():
    kinds = [uq.NORMAL, uq.NORMAL, uq.UNIFORM, uq.NORMAL]
    al = uq.total_degree_indices(4, 3)
    rng = np.random.default_rng(5)
    Wt = rng.normal(size=(len(al), 3))
    X, _ = uq.smolyak_grid(kinds, 4)
    assert X.shape[0] > len(al)
    W = uq.fit(uq.vandermonde(kinds, al, X), uq.vandermonde(kinds, al, X) @ Wt)
    assert np.abs(W - Wt).max() <= 1e-11


def test_sobol_indices_equal_conditional_variances():
    # f = xi1 + 0.5 xi2^2 + 0.3 xi1 xi3 + 0.2 xi2 xi3^2 (not in the basis form)
    kinds = [uq.NORMAL, uq.NORMAL, uq.UNIFORM]

    def f(x):
        return x[..., 0] + 0.5 * x[..., 1] ** 2 + 0.3 * x[..., 0] * x[..., 2] + 0.2 * x[..., 1] * x[..., 2] ** 2

    al = uq.total_degree_indices(3, 3)
    X, w = uq.tensor_grid(kinds, 4)
    W = uq.fit(uq.vandermonde(kinds, al, X), f(X))
    mean, var, first, total = uq.statistics(al, W)
    # conditional variances by nested Gauss quadrature (exact for this f)
    rules = [uq.gauss_rule(k, 4) for k in kinds]
    grid = np.stack(np.meshgrid(*[r[0] for r in rules], indexing="ij"), axis=-1)
    wt = np.einsum("i,j,k->ijk", *[r[1] for r in rules])
    F = f(grid)
    m = (wt * F).sum()
    V = (wt * (F - m) ** 2).sum()
    assert abs(mean - m) <= 1e-12 and abs(var - V) <= 1e-12 * V
    for j in range(3):
        others = tuple(k for k in range(3) if k != j)
        wj = rules[j][1]
        # first order: Var_j(E[f | xi_j])
        cond = (wt * F).sum(axis=others) / wj
        s1 = (wj * (cond - m) ** 2).sum() / V
        # total: E_{~j}(Var_j(f | xi_~j))
        wo = wt.sum(axis=j)
        mj = (wt * F).sum(axis=j) / wo
        var_j = (wt * (F - np.expand_dims(mj, j)) ** 2).sum(axis=j) / wo
        st = (wo * var_j).sum() / V
        assert abs(first[j] - s1) <= 1e-12 and abs(total[j] - st) <= 1e-12, (j, first[j], s1, total[j], st)


def test_latin_hypercube_has_one_point_per_stratum():
    from synth import latin_hypercube

    X, U = latin_hypercube(["normal", "uniform", "normal"], 60, seed=3)
    for j in range(3):
        assert np.array_equal(np.sort(np.floor(U[:, j] * 60).astype(int)), np.arange(60))
    assert np.all(np.abs(X[:, 1]) <= 1.0)
