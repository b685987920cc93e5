"""The library's host-side collocation set-up (Gauss rules, tensor and
Smolyak node sets, basis order) against the oracle, on the CPU: node sets
equal to 1e-14 and weights to 1e-14, the paper's node counts, the same
multi-indices in the same order."""
import json
import os

import numpy as np
import pytest

from oracle import uq

HERE = os.path.dirname(__file__)


def _pce(kinds, degree=3):
    import paper_1810_08572_amd as ppe

    return ppe.PolynomialChaos(kinds, degree)


def _same_sets(X, w, Xo, wo):
    assert X.shape == Xo.shape
    i = np.lexsort(X.T[::-1])
    j = np.lexsort(Xo.T[::-1])
    assert np.abs(X[i] - Xo[j]).max() <= 1e-14 * max(1.0, np.abs(Xo).max())
    assert np.abs(w[i] - wo[j]).max() <= 1e-14


@pytest.mark.parametrize("kinds", [["normal"] * 4, ["normal", "uniform", "normal"], ["uniform"] * 2])
def test_node_sets_match_oracle(kinds):
    okinds = [uq.NORMAL if k == "normal" else uq.UNIFORM for k in kinds]
    q = _pce(kinds)
    for lvl in (1, 2, 3, 4, 5):
        _same_sets(*q.nodes("smolyak", lvl), *uq.smolyak_grid(okinds, lvl))
        if len(kinds) <= 3:
            _same_sets(*q.nodes("tensor", lvl), *uq.tensor_grid(okinds, lvl))


def test_gauss_rules_to_high_order():
    q = _pce(["normal", "uniform"])
    for n in (7, 12, 15):
        for j, kind in enumerate((uq.NORMAL, uq.UNIFORM)):
            X, w = q.nodes("tensor", n)
            xs = np.unique(np.round(X[:, j], 12))
            xo, wo = uq.gauss_rule(kind, n)
            assert np.abs(np.sort(xs) - np.sort(np.round(xo, 12))).max() <= 1e-12


def test_paper_counts_and_basis_order():
    g = json.load(open(os.path.join(HERE, "golden", "collocation_counts.json")))
    q4 = _pce(["normal"] * 4)
    for lvl, n in g["smolyak_4_inputs"].items():
        assert q4.nodes("smolyak", int(lvl))[0].shape[0] == n
    q3 = _pce(["normal"] * 3)
    for lvl, n in g["tensor_3_inputs"].items():
        assert q3.nodes("tensor", int(lvl))[0].shape[0] == n
    q = _pce(["normal", "uniform", "normal"], degree=4)
    assert np.array_equal(q.terms, uq.total_degree_indices(3, 4))
