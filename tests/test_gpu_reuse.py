"""Coarse levels kept across a changed mask (option coarse_reuse).

After a full setup, a later pressure assembly whose active set moved by at
most 10% of that build's cells keeps its coarse levels: the finest level is
the new masked operator, and its prolongator holds the earlier finest
prolongator's rows of the same cells (empty for pins).  Checked against
oracle.amg.reuse_coarse_levels applied to the oracle's own hierarchy of the
earlier system:
- the re-indexed prolongator equals the oracle's (values copied, so
  bitwise), and one V-cycle agrees to 1e-12;
- the solve meets the FP64 bars (1e-10 residual recomputed by the oracle,
  1e-9 relative L2 against sparse LU) in both precisions, within a few
  iterations of a fresh setup;
- a move of more than 10% and a spent budget of reuses both rebuild."""
import numpy as np
import pytest

from oracle import amg, assembly, direct
from synth import box_mesh, face_coeff, rhs_uniform
from tests.gpu_util import gpu_solver, to_dev

pytestmark = pytest.mark.gpu

M = box_mesh((24, 22, 20), jitter=0.1, seed=8)
C = face_coeff(M, 2400.0)
B = rhs_uniform(M.n_cells, seed=3)


def _fl(s):
    return np.clip((M.cell_centre[:, 0] - s) / 0.1, 0.0, 1.0)


def _assemble(s, front):
    import torch

    s.assemble(to_dev(C, torch.float64), to_dev(_fl(front), torch.float64))
    return s.stats()


def _oracle_reuse(base_front, front):
    sy0 = assembly.masked_system(M.n_cells, M.owner, M.neigh, C, _fl(base_front))
    sy = assembly.masked_system(M.n_cells, M.owner, M.neigh, C, _fl(front))
    H0 = amg.build_hierarchy(sy0.A)
    base_of_cell = np.full(M.n_cells, -1)
    base_of_cell[sy0.perm] = np.arange(sy0.n_active)
    pinned = np.zeros(sy.n_active, dtype=bool)
    pinned[sy.pinned] = True
    return sy, amg.reuse_coarse_levels(H0, sy.A, base_of_cell[sy.perm], pinned)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reused_coarse_levels_match_the_oracle_and_meet_the_bars(precision):
    import torch

    s = gpu_solver(M, _fl(0.18), C, precision=precision, coarse_reuse=4)
    assert s.stats()["coarse_reused"] == 0
    for front in (0.22, 0.23):   # 5% of the cells moved, then 9.2% with dangling cells
        st = _assemble(s, front)
        assert st["coarse_reused"] >= 1, front   # the same coarse levels as the 0.18 build
        sy, G = _oracle_reuse(0.18, front)
        assert s.n_levels() == len(G.levels)
        rp, ci, v = s.prolongator(0)
        P = G.levels[0].P
        assert np.array_equal(rp.cpu().numpy(), P.indptr)
        assert np.array_equal(ci.cpu().numpy()[:P.nnz], P.indices)
        if precision == "fp64":
            assert np.array_equal(v.cpu().numpy()[:P.nnz], P.data)
            r = np.random.default_rng(2).normal(size=sy.n_active)
            z = s.apply_vcycle(to_dev(r, torch.float64)).cpu().numpy()
            zr = amg.vcycle(G, r)
            assert np.linalg.norm(z - zr) <= 1e-12 * np.linalg.norm(zr)
        res = s.solve(to_dev(B, torch.float64))
        p = res.p.cpu().numpy()
        pref = direct.solve_sparse(sy, B)
        fresh = gpu_solver(M, _fl(front), C, precision=precision)
        it_fresh = fresh.solve(to_dev(B, torch.float64)).stats["iterations"]
        rr = assembly.relative_residual(sy, B, p)
        err = np.linalg.norm(p - pref) / np.linalg.norm(pref)
        print(f"{precision} front {front}: {sy.n_active} active, reused {res.stats['iterations']} "
              f"iterations (fresh {it_fresh}), residual {rr:.2e}, L2 {err:.2e}", flush=True)
        assert res.status == 0 and rr <= 1e-10 and err <= 1e-9
        assert res.stats["iterations"] <= it_fresh + 3
        assert np.all(p[~sy.active] == 0)


def test_a_large_move_or_a_spent_budget_rebuilds():
    s = gpu_solver(M, _fl(0.18), C, coarse_reuse=1)
    assert _assemble(s, 0.22)["coarse_reused"] == 1
    # budget of one reuse spent: the next changed mask gets a full setup
    assert _assemble(s, 0.23)["coarse_reused"] == 1
    # that full setup is the new base; a move of a third of its cells rebuilds
    assert _assemble(s, 0.50)["coarse_reused"] == 1
    # and 8.3% of the 0.50 build's cells is reused again
    assert _assemble(s, 0.53)["coarse_reused"] == 2
    import torch

    res = s.solve(to_dev(B, torch.float64))
    sy = assembly.masked_system(M.n_cells, M.owner, M.neigh, C, _fl(0.53))
    assert assembly.relative_residual(sy, B, res.p.cpu().numpy()) <= 1e-10
