"""GPU parity of the smoothed-aggregation setup and of the operators the
V-cycle applies: aggregates equal the oracle's exactly; P, coarse operators,
spectral bounds, SpMV and the V-cycle agree to rounding."""
import numpy as np
import pytest

from oracle import amg, assembly
from synth import box_mesh, face_coeff, fl_planar_front
from tests.gpu_util import case, csr, gpu_solver, rel_max, to_dev

pytestmark = pytest.mark.gpu


def _cases():
    yield "c1", case()
    m = box_mesh((23, 19, 17), jitter=0.1, seed=4)
    f = fl_planar_front(m.cell_centre, seed=7)
    yield "ragged_front", (m, f, face_coeff(m, 2400.0), None)


@pytest.mark.parametrize("name,cs", list(_cases()), ids=lambda x: x if isinstance(x, str) else "")
def test_hierarchy_matches_oracle(name, cs):
    m, f, c, _ = cs
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    H = amg.build_hierarchy(sy.A)
    s = gpu_solver(m, f, c)
    assert s.n_levels() == len(H.levels)
    for lvl, lev in enumerate(H.levels):
        info = s.level_info(lvl)
        n = lev.A.shape[0]
        assert info["n"] == n
        assert abs(info["rho"] - lev.rho) <= 1e-12 * lev.rho, (lvl, info["rho"], lev.rho)
        A = csr(*s.level_matrix(lvl), (n, n))
        assert rel_max(A, lev.A) <= 1e-13, lvl
        if lvl < len(H.levels) - 1:
            agg = s.aggregates(lvl).cpu().numpy()
            assert np.array_equal(agg, lev.agg), lvl           # exact
            P = csr(*s.prolongator(lvl), lev.P.shape)
            assert rel_max(P, lev.P) <= 1e-13, lvl


def test_spmv_and_vcycle_match_oracle():
    import torch

    m, f, c, _ = case()
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    H = amg.build_hierarchy(sy.A)
    s = gpu_solver(m, f, c)
    rng = np.random.default_rng(3)
    for lvl, lev in enumerate(H.levels):
        x = rng.normal(size=lev.A.shape[0])
        y = s.apply_matrix(lvl, to_dev(x, torch.float64)).cpu().numpy()
        ref = lev.A @ x
        assert np.abs(y - ref).max() <= 1e-14 * np.abs(lev.A).max() * np.abs(x).sum() / len(x) * 50
    r = rng.normal(size=sy.n_active)
    z = s.apply_vcycle(to_dev(r, torch.float64)).cpu().numpy()
    zr = amg.vcycle(H, r)
    assert np.linalg.norm(z - zr) <= 1e-12 * np.linalg.norm(zr)


def test_setup_is_deterministic():
    m, f, c, _ = case(shape=(20, 20, 20), fl="front")
    s1 = gpu_solver(m, f, c)
    s2 = gpu_solver(m, f, c)
    for lvl in range(s1.n_levels()):
        for a, b in zip(s1.level_matrix(lvl), s2.level_matrix(lvl)):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
