"""Mixed precision (the V-cycle reads FP32 copies of the hierarchy's values
and computes in FP64; FP64 outer PCG): the final pressure meets the same
FP64 bars as the FP64 path - relative residual <= 1e-10 recomputed by the
oracle and relative L2 error <= 1e-9 against an exact reference - with the
FP64 path's iteration count, and one mixed V-cycle differs from the oracle's
FP64 V-cycle only by the rounding of the stored values."""
import numpy as np
import pytest

from oracle import amg, assembly, direct
from tests.gpu_util import case, gpu_solver, to_dev

pytestmark = pytest.mark.gpu

# One V-cycle is a fixed linear map whose matrices' values are rounded to
# FP32 (unit roundoff 2^-24 = 6e-8 per value); the smoothing polynomials and
# the restriction and prolongation of 3-4 levels combine a few dozen such
# values per output, so the relative difference to the FP64 V-cycle stays
# well below 1e-6 (a CPU emulation of exactly that rounding at 24^3 gives
# 9.9e-8).
VCYCLE_FP32_RTOL = 1e-6


@pytest.mark.parametrize("shape,fl", [((16, 16, 16), "linear"), ((32, 32, 32), "front"),
                                      ((29, 17, 23), "front")])
def test_mixed_solve_meets_fp64_bars(shape, fl):
    import torch

    m, f, c, b = case(shape=shape, fl=fl)
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    pref = direct.solve_sparse(sy, b)
    s64 = gpu_solver(m, f, c)
    it64 = s64.solve(to_dev(b, torch.float64)).stats["iterations"]
    s32 = gpu_solver(m, f, c, precision="mixed")
    res = s32.solve(to_dev(b, torch.float64))
    p = res.p.cpu().numpy()
    assert res.status == 0
    assert assembly.relative_residual(sy, b, p) <= 1e-10
    assert np.linalg.norm(p - pref) <= 1e-9 * np.linalg.norm(pref)
    assert abs(res.stats["iterations"] - it64) <= 1


def test_fp32_vcycle_close_to_fp64_oracle():
    import torch

    m, f, c, _ = case(shape=(24, 24, 24), fl="front")
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    H = amg.build_hierarchy(sy.A)
    s32 = gpu_solver(m, f, c, precision="mixed")
    r = np.random.default_rng(1).normal(size=sy.n_active)
    z = s32.apply_vcycle(to_dev(r, torch.float64)).cpu().numpy()
    zr = amg.vcycle(H, r)
    rel = np.linalg.norm(z - zr) / np.linalg.norm(zr)
    assert rel <= VCYCLE_FP32_RTOL, rel
    assert rel > 1e-12   # it really read the FP32 copies
    # the oracle's V-cycle on the same FP32-rounded values, computed in FP64:
    # equal up to FP64 summation order
    zq = amg.vcycle(_rounded(H), r)
    assert np.linalg.norm(z - zq) <= 1e-12 * np.linalg.norm(zq)


def _rounded(H):
    """A copy of the oracle's hierarchy with every stored level operator,
    diagonal, P and R value rounded to FP32 (the coarsest inverse kept)."""
    import copy

    G = copy.deepcopy(H)
    q = lambda a: a.astype(np.float32).astype(np.float64)
    for lev in G.levels:
        lev.A, lev.diag = q(lev.A), q(lev.diag)
        if lev.P is not None:
            lev.P, lev.R = q(lev.P), q(lev.R)
    return G
