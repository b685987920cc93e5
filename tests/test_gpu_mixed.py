"""Mixed precision (FP32 hierarchy and smoother, FP64 outer PCG with the
flexible beta): the final pressure meets the same FP64 bars as the FP64
path - relative residual <= 1e-10 recomputed by the oracle and relative L2
error <= 1e-9 against an exact reference - and one FP32 V-cycle differs from
the oracle's FP64 V-cycle only by FP32 rounding."""
import numpy as np
import pytest

from oracle import amg, assembly, direct
from tests.gpu_util import case, gpu_solver, to_dev

pytestmark = pytest.mark.gpu

# One V-cycle is a fixed linear map built from about 10 kernels per level,
# each rounding to FP32 (unit roundoff 2^-24 = 6e-8) once per entry; with
# 3-4 levels and the Chebyshev recurrences amplifying by at most a few, the
# relative difference to the FP64 V-cycle stays below ~1e-5.
VCYCLE_FP32_RTOL = 2e-5


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
    assert res.stats["iterations"] <= it64 + 3


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
    assert rel > 1e-12   # it really ran in FP32
