"""PCG iterations replayed from a captured HIP graph give bitwise the same
pressure, iteration counts and residuals as the same iterations launched
one by one.  The graph is replayed across several solves, with eager work
and synchronisations in between, and recaptured after a new assembly."""
import numpy as np
import pytest

from synth import box_mesh, face_coeff, fl_growing_front, fl_planar_front, rhs_uniform
from tests.gpu_util import case, to_dev, torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_equal_eager(precision):
    import torch

    import paper_1810_08572_amd as ppe

    torch_dev()
    m = box_mesh((28, 24, 20), jitter=0.1, seed=3)
    c = face_coeff(m, 2400.0)
    solvers = {g: ppe.Solver(precision=precision, use_graph=g) for g in (True, False)}
    for sv in solvers.values():
        sv.set_mesh(m.n_cells, to_dev(m.owner, torch.int32), to_dev(m.neigh, torch.int32))
    for step, t in enumerate([0.02, 0.09, 0.17]):
        fl = fl_growing_front(m.cell_centre, t, 0.2)
        for sv in solvers.values():
            sv.assemble(to_dev(c, torch.float64), to_dev(fl, torch.float64))
        for rep in range(3):
            b = rhs_uniform(m.n_cells, seed=10 * step + rep, center_mask=fl > 0)
            out = {}
            for g, sv in solvers.items():
                r = sv.solve(to_dev(b, torch.float64))
                torch.cuda.synchronize()
                _ = (r.p * 2.0).sum().item()   # eager torch work between replays
                out[g] = (r.p.cpu().numpy(), r.stats["iterations"], r.stats["rel_residual"])
            assert np.array_equal(out[True][0], out[False][0]), (step, rep)
            assert out[True][1] == out[False][1]
            assert out[True][2] == out[False][2]
            assert out[True][2] <= 1e-10
