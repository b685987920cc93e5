"""ppe_warm_start_features_noalloc, the variant for callers that cannot
allocate, against ppe_warm_start_features on the same solver: bitwise equal
features and scale, on two calls in a row whose second has fewer active
cells (the static workspace keeps the first call's contents), and once more
on the first solver after that."""
import numpy as np
import pytest

from synth import box_mesh, face_coeff, fl_growing_front, rhs_smooth_series
from tests.gpu_util import to_dev, torch_dev

pytestmark = pytest.mark.gpu


def _solver_and_inputs(shape, t, seed):
    import torch

    import paper_1810_08572_amd as ppe

    m = box_mesh(shape, jitter=0.1, seed=seed)
    c = face_coeff(m, 2400.0)
    fl = fl_growing_front(m.cell_centre, t, 0.2, s_max=0.5)
    b = rhs_smooth_series(m.cell_centre, t, seed=seed, center_mask=fl > 0)
    dp = np.random.default_rng(seed).normal(size=m.n_cells)
    s = ppe.Solver()
    s.set_mesh(m.n_cells, to_dev(m.owner, torch.int32), to_dev(m.neigh, torch.int32))
    args = [to_dev(a, torch.float64) for a in (dp, b, c, fl, m.cell_volume)]
    s.assemble(args[2], args[3])
    return s, args


def test_noalloc_features_equal_the_allocating_call():
    import torch

    import paper_1810_08572_amd as ppe

    dev = torch_dev()
    mu = torch.linspace(-0.5, 0.5, 10, dtype=torch.float32, device=dev)
    sigma = torch.linspace(0.5, 2.0, 10, dtype=torch.float32, device=dev)
    big, big_args = _solver_and_inputs((30, 26, 22), 0.05, 3)
    small, small_args = _solver_and_inputs((11, 9, 8), 0.12, 4)
    ref = {}
    for name, s, args in (("big", big, big_args), ("small", small, small_args)):
        F, scale = ppe.warm_start_features(s, *args, mu, sigma)
        ref[name] = (F.clone(), scale)
    n_big, n_small = ref["big"][0].shape[0], ref["small"][0].shape[0]
    print(f"active cells: {n_big}, then {n_small}", flush=True)
    assert n_small < n_big
    outs = {k: torch.full((n_big, 10), float("nan"), dtype=torch.float32, device=dev)
            for k in ("big", "small", "big_again")}
    # two calls in a row, the second smaller, then the first one again
    scales = {
        "big": ppe.warm_start_features_noalloc(big, *big_args, mu, sigma, outs["big"]),
        "small": ppe.warm_start_features_noalloc(small, *small_args, mu, sigma, outs["small"]),
        "big_again": ppe.warm_start_features_noalloc(big, *big_args, mu, sigma,
                                                     outs["big_again"]),
    }
    for k, out in outs.items():
        F, scale = ref["small" if k == "small" else "big"]
        assert scales[k] == scale, k
        assert torch.equal(out[:F.shape[0]], F), k
        # rows past the solver's active cells are not written
        assert bool(torch.isnan(out[F.shape[0]:]).all()), k
