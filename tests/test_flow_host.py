"""Host-side parts of the time-step driver's binding: a snapshot saved and
loaded again restores every field bit for bit, the step counter and the
simulated time (CPU tensors stand in for device memory here)."""
import numpy as np
import torch

import paper_1810_08572_amd as ppe


def test_snapshot_round_trip(tmp_path):
    rng = np.random.default_rng(0)
    n, nf = 37, 101
    t = lambda *shape: torch.as_tensor(rng.normal(size=shape), dtype=torch.float64)
    st = ppe.FlowState(t(n, 3), t(n), t(n), t(nf), t(n), t(n, 3), t(n), have_history=True,
                       step=12, time=3.5e-4)
    path = tmp_path / "snap.npz"
    st.save(path)
    back = ppe.FlowState.load(path, torch.device("cpu"))
    for k in ppe.FlowState._FIELDS:
        a, b = getattr(st, k), getattr(back, k)
        assert a.shape == b.shape and torch.equal(a, b), k
    assert back.have_history and back.step == 12 and back.time == 3.5e-4
