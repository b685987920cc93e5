"""Parity at the full workload sizes, in the configuration the benchmark
launches (one assembly and one solve per timestep, default options):

- 64^3 jittered cube, growing solid front, smooth right-hand side.  This is
  the first timestep the benchmark times.
- 128^3 jittered cube, seeded random planar front, in FP64 and in mixed
  precision.
- The 1.5 M-cell plate with ribs at a timestep of the benchmark's run.
- 256 uneven uncertainty samples (13.5 M cells) in one batched solve, with
  eight seeded samples checked against their own oracle solves.

The oracle assembles each system, builds the same smoothed-aggregation
hierarchy and runs PCG to 1e-13 as the reference.  Every GPU pressure must
reach relative residual <= 1e-10, recomputed in FP64 from the oracle's
matrix, and be within 1e-9 relative L2 of the reference, in FP64 and in
mixed precision alike (the mixed V-cycle reads FP32 copies of the
hierarchy's values but computes in FP64, so it is a fixed SPD
preconditioner and the outer iteration keeps its FP64 behaviour).
"""
import numpy as np
import pytest

from oracle import amg, assembly, pcg
from synth import box_mesh, face_coeff, fl_growing_front, fl_planar_front, rhs_smooth_series, \
    rhs_uniform
from tests.gpu_util import gpu_solver, to_dev

pytestmark = pytest.mark.gpu


def _reference(m, f, c, b):
    sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, f)
    H = amg.build_hierarchy(sy.A)
    bp = assembly.pinned_rhs(sy, b)
    loose = pcg.pcg(sy.A, bp, M=lambda r: amg.vcycle(H, r), rtol=1e-10)
    tight = pcg.pcg(sy.A, bp, M=lambda r: amg.vcycle(H, r), rtol=1e-13, max_iter=200)
    return sy, H, loose, assembly.scatter(sy, tight.x)


def _check(sy, b, pref, s, res, label, l2_bar=1e-9):
    p = res.p.cpu().numpy()
    rr = assembly.relative_residual(sy, b, p)
    err = np.linalg.norm(p - pref) / np.linalg.norm(pref)
    print(f"{label}: iterations {res.stats['iterations']}, residual {rr:.3e}, L2 error {err:.3e}",
          flush=True)
    assert res.status == 0
    assert rr <= 1e-10, (label, rr)
    assert err <= l2_bar, (label, err)
    assert np.all(p[~sy.active] == 0)


def test_c2_timestep_against_oracle():
    import torch

    m = box_mesh((64, 64, 64), lengths=(0.01,) * 3, jitter=0.1, seed=0)
    c = face_coeff(m, 2400.0)
    t = 0.101
    f = fl_growing_front(m.cell_centre, t=t, t_end=0.2, s_max=0.6, delta=0.1, axis=0, length=0.01)
    b = rhs_smooth_series(m.cell_centre, t, seed=5, center_mask=f > 0)
    sy, H, loose, pref = _reference(m, f, c, b)
    s = gpu_solver(m, f, c)
    res = s.solve(to_dev(b, torch.float64))
    _check(sy, b, pref, s, res, "64^3 fp64")
    assert abs(res.stats["iterations"] - loose.iterations) <= 1
    assert res.stats["levels"] == len(H.levels)


@pytest.fixture(scope="module")
def c3():
    m = box_mesh((128, 128, 128), jitter=0.1, seed=0)
    c = face_coeff(m, 2400.0)
    f = fl_planar_front(m.cell_centre, seed=2)
    b = rhs_uniform(m.n_cells, seed=1, center_mask=f > 0)
    sy, H, loose, pref = _reference(m, f, c, b)
    return m, f, c, b, sy, loose, pref


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c3_against_oracle(c3, precision):
    import torch

    m, f, c, b, sy, loose, pref = c3
    s = gpu_solver(m, f, c, precision=precision)
    res = s.solve(to_dev(b, torch.float64))
    _check(sy, b, pref, s, res, f"128^3 {precision}", 1e-9)
    assert abs(res.stats["iterations"] - loose.iterations) <= 1


def test_c5_plate_timestep_against_oracle():
    """The 1.5 M-cell plate with ribs at timestep 42 (front rising from the
    bottom face), FP64 with autotuned launch choices as the benchmark runs it."""
    import torch

    from synth import plate_with_ribs_mesh

    m = plate_with_ribs_mesh()
    height = float(m.cell_centre[:, 2].max() - m.cell_centre[:, 2].min()) + 2.0e-3 / 3.0
    c = face_coeff(m, 2400.0)
    t = 0.043
    f = fl_growing_front(m.cell_centre, t=t, t_end=0.2, s_max=0.6, delta=0.1, axis=2,
                         length=height)
    b = rhs_smooth_series(m.cell_centre, t, seed=5, center_mask=f > 0)
    sy, H, loose, pref = _reference(m, f, c, b)
    s = gpu_solver(m, f, c, autotune=True)
    res = s.solve(to_dev(b, torch.float64))
    _check(sy, b, pref, s, res, "plate fp64")
    assert abs(res.stats["iterations"] - loose.iterations) <= 2


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c4_batch_of_256_samples(precision):
    """256 uneven samples (sides 24..48, 13.5 M cells) in one batched solve:
    every sample's true residual (recomputed by the library in FP64) meets
    1e-10; eight seeded samples are checked against their own oracle solves."""
    import torch

    from synth import batch_samples, concat_meshes, uq_front_fl

    samples = batch_samples(256)
    meshes = [box_mesh((sm["side"],) * 3, lengths=(0.01,) * 3, jitter=0.1, seed=q)
              for q, sm in enumerate(samples)]
    u = concat_meshes(meshes)
    fls = [uq_front_fl(mm.cell_centre, sm, 0.011, 0.05, length=0.01)
           for mm, sm in zip(meshes, samples)]
    bs = [rhs_uniform(mm.n_cells, seed=1000 * q + 10, center_mask=f > 0)
          for q, (mm, f) in enumerate(zip(meshes, fls))]
    import paper_1810_08572_amd as ppe

    s = ppe.Solver(precision=precision)
    s.set_mesh(u.n_cells, to_dev(u.owner, torch.int32), to_dev(u.neigh, torch.int32))
    s.set_segments(u.extra["cell_offsets"])
    s.assemble(to_dev(face_coeff(u, 2400.0), torch.float64),
               to_dev(np.concatenate(fls), torch.float64))
    res = s.solve(to_dev(np.concatenate(bs), torch.float64))
    its, rr = s.segment_stats()
    assert res.status == 0
    assert max(rr) <= 1e-10, max(rr)
    off = u.extra["cell_offsets"]
    p_all = res.p.cpu().numpy()
    for q in sorted(np.random.default_rng(7).choice(256, 8, replace=False)):
        mm, f, b = meshes[q], fls[q], bs[q]
        sy, H, loose, pref = _reference(mm, f, face_coeff(mm, 2400.0), b)
        p = p_all[off[q]:off[q + 1]]
        rq = assembly.relative_residual(sy, b, p)
        err = np.linalg.norm(p - pref) / np.linalg.norm(pref)
        print(f"{precision} sample {q} side {samples[q]['side']}: iterations {its[q]} "
              f"(oracle {loose.iterations}), residual {rq:.2e}, L2 {err:.2e}", flush=True)
        assert rq <= 1e-10
        assert err <= 1e-9
