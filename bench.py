"""Benchmark: masked pressure-correction Poisson solves per second on one GPU.

Workload: 64^3 = 262,144-cell jittered (+-10 %) hex cube stored as an
unstructured face list, a 10 mm cavity, aluminium density rho = 2400.
- Solid front: grows from the cold wall x = 0 as sqrt(t) over a 200-step
  schedule of 1e-3 s (mushy band 10 % of the cube).
- RHS: varies smoothly from step to step, standing in for the velocity
  divergence of a flow solve; it is centred over the liquid cells.
- Each timestep does one masked SA-AMG-PCG solve to 1e-10 relative
  residual.

One bench step = one timestep's whole hot path: masked assembly, AMG setup,
then PCG.  K consecutive timesteps are timed from the middle of the
schedule, after W warmup steps, and all inputs are resident in device
memory first.

Reported:
- value: FP64 AMG-PCG from a zero guess (the plain method).
- variants.mixed: FP32 hierarchy under the FP64 outer PCG.
- variants.mixed_learned: mixed precision, with the initial guess predicted
  by the warm-start network from the previous step.  The network is trained
  beforehand, untimed, on snapshots the solver produced for earlier
  timesteps of the same run.
- roofline: the dominant kernel's achieved HBM bandwidth.
- cpu_baseline: the FP64 oracle on host cores.
- variants.uq_batched: optional (--uq), 256 uneven uncertainty samples
  solved as one batch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_TIMESTEPS = 200
DT = 1e-3
SIDE = 64
RHO = 2400.0
CAVITY = 0.01  # m
FIRST_TIMED = 100
TRAIN_STEPS = range(20, 80)
RHS_SEED = 5


def note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def step_inputs(m, k):
    from synth import fl_growing_front, rhs_smooth_series

    t = (k + 1) * DT
    fl = fl_growing_front(m.cell_centre, t=t, t_end=N_TIMESTEPS * DT, s_max=0.6, delta=0.1,
                          axis=0, length=CAVITY)
    b = rhs_smooth_series(m.cell_centre, t, seed=RHS_SEED, center_mask=fl > 0)
    return fl, b


def cpu_baseline(m, c, inputs, steps, budget_s=20.0):
    """The FP64 oracle (assembly + SA setup + PCG from zero, unmodified) on
    host cores, single-threaded, over as many timed steps as fit the budget."""
    from threadpoolctl import threadpool_limits

    from oracle import amg, assembly, pcg

    done, iters, t0 = 0, 0, time.perf_counter()
    with threadpool_limits(limits=1):
        for k in steps:
            fl, b = inputs[k]
            sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, fl)
            H = amg.build_hierarchy(sy.A)
            res = pcg.pcg(sy.A, assembly.pinned_rhs(sy, b), M=lambda r: amg.vcycle(H, r),
                          rtol=1e-10)
            iters += res.iterations
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="solves/s", cores=1, kind="oracle",
                sample=f"{done} consecutive timed timesteps from step {steps[0]} of the 64^3 run: "
                       f"assembly + SA setup + PCG to 1e-10 from zero ({iters} PCG iterations), "
                       f"{dt:.1f} s on one host thread")


def run_leg(ppe, torch, m, dev, d_in, steps, warm, precision, learned=None):
    """Solve warm + steps timesteps; time the last len(steps).  learned =
    (net, mu, sigma) uses the warm-start network from the previous step."""
    s = ppe.Solver(precision=precision)
    s.set_mesh(m.n_cells, d_in["owner"], d_in["neigh"])
    p_prev = torch.zeros(m.n_cells, dtype=torch.float64, device=dev)
    dp_prev = torch.zeros_like(p_prev)
    out = torch.zeros_like(p_prev)
    rec = dict(iters=0, setup_ms=0.0, solve_ms=0.0, worst=0.0, n_act=[])

    def one(k, timed):
        nonlocal p_prev, dp_prev, out
        fl, b = d_in["fl"][k], d_in["b"][k]
        s.assemble(d_in["coeff"], fl)
        x0 = None
        if learned is not None:
            net, mu, sigma = learned
            F, scale = ppe.warm_start_features(s, dp_prev, b, d_in["coeff"], fl, d_in["vol"], mu,
                                               sigma)
            y = net.forward(F, bf16=True)
            x0 = ppe.warm_start_apply(s, p_prev, y, scale)
        r = s.solve(b, x0=x0, out=out)
        if learned is not None:
            dp_prev = out - p_prev
            p_prev, out = out, p_prev
        if timed:
            st = r.stats
            rec["iters"] += st["iterations"]
            rec["setup_ms"] += st["setup_ms"]
            rec["solve_ms"] += st["solve_ms"]
            rec["worst"] = max(rec["worst"], st["rel_residual"])
            rec["n_act"].append(st["n_active"])

    for k in warm:
        one(k, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in steps:
        one(k, True)
    torch.cuda.synchronize()
    rec["elapsed"] = time.perf_counter() - t0
    rec["solver"] = s
    return rec


def train_network(ppe, torch, m, dev, d_in, n_adam=400, batch=8192):
    """Snapshots produced by the solver on earlier timesteps -> trained
    network and feature standardisation (untimed)."""
    import numpy as np

    from synth import mlp_initial_weights

    s = ppe.Solver(precision="mixed")
    s.set_mesh(m.n_cells, d_in["owner"], d_in["neigh"])
    zero10 = torch.zeros(10, dtype=torch.float32, device=dev)
    one10 = torch.ones(10, dtype=torch.float32, device=dev)
    p_prev = torch.zeros(m.n_cells, dtype=torch.float64, device=dev)
    dp_prev = torch.zeros_like(p_prev)
    feats, targs, masks = [], [], []
    for k in TRAIN_STEPS:
        fl, b = d_in["fl"][k], d_in["b"][k]
        masks.append(fl > 0)
        s.assemble(d_in["coeff"], fl)
        stable = len(masks) >= 3 and bool(torch.equal(masks[-1], masks[-2])) and \
            bool(torch.equal(masks[-2], masks[-3]))
        if stable:
            F, scale = ppe.warm_start_features(s, dp_prev, b, d_in["coeff"], fl, d_in["vol"],
                                               zero10, one10)
        p = s.solve(b).p.clone()
        if stable:
            feats.append(F.clone())
            targs.append(ppe.warm_start_targets(s, p, p_prev, scale).clone())
        dp_prev = p - p_prev
        p_prev = p
    X = torch.cat(feats)
    T = torch.cat(targs)
    mu, sigma = X.mean(0).contiguous(), X.std(0).clamp_min(1e-6).contiguous()
    Xs = ((X - mu) / sigma).contiguous()
    net = ppe.WarmStartNet()
    net.set_params(torch.as_tensor(mlp_initial_weights(seed=0).astype(np.float32), device=dev))
    g = torch.Generator(device=dev).manual_seed(0)
    losses = []
    for _ in range(n_adam):
        idx = torch.randint(0, Xs.shape[0], (batch,), device=dev, generator=g)
        losses.append(net.train_step(Xs[idx].contiguous(), T[idx].contiguous(), 1e-3))
    return net, mu, sigma, dict(snapshots=len(feats), rows=int(X.shape[0]),
                                loss_first=float(np.mean(losses[:10])),
                                loss_last=float(np.mean(losses[-10:])))


def uq_batched(ppe, torch, dev, n_samples=256, steps=3, warm=1):
    """Batched uncertainty samples (sides U{24..48}, 50-step schedule):
    per step, one assembly and one segmented solve of all samples."""
    import numpy as np

    from synth import batch_samples, box_mesh, concat_meshes, face_coeff, rhs_uniform, uq_front_fl

    samples = batch_samples(n_samples)
    meshes = [box_mesh((sm["side"],) * 3, lengths=(CAVITY,) * 3, jitter=0.1, seed=q)
              for q, sm in enumerate(samples)]
    u = concat_meshes(meshes)
    off = u.extra["cell_offsets"]
    c = torch.as_tensor(face_coeff(u, RHO), device=dev)
    s = ppe.Solver(precision="mixed")
    s.set_mesh(u.n_cells, torch.as_tensor(u.owner, device=dev), torch.as_tensor(u.neigh, device=dev))
    s.set_segments(off)
    ks = list(range(10, 10 + warm + steps))
    data = {}
    for k in ks:
        fls = [uq_front_fl(mm.cell_centre, sm, (k + 1) * DT, 50 * DT, length=CAVITY)
               for mm, sm in zip(meshes, samples)]
        bs = [rhs_uniform(mm.n_cells, seed=1000 * q + k, center_mask=f > 0)
              for q, (mm, f) in enumerate(zip(meshes, fls))]
        data[k] = (torch.as_tensor(np.concatenate(fls), device=dev),
                   torch.as_tensor(np.concatenate(bs), device=dev))
    out = torch.zeros(u.n_cells, dtype=torch.float64, device=dev)
    its, worst = [], 0.0
    for i, k in enumerate(ks):
        if i == warm:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        s.assemble(c, data[k][0])
        r = s.solve(data[k][1], out=out)
        if i >= warm:
            it, rr = s.segment_stats()
            its.append(float(np.mean(it)))
            worst = max(worst, max(rr))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(value=n_samples * steps / dt, unit="sample-solves/s", samples=n_samples,
                cells=u.n_cells, steps=steps, ms_per_step=1e3 * dt / steps,
                mean_sample_iterations=float(np.mean(its)), worst_rel_residual=worst,
                precision="mixed")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="time the FP64 leg only")
    ap.add_argument("--uq", action="store_true", help="add the batched-UQ measurement")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding design); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1810_08572_amd as ppe
    from synth import box_mesh, face_coeff

    dev = torch.device("cuda", 0)
    K, W = args.steps, args.warmup
    steps = list(range(FIRST_TIMED, FIRST_TIMED + K))
    warm = list(range(FIRST_TIMED - W, FIRST_TIMED))
    m = box_mesh((SIDE,) * 3, lengths=(CAVITY,) * 3, jitter=0.1, seed=0)
    c = face_coeff(m, RHO)
    need = sorted(set(warm + steps + ([] if args.no_variants else list(TRAIN_STEPS))))
    inputs = {k: step_inputs(m, k) for k in need}
    d_in = dict(owner=torch.as_tensor(m.owner, device=dev), neigh=torch.as_tensor(m.neigh, device=dev),
                coeff=torch.as_tensor(c, device=dev), vol=torch.as_tensor(m.cell_volume, device=dev),
                fl={k: torch.as_tensor(v[0], device=dev) for k, v in inputs.items()},
                b={k: torch.as_tensor(v[1], device=dev) for k, v in inputs.items()})

    note(f"inputs ready: {len(need)} timesteps of {m.n_cells} cells")
    base = run_leg(ppe, torch, m, dev, d_in, steps, warm, "fp64")
    note(f"fp64 leg: {K / base['elapsed']:.1f} solves/s")
    assert base["worst"] <= 1e-10, f"a timed solve missed the tolerance: {base['worst']}"
    n_act = base["n_act"]
    out = {
        "metric": "pressure solves/s at 1e-10 rel. residual",
        "value": K / base["elapsed"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * base["elapsed"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "64^3 jittered hex cube, sqrt(t) solid front, smooth-in-time RHS, "
                        f"timesteps {steps[0]}..{steps[-1]} of 200 x 1e-3 s; one masked SA-AMG-PCG "
                        "pressure solve per step (assembly + setup + solve), FP64, zero guess",
            "cells": m.n_cells,
            "mean_active_cells": float(np.mean(n_act)),
            "pcg_iterations_per_solve": base["iters"] / K,
            "dof_iterations_per_s": float(np.sum(n_act)) * (base["iters"] / K) / base["elapsed"],
            "worst_rel_residual": base["worst"],
            "setup_ms_per_step": base["setup_ms"] / K,
            "solve_ms_per_step": base["solve_ms"] / K,
        },
    }

    if not args.no_profile:
        s = base["solver"]
        s.profile(True)
        for k in steps:
            s.assemble(d_in["coeff"], d_in["fl"][k])
            s.solve(d_in["b"][k])
        prof = s.profile_read()
        s.profile(False)
        avg_ms = prof["kernel_ms"] / max(prof["launches"], 1)
        per_launch = prof["bytes"] / max(prof["launches"], 1)
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        out["roofline"] = {
            "bound": "hbm",
            "kernel": "finest-level fused Chebyshev step (ELL SpMV + smoother update), FP64",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_us": avg_ms * 1e3,
            "bytes_per_launch": per_launch,
            "launches": prof["launches"],
        }

    if not args.no_variants:
        variants = {}
        mixed = run_leg(ppe, torch, m, dev, d_in, steps, warm, "mixed")
        variants["mixed"] = dict(value=K / mixed["elapsed"], unit="solves/s",
                                 pcg_iterations_per_solve=mixed["iters"] / K,
                                 setup_ms_per_step=mixed["setup_ms"] / K,
                                 solve_ms_per_step=mixed["solve_ms"] / K,
                                 worst_rel_residual=mixed["worst"])
        note(f"mixed leg: {K / mixed['elapsed']:.1f} solves/s")
        net, mu, sigma, tr = train_network(ppe, torch, m, dev, d_in)
        note(f"network trained: {tr}")
        ml = run_leg(ppe, torch, m, dev, d_in, steps, warm, "mixed", learned=(net, mu, sigma))
        assert ml["worst"] <= 1e-10
        variants["mixed_learned"] = dict(
            value=K / ml["elapsed"], unit="solves/s",
            pcg_iterations_per_solve=ml["iters"] / K,
            setup_ms_per_step=ml["setup_ms"] / K, solve_ms_per_step=ml["solve_ms"] / K,
            worst_rel_residual=ml["worst"],
            solve_time_ratio_vs_fp64=base["solve_ms"] / max(ml["solve_ms"], 1e-12),
            training=tr)
        note(f"mixed+learned leg: {K / ml['elapsed']:.1f} solves/s")
        out["variants"] = variants
    if args.uq:
        out.setdefault("variants", {})["uq_batched"] = uq_batched(ppe, torch, dev)
    if not args.no_cpu_baseline:
        note("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(m, c, inputs, steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
