"""Benchmark: masked pressure-correction Poisson solves per second on one GPU.

Workload (default): 64^3 = 262,144-cell jittered (+-10 %) hex cube stored as
an unstructured face list, aluminium density rho = 2400, a solid layer
growing from the cold wall x = 0 as sqrt(t) over 200 timesteps of 1e-3 s
(mushy band 10 % of the cube), right-hand side U(-1, 1) centred over the
liquid cells, one masked SA-AMG-PCG solve to 1e-10 relative residual per
timestep.  One bench step = one timestep's whole hot path: masked assembly,
AMG setup, PCG solve.  Timed steps are spread evenly over the 200-step
schedule; all inputs are resident in device memory before timing starts.

Prints one JSON line (see the keys below); also reports the dominant
kernel's achieved bandwidth against the HBM roofline and the FP64 oracle
timed on host cores.
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


def schedule(K, W):
    """Timestep indices for W warmup and K timed steps."""
    timed = [int(round(j * (N_TIMESTEPS - 1) / max(K - 1, 1))) for j in range(K)]
    warm = [(k * 37 + 5) % N_TIMESTEPS for k in range(W)]
    return warm, timed


def make_inputs(steps, side=SIDE):
    import numpy as np

    from synth import box_mesh, face_coeff, fl_growing_front, rhs_uniform

    m = box_mesh((side, side, side), lengths=(CAVITY,) * 3, jitter=0.1, seed=0)
    c = face_coeff(m, RHO)
    t_end = N_TIMESTEPS * DT
    fls, bs = {}, {}
    for k in steps:
        fl = fl_growing_front(m.cell_centre, t=(k + 1) * DT, t_end=t_end, s_max=0.6,
                              delta=0.1, axis=0, length=CAVITY)
        fls[k] = fl
        bs[k] = rhs_uniform(m.n_cells, seed=1000 + k, center_mask=fl > 0)
    return m, c, fls, bs


def cpu_baseline(m, c, fls, bs, steps, budget_s=20.0):
    """The FP64 oracle (assembly + SA setup + PCG, unmodified) on host cores,
    single-threaded, over as many of the timed steps as fit the budget."""
    from threadpoolctl import threadpool_limits

    from oracle import amg, assembly, pcg

    done, t0 = 0, time.perf_counter()
    iters = []
    with threadpool_limits(limits=1):
        for k in steps:
            sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, c, fls[k])
            H = amg.build_hierarchy(sy.A)
            res = pcg.pcg(sy.A, assembly.pinned_rhs(sy, bs[k]), M=lambda r: amg.vcycle(H, r),
                          rtol=1e-10)
            iters.append(res.iterations)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="solves/s", cores=1, kind="oracle",
                sample=f"{done} of the timed timesteps (64^3, steps {steps[:done]}), "
                       f"assembly + SA setup + PCG to 1e-10, {sum(iters)} PCG iterations, "
                       f"{dt:.1f} s single-threaded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding design); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1810_08572_amd as ppe

    dev = torch.device("cuda", 0)
    warm, timed = schedule(args.steps, args.warmup)
    m, c, fls, bs = make_inputs(sorted(set(warm + timed)))
    owner = torch.as_tensor(m.owner, device=dev)
    neigh = torch.as_tensor(m.neigh, device=dev)
    coeff = torch.as_tensor(c, device=dev)
    fl_d = {k: torch.as_tensor(v, device=dev) for k, v in fls.items()}
    b_d = {k: torch.as_tensor(v, device=dev) for k, v in bs.items()}
    p = torch.zeros(m.n_cells, dtype=torch.float64, device=dev)

    s = ppe.Solver(precision=args.precision)
    s.set_mesh(m.n_cells, owner, neigh)

    def step(k):
        s.assemble(coeff, fl_d[k])
        r = s.solve(b_d[k], out=p)
        return r.stats

    for k in warm:
        step(k)
    torch.cuda.synchronize()
    iters, worst, n_act, setup_ms, solve_ms = 0, 0.0, [], 0.0, 0.0
    t0 = time.perf_counter()
    for k in timed:
        st = step(k)
        setup_ms += st["setup_ms"]
        solve_ms += st["solve_ms"]
        iters += st["iterations"]
        worst = max(worst, st["rel_residual"])
        n_act.append(st["n_active"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert worst <= 1e-10, f"a timed solve missed the tolerance: {worst}"

    K = args.steps
    out = {
        "metric": "pressure solves/s at 1e-10 rel. residual",
        "value": K / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "64^3 jittered hex cube, sqrt(t) solid front over 200 x 1e-3 s steps, "
                        "one masked SA-AMG-PCG pressure solve per step (assembly + setup + solve)",
            "cells": m.n_cells,
            "mean_active_cells": float(np.mean(n_act)),
            "precision": args.precision,
            "pcg_iterations_per_solve": iters / K,
            "dof_iterations_per_s": float(np.sum(n_act)) * (iters / K) / elapsed,
            "worst_rel_residual": worst,
            "setup_ms_per_step": setup_ms / K,
            "solve_ms_per_step": solve_ms / K,
        },
    }

    if not args.no_profile:
        s.profile(True)
        for k in timed:
            step(k)
        prof = s.profile_read()
        s.profile(False)
        avg_ms = prof["kernel_ms"] / max(prof["launches"], 1)
        per_launch = prof["bytes"] / max(prof["launches"], 1)
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        out["roofline"] = {
            "bound": "hbm",
            "kernel": "finest-level fused Chebyshev step (ELL SpMV + smoother update)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_us": avg_ms * 1e3,
            "bytes_per_launch": per_launch,
            "launches": prof["launches"],
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m, c, fls, bs, timed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
