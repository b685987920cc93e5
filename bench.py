"""Benchmark: masked pressure-correction Poisson solves per second on one GPU.

Headline workload: timesteps on a 64^3 cube.
- Mesh: 64^3 = 262,144-cell jittered (+-10 %) hex cube stored as an
  unstructured face list; 10 mm cavity; aluminium density rho = 2400.
- Solid front: grows from the cold wall x = 0 as sqrt(t) over a 200-step
  schedule of 1e-3 s (mushy band 10 % of the cube).
- Right-hand side: varies smoothly from step to step, standing in for the
  velocity divergence of a flow solve; centred over the liquid cells.
- Each timestep does one masked SA-AMG-PCG solve to 1e-10 relative residual.

One bench step is one timestep's whole hot path: masked assembly, AMG setup,
then PCG.  K consecutive timesteps are timed from the middle of the
schedule, after W warmup steps, with all inputs already in device memory.

Reported:
- value: FP64 AMG-PCG from a zero guess (the plain method).
- variants.mixed: FP32 hierarchy under the FP64 outer PCG.
- variants.mixed_learned: mixed precision, with the initial guess predicted
  by the warm-start network from the previous step.  The network is trained
  beforehand, untimed, on snapshots the solver produced for earlier
  timesteps of the same run.
- variants.c3_128cube (unless --no-c3): repeated solves of one 128^3 system
  (2.1 M cells, random planar front) in FP64 and mixed precision, each with
  its finest-level roofline; at this size the hierarchy outgrows the
  256 MB Infinity Cache.
- variants.c5_plate_ribs (unless --no-c5): timesteps on the 1.5 M-cell plate
  with four ribs, with the front rising from the bottom face.  Compares zero
  and previous-solution guesses in FP64 and mixed precision with the guess
  of the network trained on the cube (a geometry it never saw).
- variants.uq_batched (--uq): 256 uneven uncertainty samples solved as one
  batch.
- roofline: the dominant kernel's achieved HBM bandwidth on the headline
  workload.
- cpu_baseline: the FP64 oracle on host cores.
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
RHO = 2400.0
CAVITY = 0.01  # m
FIRST_TIMED = 100
TRAIN_STEPS = range(20, 80)
RHS_SEED = 5
USTAR_SEED = 7


def note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class Timesteps:
    """A mesh with a growing solid front and a smooth right-hand side per
    timestep k (time (k + 1) dt of a 200-step schedule)."""

    def __init__(self, mesh, axis, length, s_max=0.6):
        from synth import face_coeff

        self.m = mesh
        self.c = face_coeff(mesh, RHO)
        self.axis, self.length, self.s_max = axis, length, s_max

    def inputs(self, k):
        from synth import fl_growing_front, rhs_smooth_series

        t = (k + 1) * DT
        fl = fl_growing_front(self.m.cell_centre, t=t, t_end=N_TIMESTEPS * DT, s_max=self.s_max,
                              delta=0.1, axis=self.axis, length=self.length)
        b = rhs_smooth_series(self.m.cell_centre, t, seed=RHS_SEED, center_mask=fl > 0)
        return fl, b

    def to_device(self, torch, dev, steps):
        m = self.m
        host = {k: self.inputs(k) for k in sorted(set(steps))}
        self.host = host
        return dict(owner=torch.as_tensor(m.owner, device=dev),
                    neigh=torch.as_tensor(m.neigh, device=dev),
                    coeff=torch.as_tensor(self.c, device=dev),
                    vol=torch.as_tensor(m.cell_volume, device=dev),
                    fl={k: torch.as_tensor(v[0], device=dev) for k, v in host.items()},
                    b={k: torch.as_tensor(v[1], device=dev) for k, v in host.items()})


def cpu_baseline(wl, steps, budget_s=20.0):
    """The FP64 oracle (assembly + SA setup + PCG from zero, unmodified) on
    host cores, single-threaded, over as many timed steps as fit the budget."""
    from threadpoolctl import threadpool_limits

    from oracle import amg, assembly, pcg

    m = wl.m
    done, iters, t0 = 0, 0, time.perf_counter()
    with threadpool_limits(limits=1):
        for k in steps:
            fl, b = wl.host[k]
            sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, wl.c, fl)
            H = amg.build_hierarchy(sy.A)
            res = pcg.pcg(sy.A, assembly.pinned_rhs(sy, b), M=lambda r: amg.vcycle(H, r),
                          rtol=1e-10)
            iters += res.iterations
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
    dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=done / dt, unit="solves/s", cores=1, kind="oracle",
                host_cpu=model, host_logical_cpus=os.cpu_count(),
                sample=f"{done} consecutive timed timesteps from step {steps[0]} of the 64^3 run: "
                       f"assembly + SA setup + PCG to 1e-10 from zero ({iters} PCG iterations), "
                       f"{dt:.1f} s on one host thread")


def run_leg(ppe, torch, wl, d_in, steps, warm, precision, guess="zero", net=None,
            autotune=False, reuse=False):
    """Solve warm + steps timesteps; time the last len(steps).  guess: "zero",
    "prev" (the previous step's pressure) or "learned" (net = (network, mu,
    sigma) predicts the increment from the previous step).  autotune: the
    library times its per-level launch choices at assembly (cached by level
    shape; the warmup steps take the first tunings).  reuse: assemblies that
    find the mask and coefficients unchanged keep the system and hierarchy."""
    m, dev = wl.m, d_in["coeff"].device
    s = ppe.Solver(precision=precision, autotune=autotune, reuse_unchanged=reuse)
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
        if guess == "learned":
            network, mu, sigma = net
            F, scale = ppe.warm_start_features(s, dp_prev, b, d_in["coeff"], fl, d_in["vol"], mu,
                                               sigma)
            y = network.forward(F, bf16=True)
            x0 = ppe.warm_start_apply(s, p_prev, y, scale)
        elif guess == "prev":  # the previous pressure re-referenced to the current pins
            zero = torch.zeros(max(s.stats()["n_active"], 1), dtype=torch.float32, device=dev)
            x0 = ppe.warm_start_apply(s, p_prev, zero, 0.0)
        r = s.solve(b, x0=x0, out=out)
        if guess != "zero":
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
    assert rec["worst"] <= 1e-10, f"a timed solve missed the tolerance: {rec['worst']}"
    return rec


def leg_summary(rec, K, base=None):
    import numpy as np

    out = dict(value=K / rec["elapsed"], unit="solves/s",
               ms_per_step=1e3 * rec["elapsed"] / K,
               pcg_iterations_per_solve=rec["iters"] / K,
               setup_ms_per_step=rec["setup_ms"] / K,
               solve_ms_per_step=rec["solve_ms"] / K,
               mean_active_cells=float(np.mean(rec["n_act"])),
               worst_rel_residual=rec["worst"])
    if base is not None:
        out["wall_time_ratio_vs_fp64"] = base["elapsed"] / rec["elapsed"]
        out["solve_time_ratio_vs_fp64"] = base["solve_ms"] / max(rec["solve_ms"], 1e-12)
    return out


def counter_traffic(workload):
    """Bytes per launch of the roofline kernel from the committed memory
    counter summary, or None when the kernel's source region (its operand,
    epilogue and row helpers and the kernel) changed since."""
    import hashlib

    try:
        with open(os.path.join(ROOT, "profiles", "roofline_traffic.json")) as f:
            data = json.load(f)
        with open(os.path.join(ROOT, data["source_file"])) as f:
            text = f.read()
        begin, end = data["source_region"]
        region = text[text.index(begin):text.index(end)]
        if hashlib.sha256(region.encode()).hexdigest() != data["source_sha256"]:
            return None
        return data["workloads"][workload]["bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def roofline(s, run, workload=None):
    """Live measurement of the finest-level Chebyshev step over run(): mean
    dispatch duration from the library's event pairs, algorithmic bytes;
    traffic from the committed counter summary of that workload."""
    s.profile(True)
    run()
    prof = s.profile_read()
    s.profile(False)
    launches = max(prof["launches"], 1)
    avg_ms = prof["kernel_ms"] / launches
    per_launch = prof["bytes"] / launches
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm",
            "kernel": "finest-level Chebyshev step (ELL SpMV + smoother update)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": counter_traffic(workload) if workload else None,
            "avg_launch_us": avg_ms * 1e3, "bytes_per_launch": per_launch,
            "launches": prof["launches"]}


def train_network(ppe, torch, wl, d_in, n_adam=400, batch=8192):
    """Snapshots produced by the solver on earlier timesteps -> trained
    network and feature standardisation (untimed)."""
    import numpy as np

    from synth import mlp_initial_weights

    m, dev = wl.m, d_in["coeff"].device
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


def projection_leg(ppe, torch, wl, d_in, steps, warm, dev, base, krylov="bicgstab"):
    """The whole pressure-correction step on the same 64^3 timesteps: a smooth
    synthetic u* per step, masked assembly, then ppe_project (cross diffusion
    by deferred correction around the AMG-PCG solve, consistent face fluxes
    and corrected velocities).  The fluxes' divergence is checked on the
    device after the timed region."""
    import numpy as np

    from synth import ustar_smooth_series

    m = wl.m

    def dev_t(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)

    s = ppe.Solver(precision="fp64", krylov=krylov)
    s.set_mesh(m.n_cells, d_in["owner"], d_in["neigh"])
    s.set_geometry(dev_t(m.nodes, torch.float64), dev_t(m.extra["face_nodes"], torch.int32),
                   dev_t(m.extra["cell_nodes"], torch.int32), dev_t(m.cell_centre, torch.float64),
                   dev_t(m.face_area, torch.float64))
    us = {k: dev_t(ustar_smooth_series(m.cell_centre, (k + 1) * DT, seed=USTAR_SEED), torch.float64)
          for k in warm + steps}
    coeff = d_in["coeff"]
    for k in warm:
        s.assemble(coeff, d_in["fl"][k])
        s.project(coeff, us[k], RHO, DT)
    torch.cuda.synchronize()
    outer = iters = 0
    worst = 0.0
    t0 = time.perf_counter()
    for k in steps:
        s.assemble(coeff, d_in["fl"][k])
        _, F, _, st = s.project(coeff, us[k], RHO, DT)
        outer += st["outer"]
        iters += st["pcg_iterations"]
        worst = max(worst, st["rel_residual"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    own, nb = d_in["owner"].long(), d_in["neigh"].long()
    inner = nb >= 0
    div = torch.zeros(m.n_cells, dtype=torch.float64, device=dev)
    div.index_add_(0, own[inner], F[inner])
    div.index_add_(0, nb[inner], -F[inner])
    K = len(steps)
    return {
        "workload": "64^3 timesteps of the headline run with a smooth synthetic u* per step; "
                    "assembly + cross-diffusion pressure step ("
                    + ("deferred correction around AMG-PCG" if krylov == "deferred" else
                       "BiCGSTAB on the full system, one V-cycle of L per preconditioning")
                    + ") + Eq. 17 fluxes + corrected velocities, FP64",
        "steps_per_s": K / el,
        "ms_per_step": 1e3 * el / K,
        "time_ratio_vs_direct_only_solve": (el / K) / (base["elapsed"] / K),
        ("outer_passes_per_step" if krylov == "deferred" else "bicgstab_iterations_per_step"):
            outer / K,
        ("pcg_iterations_per_step" if krylov == "deferred" else "vcycles_per_step"): iters / K,
        "worst_rel_residual_full_system": worst,
        "last_step_max_divergence_rel_to_max_flux": float(div.abs().max() / F.abs().max()),
    }


FLOW_DT = 5e-6          # alpha dt / h^2 of about 0.008 at 64^3 (h = 10 mm / 64)
FLOW_LAYER = 1.5e-3     # m, width of the initial thermal boundary layer


def fractional_step_leg(ppe, torch, dev, K, W, krylov="bicgstab"):
    """Whole fractional steps (section 2.2 steps 1-4) on the 64^3 cube: the
    paper's die casting (Al-10 % Si melt at 1000 K, walls held at 500 K)
    from a developed boundary layer, so a solid rim and a mushy front exist
    and the front moves; natural convection on.  Inputs resident in HBM;
    the state stays on the device between steps."""
    import numpy as np

    from synth import al_si_alloy, box_mesh, t_wall_layer

    m = box_mesh((64, 64, 64), lengths=(CAVITY,) * 3, jitter=0.1, seed=0)
    props = al_si_alloy(T_wall=500.0)

    def dev_t(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)

    fw = ppe.Flow(krylov=krylov)
    fw.set_mesh(dev_t(m.owner, torch.int32), dev_t(m.neigh, torch.int32),
                dev_t(m.nodes, torch.float64), dev_t(m.extra["face_nodes"], torch.int32),
                dev_t(m.extra["cell_nodes"], torch.int32), dev_t(m.cell_centre, torch.float64),
                dev_t(m.face_area, torch.float64), dev_t(m.face_centre, torch.float64),
                dev_t(m.cell_volume, torch.float64))
    T0 = t_wall_layer(m, props["T_wall"], 1000.0, FLOW_LAYER)
    st = fw.new_state(dev_t(T0, torch.float64), props=props)  # f_s(T0) on the device
    for _ in range(max(W, 1)):
        fw.step(props, st, FLOW_DT)
    torch.cuda.synchronize()
    keys = ("picard", "momentum_iterations", "pressure_outer", "pressure_iterations",
            "energy_iterations", "momentum_ms", "pressure_ms", "energy_ms")
    acc = dict.fromkeys(keys, 0.0)
    worst_picard = 0
    solid = []
    t0 = time.perf_counter()
    for _ in range(K):
        _, stt = fw.step(props, st, FLOW_DT)
        solid.append(stt["n_solid"])
        for q in keys:
            acc[q] += stt[q]
        worst_picard = max(worst_picard, stt["picard"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {
        "workload": "64^3 jittered hex cube (10 mm), Al-10% Si melt at 1000 K against walls at "
                    f"500 K from a {FLOW_LAYER * 1e3:.1f} mm boundary layer, dt {FLOW_DT:g} s, "
                    "natural convection; momentum predictor (3 AMG-PCG solves of a shifted "
                    f"system) + masked cross-diffusion projection ({krylov}) + energy Picard loop "
                    "(shifted AMG setup on the first pass, finest-level refresh on the later "
                    "ones, one solve per pass), FP64",
        "steps_per_s": K / el,
        "ms_per_step": 1e3 * el / K,
        "cells": m.n_cells,
        "solid_cells_first_last": [int(solid[0]), int(solid[-1])],
        "max_picard": int(worst_picard),
        **{f"{q}_per_step": acc[q] / K for q in keys},
    }


def uq_fractional_step(ppe, torch, dev, side=32, n_steps=10, dt=2e-5, level=3, degree=2,
                       n_test=20):
    """The paper's die-casting uncertainty study (section 4) on the time-step
    driver: solute C0 ~ N(10, 0.2) wt %, initial melt temperature
    ~ N(1000, 10) K and wall temperature ~ N(500, 5) K; the full tensor grid
    of `level` Gauss points per input (27 samples at level 3, the paper's
    smaller set); each sample runs n_steps fractional steps on a side^3 cube
    from a boundary layer of 1.5 mm; outputs are the mean temperature, the
    solid volume fraction and the peak speed after those steps; a
    total-degree expansion of them, its Sobol indices, and the paper's
    Latin-hypercube check (RMS of expansion minus simulation, here over the
    outputs' spread across the test points)."""
    import numpy as np

    from synth import al_si_alloy, box_mesh, latin_hypercube, t_wall_layer

    kinds = ["normal", "normal", "normal"]
    q = ppe.PolynomialChaos(kinds, degree)
    m = box_mesh((side,) * 3, lengths=(CAVITY,) * 3, jitter=0.1, seed=0)

    def dev_t(a, dtp):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dtp, device=dev)

    fw = ppe.Flow()
    fw.set_mesh(dev_t(m.owner, torch.int32), dev_t(m.neigh, torch.int32),
                dev_t(m.nodes, torch.float64), dev_t(m.extra["face_nodes"], torch.int32),
                dev_t(m.extra["cell_nodes"], torch.int32), dev_t(m.cell_centre, torch.float64),
                dev_t(m.face_area, torch.float64), dev_t(m.face_centre, torch.float64),
                dev_t(m.cell_volume, torch.float64))
    V = dev_t(m.cell_volume, torch.float64)

    def run(X):
        Y = torch.empty((X.shape[0], 3), dtype=torch.float64, device=dev)
        picard = 0
        for k, x in enumerate(X):
            props = al_si_alloy(si_wt=10.0 + 0.2 * x[0], T_wall=500.0 + 5.0 * x[2])
            T0 = t_wall_layer(m, props["T_wall"], 1000.0 + 10.0 * x[1], 1.5e-3)
            st = fw.new_state(dev_t(T0, torch.float64), props=props)
            for stt in fw.run(props, st, dt, n_steps):
                picard += stt["picard"]
            Y[k, 0] = (V * st.T).sum() / V.sum()
            Y[k, 1] = (V * st.fs).sum() / V.sum()
            Y[k, 2] = st.u.norm(dim=1).max()
        return Y, picard

    X, _ = q.nodes("tensor", level)
    run(X[:1])  # warm-up of the driver's buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Y, picard = run(X)
    torch.cuda.synchronize()
    t_runs = time.perf_counter() - t0
    W = q.fit(X, Y)
    mean, var, first, total = (v.cpu().numpy() for v in q.stats(W))
    T, _ = latin_hypercube(kinds, n_test, seed=17)
    Yt, _ = run(T)
    yt, ye = Yt.cpu().numpy(), q.eval(T, W).cpu().numpy()
    spread = yt.max(axis=0) - yt.min(axis=0)
    names = ["mean_T", "solid_fraction", "max_speed"]
    return {
        "workload": f"{side}^3 cube, Al-Si die casting with C0 ~ N(10, 0.2) wt %, T_init ~ "
                    f"N(1000, 10) K, T_wall ~ N(500, 5) K; {X.shape[0]}-point tensor grid, "
                    f"{n_steps} fractional steps of {dt:g} s per sample (BiCGSTAB projection), "
                    f"degree-{degree} expansion; {n_test} Latin-hypercube test runs",
        "samples": int(X.shape[0]),
        "sample_steps_per_s": X.shape[0] * n_steps / t_runs,
        "seconds_for_all_samples": t_runs,
        "picard_per_step": picard / (X.shape[0] * n_steps),
        "outputs": {
            nm: {"mean": float(mean[j]), "std": float(np.sqrt(var[j])),
                 "sobol_first": [float(v) for v in first[:, j]],
                 "sobol_total": [float(v) for v in total[:, j]],
                 "lhs_rms_error_over_spread": float(np.sqrt(np.mean((ye[:, j] - yt[:, j]) ** 2))
                                                     / max(spread[j], 1e-300)),
                 # the paper's measure: the difference over the output's mean value
                 "lhs_rms_error_over_mean": float(np.sqrt(np.mean((ye[:, j] - yt[:, j]) ** 2))
                                                   / max(abs(float(mean[j])), 1e-300))}
            for j, nm in enumerate(names)},
    }


def c3_leg(ppe, torch, dev, reps=4):
    """One 128^3 system (random planar front), solved repeatedly."""
    from synth import box_mesh, face_coeff, fl_planar_front, rhs_uniform

    m = box_mesh((128, 128, 128), jitter=0.1, seed=0)
    fh = fl_planar_front(m.cell_centre, seed=2)
    c = torch.as_tensor(face_coeff(m, RHO), device=dev)
    f = torch.as_tensor(fh, device=dev)
    b = torch.as_tensor(rhs_uniform(m.n_cells, seed=1, center_mask=fh > 0), device=dev)
    owner = torch.as_tensor(m.owner, device=dev)
    neigh = torch.as_tensor(m.neigh, device=dev)
    out = {"workload": "128^3 jittered cube, planar front (normal seed 2), uniform RHS; "
                       f"{reps} timed solves of one assembled system after one untimed; "
                       "launch choices autotuned at assembly (setup_ms includes the tuning)"}
    for prec in ("fp64", "mixed"):
        s = ppe.Solver(precision=prec, autotune=True)
        s.set_mesh(m.n_cells, owner, neigh)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.assemble(c, f)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        p = torch.zeros(m.n_cells, dtype=torch.float64, device=dev)
        r = s.solve(b, out=p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = s.solve(b, out=p)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        assert r.stats["rel_residual"] <= 1e-10
        out[prec] = dict(solves_per_s=1.0 / dt, solve_ms=1e3 * dt, setup_ms=1e3 * t_setup,
                         pcg_iterations=r.stats["iterations"], active_cells=r.stats["n_active"],
                         levels=r.stats["levels"], rel_residual=r.stats["rel_residual"],
                         roofline=roofline(s, lambda: s.solve(b, out=p),
                                           "128cube_planar_front" if prec == "fp64" else None))
    return out


def c5_leg(ppe, torch, dev, net, steps=10, warm=3, first=40):
    """Timesteps on the plate with ribs, front rising from the bottom face."""
    from synth import plate_with_ribs_mesh

    m = plate_with_ribs_mesh()
    height = float(m.cell_centre[:, 2].max() - m.cell_centre[:, 2].min()) + 2.0e-3 / 3.0
    wl = Timesteps(m, axis=2, length=height)
    K = list(range(first, first + steps))
    W = list(range(first - warm, first))
    d_in = wl.to_device(torch, dev, W + K)
    base = run_leg(ppe, torch, wl, d_in, K, W, "fp64", autotune=True)
    out = {"workload": f"plate with ribs, {m.n_cells} cells (+-5 % jitter), front rising from "
                       f"the bottom face, timesteps {K[0]}..{K[-1]} of 200 x 1e-3 s; network "
                       "trained on the 64^3 cube run only; launch choices autotuned",
           "fp64_zero_guess": leg_summary(base, steps)}
    for name, prec, guess in (("fp64_previous_guess", "fp64", "prev"),
                              ("mixed_zero_guess", "mixed", "zero"),
                              ("mixed_previous_guess", "mixed", "prev"),
                              ("mixed_learned", "mixed", "learned")):
        rec = run_leg(ppe, torch, wl, d_in, K, W, prec, guess=guess, net=net, autotune=True)
        out[name] = leg_summary(rec, steps, base)
    return out


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
        s.solve(data[k][1], out=out)
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


def uq_collocation(ppe, torch, dev, side=32, level=6, degree=5, n_test=60):
    """The paper's uncertainty wrapper on the batched solver: three inputs
    (melt and wall temperature normal, liquidus shift uniform), the full
    tensor grid of `level` Gauss points per input (216 samples at level 6,
    the paper's three-input size), one batched assembly and solve of all
    samples on identical side^3 meshes, a total-degree polynomial-chaos fit
    of the whole pressure field, its statistics, and the paper's check on
    Latin-hypercube test points (RMS of expansion minus simulation over the
    largest pressure magnitude)."""
    import numpy as np

    from synth import box_mesh, concat_meshes, face_coeff, latin_hypercube, rhs_smooth_series, \
        uq_front_fl

    kinds = ["normal", "normal", "uniform"]
    q = ppe.PolynomialChaos(kinds, degree)
    m = box_mesh((side,) * 3, lengths=(CAVITY,) * 3, jitter=0.1, seed=0)
    t, t_end = 30 * DT, 50 * DT

    def fields(X):
        fls, bs = [], []
        for x in X:
            sm = dict(t_melt=950.0 + 10.0 * x[0], t_wall=600.0 + 20.0 * x[1], d_liq=5.0 * x[2])
            f = uq_front_fl(m.cell_centre, sm, t, t_end, length=CAVITY)
            fls.append(f)
            bs.append(rhs_smooth_series(m.cell_centre, t, seed=RHS_SEED, center_mask=f > 0))
        return np.concatenate(fls), np.concatenate(bs)

    def batch(X):
        u = concat_meshes([m] * X.shape[0])
        s = ppe.Solver(precision="mixed")
        s.set_mesh(u.n_cells, torch.as_tensor(u.owner, device=dev), torch.as_tensor(u.neigh, device=dev))
        s.set_segments(u.extra["cell_offsets"])
        fl, b = fields(X)
        return s, torch.as_tensor(face_coeff(u, RHO), device=dev), torch.as_tensor(fl, device=dev), \
            torch.as_tensor(b, device=dev)

    X, _ = q.nodes("tensor", level)
    s, c, fl, b = batch(X)
    s.assemble(c, fl)  # warm-up assembly and solve
    s.solve(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.assemble(c, fl)
    res = s.solve(b)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    its, rr = s.segment_stats()
    Y = res.p.reshape(X.shape[0], m.n_cells)
    q.fit(X, Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W = q.fit(X, Y)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    mean, var, first, total = q.stats(W)
    T, _ = latin_hypercube(kinds, n_test, seed=17)
    s2, c2, fl2, b2 = batch(T)
    s2.assemble(c2, fl2)
    Yt = s2.solve(b2).p.reshape(n_test, m.n_cells)
    Ye = q.eval(T, W)
    rms = float(torch.sqrt(((Ye - Yt) ** 2).mean()) / Yt.abs().max())
    varying = var > 1e-6 * var.max()
    return {
        "workload": f"3 inputs (T_melt ~ N(950,10), T_wall ~ N(600,20), dT_liq ~ U(-5,5)), tensor grid of "
                    f"{level} Gauss points per input ({X.shape[0]} samples) on {side}^3 cubes, one "
                    f"batched assembly + solve (mixed precision), total-degree-{degree} expansion "
                    f"({q.n_terms} terms) of every cell's pressure",
        "samples": int(X.shape[0]),
        "cells": int(X.shape[0] * m.n_cells),
        "sample_solves_per_s": X.shape[0] / t_solve,
        "batch_ms": 1e3 * t_solve,
        "mean_sample_iterations": float(np.mean(its)),
        "worst_rel_residual": float(max(rr)),
        "fit_ms": 1e3 * t_fit,
        "fit_gb_per_s": X.shape[0] * m.n_cells * 8 / t_fit / 1e9,
        "lhs_test_points": n_test,
        "lhs_rms_error_rel_to_max": rms,
        "mean_total_sobol_of_varying_cells": [float(total[j][varying].mean()) for j in range(3)],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="time the FP64 leg only")
    ap.add_argument("--no-c3", action="store_true", help="skip the 128^3 leg")
    ap.add_argument("--no-c5", action="store_true", help="skip the plate-with-ribs leg")
    ap.add_argument("--no-projection", action="store_true",
                    help="skip the cross-diffusion pressure-correction leg")
    ap.add_argument("--no-uq-collocation", action="store_true",
                    help="skip the polynomial-chaos collocation leg")
    ap.add_argument("--projection-only", action="store_true",
                    help="time the FP64 leg and the pressure-correction leg only (for profiling)")
    ap.add_argument("--no-flow", action="store_true", help="skip the fractional-step legs")
    ap.add_argument("--flow-only", action="store_true",
                    help="time the FP64 leg and the fractional-step leg only (for profiling)")
    ap.add_argument("--uq", action="store_true", help="add the batched-UQ measurement")
    ap.add_argument("--c3-only", action="store_true",
                    help="run only the 128^3 leg and print its JSON (for profiling it alone)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy a 512 MiB buffer three times (a kernel of known traffic, "
                         "for scaling memory counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding design); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1810_08572_amd as ppe
    from synth import box_mesh

    dev = torch.device("cuda", 0)
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.c3_only:
        print(json.dumps(c3_leg(ppe, torch, dev)), flush=True)
        return
    K, W = args.steps, args.warmup
    steps = list(range(FIRST_TIMED, FIRST_TIMED + K))
    warm = list(range(FIRST_TIMED - W, FIRST_TIMED))
    wl = Timesteps(box_mesh((64, 64, 64), lengths=(CAVITY,) * 3, jitter=0.1, seed=0), axis=0,
                   length=CAVITY)
    need = warm + steps + ([] if args.no_variants or args.projection_only or args.flow_only
                           else list(TRAIN_STEPS))
    d_in = wl.to_device(torch, dev, need)
    note(f"inputs ready: {len(set(need))} timesteps of {wl.m.n_cells} cells")

    base = run_leg(ppe, torch, wl, d_in, steps, warm, "fp64")
    note(f"fp64 leg: {K / base['elapsed']:.1f} solves/s")
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
            "cells": wl.m.n_cells,
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

        def rerun():
            for k in steps:
                s.assemble(d_in["coeff"], d_in["fl"][k])
                s.solve(d_in["b"][k])

        out["roofline"] = roofline(s, rerun, "64cube_timesteps")
        out["roofline"]["kernel"] += ", FP64"

    if args.flow_only:
        out["variants"] = {"fractional_step": fractional_step_leg(ppe, torch, dev, K, W),
                           "fractional_step_deferred": fractional_step_leg(ppe, torch, dev, K, W,
                                                                           krylov="deferred"),
                           "uq_fractional_step": uq_fractional_step(ppe, torch, dev)}
        print(json.dumps(out), flush=True)
        return
    if args.projection_only:
        out["variants"] = {
            "projection_cross_diffusion": projection_leg(ppe, torch, wl, d_in, steps, warm, dev,
                                                         base),
            "projection_cross_diffusion_deferred": projection_leg(ppe, torch, wl, d_in, steps,
                                                                  warm, dev, base, "deferred")}
        print(json.dumps(out), flush=True)
        return
    if not args.no_variants:
        variants = {}
        mixed = run_leg(ppe, torch, wl, d_in, steps, warm, "mixed")
        variants["mixed"] = leg_summary(mixed, K, base)
        note(f"mixed leg: {K / mixed['elapsed']:.1f} solves/s")
        net, mu, sigma, tr = train_network(ppe, torch, wl, d_in)
        note(f"network trained: {tr}")
        ml = run_leg(ppe, torch, wl, d_in, steps, warm, "mixed", guess="learned",
                     net=(net, mu, sigma))
        variants["mixed_learned"] = dict(leg_summary(ml, K, base), training=tr)
        note(f"mixed+learned leg: {K / ml['elapsed']:.1f} solves/s")
        ru = run_leg(ppe, torch, wl, d_in, steps, warm, "fp64", reuse=True)
        variants["fp64_reuse_unchanged"] = dict(
            leg_summary(ru, K, base),
            reused_assemblies=int(ru["solver"].stats()["reused_setup"]),
            note="the same timesteps (reused_assemblies counts warmup and timed steps); an assembly whose mask and coefficients equal the previous "
                 "one's keeps the system and hierarchy (the matrix depends on nothing else)")
        note(f"fp64 reuse leg: {K / ru['elapsed']:.1f} solves/s")
        if not args.no_projection:
            variants["projection_cross_diffusion"] = projection_leg(ppe, torch, wl, d_in, steps,
                                                                    warm, dev, base)
            variants["projection_cross_diffusion_deferred"] = projection_leg(
                ppe, torch, wl, d_in, steps, warm, dev, base, "deferred")
            note("projection legs done")
        if not args.no_flow:
            variants["fractional_step"] = fractional_step_leg(ppe, torch, dev, K, W)
            note("fractional-step leg done")
            variants["uq_fractional_step"] = uq_fractional_step(ppe, torch, dev)
            note("uncertainty over fractional steps done")
        if not args.no_uq_collocation:
            variants["uq_collocation"] = uq_collocation(ppe, torch, dev)
            note("collocation leg done")
        if not args.no_c3:
            variants["c3_128cube"] = c3_leg(ppe, torch, dev)
            note("128^3 leg done")
        if not args.no_c5:
            variants["c5_plate_ribs"] = c5_leg(ppe, torch, dev, (net, mu, sigma))
            note("plate-with-ribs leg done")
        out["variants"] = variants
    if args.uq:
        out.setdefault("variants", {})["uq_batched"] = uq_batched(ppe, torch, dev)
        note("batched UQ leg done")
    if not args.no_cpu_baseline:
        note("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(wl, steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
