"""Benchmark: masked pressure-correction Poisson solves per second on one GPU.

Headline workload: timesteps on the plate with ribs (1.5 M cells).
- Mesh: 240 x 144 x 36 cells (160 x 96 x 24 mm at h = 2/3 mm) with four
  ribs of 8 x 144 x 56 cells on top, 1,502,208 jittered (+-5 %) hex cells
  stored as an unstructured face list; aluminium density rho = 2400.
- Solid front: rises from the bottom face as s(t) = 0.6 H sqrt(t / 0.2 s)
  over a 200-step schedule of 1e-3 s (mushy band 10 % of the height H).
- Right-hand side: a sum of smooth modes varying smoothly from step to step,
  standing in for the velocity divergence of a flow solve; centred over the
  liquid cells.
- Each timestep does one masked SA-AMG-PCG solve to 1e-10 relative
  residual.  One bench step is one timestep's whole hot path: masked
  assembly, AMG setup, then PCG (inputs already in device memory).

Reported (one JSON line):
- value: FP64 AMG-PCG from a zero guess (the plain method), solves/s.
- roofline: the solve kernel with the largest total time, from the
  library's per-dispatch event pairs during a re-run of the timed steps
  (algorithmic bytes / kernel time); pcg_iteration: every solve kernel
  together (the V-cycle and the PCG vector work).
- variants.c5_plate: the same timesteps from the previous solution, in
  mixed precision, with the learned warm start (trained beforehand, untimed,
  on snapshots of earlier timesteps of the same run), with l1-Jacobi
  smoothing, and with unchanged systems reused.
- variants.c3_128cube: assembly + solve of a 128^3 cube with a random
  planar front, FP64 and mixed, with their dominant kernels' rooflines.
- variants.c4_uq_batched: 256 uneven uncertainty samples (sides 24..48)
  solved as one batch per timestep, mixed precision.
- variants.c2_64cube: the 64^3 timesteps (FP64, mixed, learned).
- variants.projection_*, fractional_step*, uq_collocation: the next rows
  of the method (cross diffusion, whole fractional steps, collocation).
- cpu_baseline: the FP64 oracle on one host core, on a bounded sample of the
  headline workload.
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

METRIC = "pressure solves/s at 1e-10 rel. residual, FP64 vs mixed+learned; HBM GB/s"
HBM_PEAK_GBS = 8000.0
N_TIMESTEPS = 200
DT = 1e-3
RHO = 2400.0
CAVITY = 0.01  # m, side of the cube workloads
RHS_SEED = 5
USTAR_SEED = 7
C5_FIRST = 40                 # first timed timestep of the plate run
C5_TRAIN = range(8, 38, 1)    # snapshot timesteps for the warm-start network
C2_FIRST = 100
C2_TRAIN = range(20, 80)


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
        self.host = {}

    def inputs(self, k):
        from synth import fl_growing_front, rhs_smooth_series

        if k not in self.host:
            t = (k + 1) * DT
            fl = fl_growing_front(self.m.cell_centre, t=t, t_end=N_TIMESTEPS * DT,
                                  s_max=self.s_max, delta=0.1, axis=self.axis,
                                  length=self.length)
            b = rhs_smooth_series(self.m.cell_centre, t, seed=RHS_SEED, center_mask=fl > 0)
            self.host[k] = (fl, b)
        return self.host[k]

    def to_device(self, torch, dev, steps):
        m = self.m
        d = dict(owner=torch.as_tensor(m.owner, device=dev),
                 neigh=torch.as_tensor(m.neigh, device=dev),
                 coeff=torch.as_tensor(self.c, device=dev),
                 vol=torch.as_tensor(m.cell_volume, device=dev), fl={}, b={})
        for k in sorted(set(steps)):
            fl, b = self.inputs(k)
            d["fl"][k] = torch.as_tensor(fl, device=dev)
            d["b"][k] = torch.as_tensor(b, device=dev)
        return d


def plate_workload():
    from synth import plate_with_ribs_mesh

    m = plate_with_ribs_mesh()
    height = float(m.cell_centre[:, 2].max() - m.cell_centre[:, 2].min()) + 2.0e-3 / 3.0
    return Timesteps(m, axis=2, length=height)


def cube_workload(side=64):
    from synth import box_mesh

    return Timesteps(box_mesh((side,) * 3, lengths=(CAVITY,) * 3, jitter=0.1, seed=0), axis=0,
                     length=CAVITY)


def host_cpu():
    try:
        with open("/proc/cpuinfo") as fh:
            return next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")),
                        "")
    except OSError:
        return ""


def cpu_baseline(wl, k, gpu_iterations, max_iter=10):
    """The FP64 oracle (assembly + SA setup + PCG from zero, unmodified) on one
    host thread, on a bounded sample of timestep k: the assembly and setup
    in full, then max_iter PCG iterations; a whole solve is the setup time
    plus gpu_iterations times the measured time per iteration (the oracle's
    count equals the GPU's within one, a tested parity property)."""
    from threadpoolctl import threadpool_limits

    from oracle import amg, assembly, pcg

    m = wl.m
    fl, b = wl.inputs(k)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        sy = assembly.masked_system(m.n_cells, m.owner, m.neigh, wl.c, fl)
        H = amg.build_hierarchy(sy.A)
        t1 = time.perf_counter()
        res = pcg.pcg(sy.A, assembly.pinned_rhs(sy, b), M=lambda r: amg.vcycle(H, r), rtol=1e-10,
                      max_iter=max_iter)
        t2 = time.perf_counter()
    per_iter = (t2 - t1) / max(res.iterations, 1)
    solve_s = (t1 - t0) + gpu_iterations * per_iter
    return dict(value=1.0 / solve_s, unit="solves/s", cores=1, kind="oracle",
                host_cpu=host_cpu(), host_logical_cpus=os.cpu_count(),
                setup_s=t1 - t0, s_per_pcg_iteration=per_iter,
                dof_iterations_per_s=sy.n_active / per_iter,
                sample=f"timestep {k} of the plate run ({sy.n_active} active cells): oracle "
                       f"assembly + SA setup in full ({t1 - t0:.1f} s) and {res.iterations} PCG "
                       f"iterations ({t2 - t1:.1f} s) on one host thread; one solve = setup + "
                       f"{gpu_iterations} iterations (the FP64 GPU count of that step)")


def run_leg(ppe, torch, wl, d_in, steps, warm, precision, guess="zero", net=None,
            autotune=False, reuse=False, smoother="chebyshev", coarse_reuse=0):
    """Solve warm + steps timesteps; time the last len(steps).  guess: "zero",
    "prev" (the previous step's pressure) or "learned" (net = (network, mu,
    sigma) predicts the increment from the previous step).  autotune: the
    library times its per-level launch choices at assembly (cached by level
    shape; the warmup steps take the first tunings).  reuse: assemblies that
    find the mask and coefficients unchanged keep the system and hierarchy.
    coarse_reuse: changed masks keep the coarse levels of the last full setup
    for up to that many assemblies (the finest level is rebuilt)."""
    m, dev = wl.m, d_in["coeff"].device
    s = ppe.Solver(precision=precision, autotune=autotune, reuse_unchanged=reuse,
                   smoother=smoother, coarse_reuse=coarse_reuse)
    s.set_mesh(m.n_cells, d_in["owner"], d_in["neigh"])
    p_prev = torch.zeros(m.n_cells, dtype=torch.float64, device=dev)
    dp_prev = torch.zeros_like(p_prev)
    out = torch.zeros_like(p_prev)
    rec = dict(iters=0, setup_ms=0.0, solve_ms=0.0, worst=0.0, n_act=[], bytes_iter=[],
               reused=0, coarse_reused=0)
    feats = None
    if guess == "learned":
        feats = torch.empty((m.n_cells, 10), dtype=torch.float32, device=dev)

    def one(k, timed):
        nonlocal p_prev, dp_prev, out
        fl, b = d_in["fl"][k], d_in["b"][k]
        st0 = s.stats()
        s.assemble(d_in["coeff"], fl)
        x0 = None
        if guess == "learned":
            network, mu, sigma = net
            scale = ppe.warm_start_features_noalloc(s, dp_prev, b, d_in["coeff"], fl, d_in["vol"],
                                                    mu, sigma, feats)
            na = s.stats()["n_active"]
            y = network.forward(feats[:na], bf16=True)
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
            rec.setdefault("first_iters", st["iterations"])
            rec["iters"] += st["iterations"]
            rec["setup_ms"] += st["setup_ms"]
            rec["solve_ms"] += st["solve_ms"]
            rec["worst"] = max(rec["worst"], st["rel_residual"])
            rec["n_act"].append(st["n_active"])
            rec["bytes_iter"].append(st["bytes_per_iter"])
            rec["reused"] += st["reused_setup"] - st0["reused_setup"]
            rec["coarse_reused"] += st["coarse_reused"] - st0["coarse_reused"]

    for k in warm:
        one(k, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in steps:
        one(k, True)
    torch.cuda.synchronize()
    rec["elapsed"] = time.perf_counter() - t0
    rec["solver"] = s
    rec["rerun"] = lambda: [one(k, False) for k in steps]
    assert rec["worst"] <= 1e-10, f"a timed solve missed the tolerance: {rec['worst']}"
    return rec


def leg_summary(rec, K, base=None):
    import numpy as np

    it = rec["iters"] / K
    out = dict(value=K / rec["elapsed"], unit="solves/s",
               ms_per_step=1e3 * rec["elapsed"] / K,
               pcg_iterations_per_solve=it,
               setup_ms_per_step=rec["setup_ms"] / K,
               solve_ms_per_step=rec["solve_ms"] / K,
               mean_active_cells=float(np.mean(rec["n_act"])),
               dof_iterations_per_s=float(np.sum(rec["n_act"])) * it / rec["elapsed"],
               worst_rel_residual=rec["worst"])
    if rec.get("reused"):
        out["reused_assemblies"] = rec["reused"]
    if rec.get("coarse_reused"):
        out["coarse_reused_assemblies"] = rec["coarse_reused"]
    if base is not None:
        out["wall_time_ratio_vs_fp64"] = base["elapsed"] / rec["elapsed"]
        out["solve_time_ratio_vs_fp64"] = base["solve_ms"] / max(rec["solve_ms"], 1e-12)
    return out


def counter_traffic(workload, kernel):
    """Bytes per launch of `kernel` from the committed memory-counter summary
    of `workload`, or None when the summary does not cover the kernel or the
    source region of the solve kernels changed since the counters were
    taken."""
    import hashlib

    try:
        with open(os.path.join(ROOT, "profiles", "roofline_traffic.json")) as f:
            data = json.load(f)
        entry = data["workloads"][workload]
        with open(os.path.join(ROOT, data["source_file"])) as f:
            text = f.read()
        begin, end = entry["source_region"]
        region = text[text.index(begin):text.index(end)]
        if hashlib.sha256(region.encode()).hexdigest() != entry["source_sha256"]:
            return None
        return entry["kernels"][kernel]["bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def profile_table(s, run):
    """Per-kernel table of the solve phase over run(): the library times each
    dispatch with its own event pair on the solver's stream."""
    s.profile(True)
    run()
    table = s.profile_read()
    s.profile(False)
    return table


COPY = {}


def copy_bandwidth(torch, dev, mib=192, reps=20):
    """Bytes read + written per second by a plain device-to-device copy of
    `mib` MiB (torch's copy kernel), the practical HBM rate that the
    kernels' rates are set beside."""
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    COPY.update(gbs=2.0 * n * 8 / (ms * 1e-3) / 1e9, mib=mib)
    return COPY["gbs"]


def roofline(table, workload=None, label=""):
    """The kernel with the largest total time in the table, against the HBM
    peak (algorithmic bytes / kernel time); plus every solve kernel
    together (pcg_iteration)."""
    name, e = max(table.items(), key=lambda kv: kv[1]["kernel_ms"])
    total_ms = sum(v["kernel_ms"] for v in table.values())
    total_b = sum(v["bytes"] for v in table.values())
    achieved = e["bytes"] / (e["kernel_ms"] * 1e-3) / 1e9
    top = sorted(table.items(), key=lambda kv: -kv[1]["kernel_ms"])[:8]
    return {"bound": "hbm",
            "kernel": name + (f" ({label})" if label else ""),
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": counter_traffic(workload, name) if workload else None,
            "avg_launch_us": 1e3 * e["kernel_ms"] / e["launches"],
            "bytes_per_launch": e["bytes"] / e["launches"],
            "launches": e["launches"],
            "share_of_solve_kernel_time": e["kernel_ms"] / total_ms,
            "pcg_iteration": {"kernels": "every V-cycle and PCG kernel of the solve",
                              "achieved": total_b / (total_ms * 1e-3) / 1e9,
                              "frac": total_b / (total_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "kernel_ms": total_ms, "bytes": total_b},
            "top_kernels": [{"kernel": k, "share": v["kernel_ms"] / total_ms,
                             "avg_launch_us": 1e3 * v["kernel_ms"] / v["launches"],
                             "frac": v["bytes"] / (v["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                            for k, v in top],
            "copy_gbs": COPY.get("gbs"),
            "copy_note": (f"a plain device copy of {COPY['mib']} MiB (read + write) measured in "
                          "the same process" if COPY else None)}


def train_network(ppe, torch, wl, d_in, steps, n_adam=600, batch=8192):
    """Snapshots produced by the solver on earlier timesteps of the same run
    -> trained network and feature standardisation (untimed).  A snapshot is
    taken on steps whose mask equals the previous step's (a mask change moves
    pins and opens cells, and its increment is not a local function of the
    features)."""
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
    for k in steps:
        fl, b = d_in["fl"][k], d_in["b"][k]
        masks.append(fl > 0)
        s.assemble(d_in["coeff"], fl)
        stable = len(masks) >= 2 and bool(torch.equal(masks[-1], masks[-2]))
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
                                steps=f"{steps[0]}..{steps[-1]}",
                                loss_first=float(np.mean(losses[:10])),
                                loss_last=float(np.mean(losses[-10:])))


def c5_legs(ppe, torch, wl, d_in, K, W, base, net):
    steps = list(range(C5_FIRST, C5_FIRST + K))
    warm = list(range(C5_FIRST - W, C5_FIRST))
    out = {"workload": f"plate with ribs, {wl.m.n_cells} cells (+-5 % jitter), front rising from "
                       f"the bottom face, timesteps {steps[0]}..{steps[-1]} of 200 x 1e-3 s "
                       f"after {W} warmup steps; assembly + setup + solve per step; fixed launch "
                       "rules unless the leg says autotuned"}
    legs = (("fp64_previous_guess", "fp64", "prev", False, "chebyshev", False),
            ("fp64_zero_guess_autotuned", "fp64", "zero", False, "chebyshev", True),
            ("fp64_zero_guess_l1jacobi", "fp64", "zero", False, "l1jacobi", False),
            ("mixed_zero_guess", "mixed", "zero", False, "chebyshev", False),
            ("mixed_previous_guess", "mixed", "prev", False, "chebyshev", False),
            ("mixed_learned", "mixed", "learned", False, "chebyshev", False),
            ("fp64_zero_guess_reuse_unchanged", "fp64", "zero", True, "chebyshev", False),
            ("mixed_learned_reuse_unchanged", "mixed", "learned", True, "chebyshev", False))
    for name, prec, guess, reuse, smoother, tune in legs:
        rec = run_leg(ppe, torch, wl, d_in, steps, warm, prec, guess=guess, net=net, reuse=reuse,
                      smoother=smoother, autotune=tune)
        out[name] = leg_summary(rec, K, base)
        note(f"plate {name}: {out[name]['value']:.1f} solves/s, "
             f"{out[name]['pcg_iterations_per_solve']:.1f} iterations")
        del rec
    # changed masks keep the coarse levels of the last full setup (at most
    # eight assemblies in a row, active set within 10 % of that build's)
    for name, prec, guess in (("fp64_zero_guess_coarse_reuse", "fp64", "zero"),
                              ("fp64_previous_guess_coarse_reuse", "fp64", "prev"),
                              ("mixed_previous_guess_coarse_reuse", "mixed", "prev"),
                              ("mixed_learned_coarse_reuse", "mixed", "learned")):
        rec = run_leg(ppe, torch, wl, d_in, steps, warm, prec, guess=guess, net=net, reuse=True,
                      coarse_reuse=8)
        out[name] = leg_summary(rec, K, base)
        note(f"plate {name}: {out[name]['value']:.1f} solves/s, "
             f"{out[name]['pcg_iterations_per_solve']:.1f} iterations")
        del rec
    return out


def c3_leg(ppe, torch, dev, reps=4):
    """One 128^3 system (random planar front): assembly + solve repeated."""
    from synth import box_mesh, face_coeff, fl_planar_front, rhs_uniform

    m = box_mesh((128, 128, 128), jitter=0.1, seed=0)
    fh = fl_planar_front(m.cell_centre, seed=2)
    c = torch.as_tensor(face_coeff(m, RHO), device=dev)
    f = torch.as_tensor(fh, device=dev)
    b = torch.as_tensor(rhs_uniform(m.n_cells, seed=1, center_mask=fh > 0), device=dev)
    owner = torch.as_tensor(m.owner, device=dev)
    neigh = torch.as_tensor(m.neigh, device=dev)
    out = {"workload": "128^3 jittered cube, planar front (normal seed 2), uniform RHS; "
                       f"{reps} timed assembly + solve rounds of one system after one untimed; "
                       "fixed launch rules"}
    for prec in ("fp64", "mixed"):
        s = ppe.Solver(precision=prec)
        s.set_mesh(m.n_cells, owner, neigh)
        p = torch.zeros(m.n_cells, dtype=torch.float64, device=dev)

        def rnd():
            s.assemble(c, f)
            return s.solve(b, out=p)

        rnd()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        setup = solve = 0.0
        for _ in range(reps):
            r = rnd()
            setup += r.stats["setup_ms"]
            solve += r.stats["solve_ms"]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        assert r.stats["rel_residual"] <= 1e-10
        na, it = r.stats["n_active"], r.stats["iterations"]
        out[prec] = dict(solves_per_s=1.0 / dt, ms_per_solve=1e3 * dt, setup_ms=setup / reps,
                         solve_ms=solve / reps, solve_only_per_s=1e3 / (solve / reps),
                         pcg_iterations=it, active_cells=na, levels=r.stats["levels"],
                         op_complexity=r.stats["op_complexity"],
                         dof_iterations_per_s=na * it / dt, rel_residual=r.stats["rel_residual"],
                         roofline=roofline(profile_table(s, lambda: [s.solve(b, out=p)
                                                                     for _ in range(2)]),
                                           f"128cube_planar_front_{prec}"))
        s.close()
    return out


def c4_leg(ppe, torch, dev, n_samples=256, steps=5, warm=1, first=10):
    """Batched uncertainty samples (sides U{24..48}) on the 50-step schedule:
    per timestep, one assembly and one segmented solve of all samples."""
    import numpy as np

    from synth import batch_samples, box_mesh, concat_meshes, face_coeff, rhs_uniform, uq_front_fl

    samples = batch_samples(n_samples)
    meshes = [box_mesh((sm["side"],) * 3, lengths=(CAVITY,) * 3, jitter=0.1, seed=q)
              for q, sm in enumerate(samples)]
    u = concat_meshes(meshes)
    c = torch.as_tensor(face_coeff(u, RHO), device=dev)
    s = ppe.Solver(precision="mixed")
    s.set_mesh(u.n_cells, torch.as_tensor(u.owner, device=dev), torch.as_tensor(u.neigh, device=dev))
    s.set_segments(u.extra["cell_offsets"])
    ks = list(range(first, first + warm + steps))
    data = {}
    for k in ks:
        fls = [uq_front_fl(mm.cell_centre, sm, (k + 1) * DT, 50 * DT, length=CAVITY)
               for mm, sm in zip(meshes, samples)]
        bs = [rhs_uniform(mm.n_cells, seed=1000 * q + k, center_mask=f > 0)
              for q, (mm, f) in enumerate(zip(meshes, fls))]
        data[k] = (torch.as_tensor(np.concatenate(fls), device=dev),
                   torch.as_tensor(np.concatenate(bs), device=dev))
    out = torch.zeros(u.n_cells, dtype=torch.float64, device=dev)
    its, worst, n_act = [], 0.0, []
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
            n_act.append(r.stats["n_active"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert worst <= 1e-10
    k_last = ks[-1]
    table = profile_table(s, lambda: s.solve(data[k_last][1], out=out))
    return dict(workload=f"{n_samples} uncertainty samples, cube sides U{{24..48}} (seed 3), "
                         f"T_melt ~ N(950,10), T_wall ~ N(600,20), dT_liq ~ U(-5,5); timesteps "
                         f"{ks[warm]}..{ks[-1]} of the 50-step schedule after {warm} warmup; one "
                         "assembly + one batched solve of every sample per step, mixed precision, "
                         "graph-replayed PCG iterations",
                value=n_samples * steps / dt, unit="sample-solves/s", samples=n_samples,
                cells=u.n_cells, mean_active_cells=float(np.mean(n_act)), steps=steps,
                ms_per_step=1e3 * dt / steps,
                mean_sample_iterations=float(np.mean(its)), worst_rel_residual=worst,
                precision="mixed", roofline=roofline(table, "c4_batch"))


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




def fractional_step_leg(ppe, torch, dev, n_steps=200, dt=1e-3, warm=3, krylov="bicgstab"):
    """The 64^3 cavity as a whole solidification run (section 2.2 steps 1-4):
    a 10 mm cube of an aluminium alloy (rho 2400, k 150, c_p 900, latent heat
    3.9e5, liquidus 913 K, solidus 833 K) melted at 950 K with every wall held
    at 600 K, natural convection on, n_steps fractional steps of dt from the
    uniform melt, all timed; the state stays on the device.  A few untimed
    steps from the same initial state first warm the driver's buffers."""
    import numpy as np

    from synth import al_alloy, box_mesh

    m = box_mesh((64, 64, 64), lengths=(CAVITY,) * 3, jitter=0.1, seed=0)
    props = al_alloy(T_wall=600.0, T_ref=950.0)

    def dev_t(a, dt_):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt_, device=dev)

    fw = ppe.Flow(krylov=krylov)
    fw.set_mesh(dev_t(m.owner, torch.int32), dev_t(m.neigh, torch.int32),
                dev_t(m.nodes, torch.float64), dev_t(m.extra["face_nodes"], torch.int32),
                dev_t(m.extra["cell_nodes"], torch.int32), dev_t(m.cell_centre, torch.float64),
                dev_t(m.face_area, torch.float64), dev_t(m.face_centre, torch.float64),
                dev_t(m.cell_volume, torch.float64))
    T0 = dev_t(np.full(m.n_cells, 950.0), torch.float64)
    st = fw.new_state(T0.clone(), props=props)
    for _ in range(warm):
        fw.step(props, st, dt)
    st = fw.new_state(T0.clone(), props=props)
    torch.cuda.synchronize()
    keys = ("picard", "momentum_iterations", "pressure_outer", "pressure_iterations",
            "energy_iterations", "momentum_ms", "pressure_ms", "energy_ms")
    acc = dict.fromkeys(keys, 0.0)
    picard, solid, unconverged = [], [], 0
    t0 = time.perf_counter()
    for _ in range(n_steps):
        status, stt = fw.step(props, st, dt, allow_not_converged=True)
        unconverged += int(status != 0)
        picard.append(stt["picard"])
        solid.append(stt["n_solid"])
        for q in keys:
            acc[q] += stt[q]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    K = n_steps
    return {
        "workload": f"64^3 jittered hex cube (10 mm), aluminium alloy (rho 2400, k 150, c_p 900, "
                    "L 3.9e5, liquidus 913 K, solidus 833 K) melted at 950 K, walls at 600 K, "
                    f"natural convection; {K} fractional steps of {dt:g} s from the uniform melt "
                    f"(alpha dt / h^2 = 2.8): momentum predictor (3 AMG-PCG solves of a shifted "
                    f"system) + masked cross-diffusion projection ({krylov}) + energy Picard loop "
                    "(branch-limited passes), FP64",
        "steps_per_s": K / el,
        "ms_per_step": 1e3 * el / K,
        "pressure_projections_per_s": 1e3 * K / acc["pressure_ms"],
        "cells": m.n_cells,
        "solid_cells_at_steps_1_50_100_200": [int(solid[i]) for i in (0, 49, 99, K - 1)
                                              if i < K],
        "picard_mean": float(np.mean(picard)), "picard_max": int(max(picard)),
        "unconverged_steps": unconverged,
        **{f"{q}_per_step": acc[q] / K for q in keys},
    }


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


def c2_legs(ppe, torch, dev, K, W):
    """The 64^3 timesteps (one GPU's share of a 128^3 mesh split eight ways):
    FP64, mixed, and mixed with a network trained on that run's earlier
    timesteps."""
    wl = cube_workload(64)
    steps = list(range(C2_FIRST, C2_FIRST + K))
    warm = list(range(C2_FIRST - W, C2_FIRST))
    d_in = wl.to_device(torch, dev, warm + steps + list(C2_TRAIN))
    base = run_leg(ppe, torch, wl, d_in, steps, warm, "fp64")
    out = {"workload": f"64^3 jittered hex cube (10 mm), sqrt(t) front from the wall x = 0, "
                       f"timesteps {steps[0]}..{steps[-1]} of 200 x 1e-3 s; assembly + setup + "
                       "solve per step; fixed launch rules",
           "fp64_zero_guess": leg_summary(base, K)}
    mixed = run_leg(ppe, torch, wl, d_in, steps, warm, "mixed")
    out["mixed_zero_guess"] = leg_summary(mixed, K, base)
    net, mu, sigma, tr = train_network(ppe, torch, wl, d_in, list(C2_TRAIN))
    ml = run_leg(ppe, torch, wl, d_in, steps, warm, "mixed", guess="learned",
                 net=(net, mu, sigma))
    out["mixed_learned"] = dict(leg_summary(ml, K, base), training=tr)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="time the headline leg only")
    ap.add_argument("--only", default="",
                    help="comma list of variant legs to run: c5, c3, c4, c2, projection, flow, "
                         "collocation (default: all)")
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

    dev = torch.device("cuda", 0)
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    copy_bandwidth(torch, dev)
    note(f"plain copy: {COPY['gbs']:.0f} GB/s")
    if args.c3_only:
        print(json.dumps(c3_leg(ppe, torch, dev)), flush=True)
        return
    only = {x for x in args.only.split(",") if x}
    want = lambda leg: not args.no_variants and (not only or leg in only)

    K, W = args.steps, args.warmup
    steps = list(range(C5_FIRST, C5_FIRST + K))
    warm = list(range(C5_FIRST - W, C5_FIRST))
    wl = plate_workload()
    need = warm + steps + (list(C5_TRAIN) if want("c5") else [])
    d_in = wl.to_device(torch, dev, need)
    note(f"inputs ready: {len(set(need))} timesteps of {wl.m.n_cells} cells")

    base = run_leg(ppe, torch, wl, d_in, steps, warm, "fp64")
    note(f"fp64 headline: {K / base['elapsed']:.1f} solves/s")
    n_act = base["n_act"]
    it = base["iters"] / K
    out = {
        "metric": METRIC,
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
            "workload": f"plate with ribs, {wl.m.n_cells} jittered hex cells (240x144x36 plate + "
                        "4 ribs of 8x144x56), front rising from the bottom face, timesteps "
                        f"{steps[0]}..{steps[-1]} of 200 x 1e-3 s; one masked SA-AMG-PCG pressure "
                        "solve per step (assembly + setup + solve), FP64, zero guess",
            "cells": wl.m.n_cells,
            "mean_active_cells": float(np.mean(n_act)),
            "pcg_iterations_per_solve": it,
            "dof_iterations_per_s": float(np.sum(n_act)) * it / base["elapsed"],
            "worst_rel_residual": base["worst"],
            "setup_ms_per_step": base["setup_ms"] / K,
            "solve_ms_per_step": base["solve_ms"] / K,
            "solve_only_per_s": 1e3 * K / base["solve_ms"],
            "algorithmic_gb_per_pcg_iteration": float(np.mean(base["bytes_iter"])) / 1e9,
        },
    }
    if not args.no_profile:
        s = base["solver"]
        out["roofline"] = roofline(profile_table(s, base["rerun"]), "plate_timesteps_fp64")
        note(f"roofline: {out['roofline']['kernel']} {out['roofline']['frac']:.3f}")
    base["solver"].close()
    if not args.no_variants:
        variants = {}
        if want("c5"):
            net, mu, sigma, tr = train_network(ppe, torch, wl, d_in, list(C5_TRAIN))
            note(f"network trained on the plate run: {tr}")
            variants["c5_plate"] = c5_legs(ppe, torch, wl, d_in, K, W, base, (net, mu, sigma))
            variants["c5_plate"]["mixed_learned"]["training"] = tr
        del d_in
        torch.cuda.empty_cache()
        if want("c3"):
            variants["c3_128cube"] = c3_leg(ppe, torch, dev)
            note("128^3 leg done")
        if want("c4"):
            variants["c4_uq_batched"] = c4_leg(ppe, torch, dev)
            note("batched uncertainty leg done")
        if want("c2"):
            variants["c2_64cube"] = c2_legs(ppe, torch, dev, K, W)
            note("64^3 legs done")
        if want("projection") or want("flow"):
            wl2 = cube_workload(64)
            st2 = list(range(C2_FIRST, C2_FIRST + K))
            wa2 = list(range(C2_FIRST - W, C2_FIRST))
            d2 = wl2.to_device(torch, dev, wa2 + st2)
            b2 = run_leg(ppe, torch, wl2, d2, st2, wa2, "fp64")
            if want("projection"):
                variants["projection_cross_diffusion"] = projection_leg(ppe, torch, wl2, d2, st2,
                                                                        wa2, dev, b2)
                variants["projection_cross_diffusion_deferred"] = projection_leg(
                    ppe, torch, wl2, d2, st2, wa2, dev, b2, "deferred")
                note("projection legs done")
            if want("flow"):
                variants["c2_fractional_step"] = fractional_step_leg(ppe, torch, dev)
                note("fractional-step leg done")
        if want("collocation"):
            variants["uq_collocation"] = uq_collocation(ppe, torch, dev)
            note("collocation leg done")
        out["variants"] = variants
    if not args.no_cpu_baseline:
        note("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(wl, steps[0], base["first_iters"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
