#!/usr/bin/env python
"""Throughput of the QSA particle-in-cell hot path on one MI355X.

A step is one beam step of the 3D workload 256 x 256 x 512 (dx = dy = dxi =
0.05 c/omega_p, warm plasma u_th = 0.01, 2x2 plasma lattice, electron beam
alpha = 1e-2, gamma_b = 1e3, 8 particles per cell): the beam source deposit,
the full quasistatic sweep over 512 slices (K = 3 predictor-corrector
iterations) and the Boris push of all 2.68e8 beam particles.  The metric is
plasma particle-slice updates per second over whole steps.  Beam steps run
--pipeline at a time in flight (lane k of a group sweeps 8 slices behind lane
k - 1 in the same launches); the results equal those of one step at a time.

Prints one JSON line (rank 0) with the measured rate, a roofline entry for
the dominant kernel (timed with HIP events on the library's stream inside
the timed region), the float64 oracle timed on a bounded sample of the
same workload on the host cores, and the adjoint/forward time of the
gradient workload (128 x 128 x 256, float32, 20 beam steps, 64 bins).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_push_pred_cube256_f64.json")
KERNEL_SOURCES = ("paper_2607_24214_amd/csrc/qsa_kernels.h", "paper_2607_24214_amd/csrc/qsa_device.h")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, precision: str, pipeline: int):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE record, if it was taken on the same
    kernel sources and configuration; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if (rec.get("source_sha256") != kernel_source_hash() or rec.get("workload") != workload
            or rec.get("precision") != precision or rec.get("steps_in_flight") != pipeline):
        return None
    return rec.get("hbm_bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def alg_bytes(kclass: str, wl, rsize: int) -> float:
    """Algorithmic HBM bytes of one launch of a kernel class: every array the
    kernel must touch, read or written once (particle state of rsize-byte
    components, nx*ny grids)."""
    npl = wl.n_plasma
    ng = wl.nx * wl.ny
    R = rsize
    if kclass == "push_pred":     # read x,y,ux,uy; read F^j and F^{j+1/2} (6+6), psi extrapolated; write 2 deposits
        return 4 * R * npl + (13 + 2) * R * ng
    if kclass == "push_final":    # read and write x,y,ux,uy; read F^j and F^{j+1/2}
        return 8 * R * npl + 12 * R * ng
    if kclass == "dep_S":
        return 2 * R * npl + R * ng
    if kclass == "dep_J":
        return 4 * R * npl + 4 * R * ng
    if kclass == "beam_push":     # read and write 6 real components + xi (float64)
        return 2 * (6 * R + 8) * wl.n_beam_total + 6 * R * wl.nxi * ng
    if kclass == "beam_deposit":
        return (6 * R + 8) * wl.n_beam_total + 4 * R * wl.nxi * ng
    raise KeyError(kclass)


def timed_step(sim, kclass: str, n: int):
    """Run n beam steps with every launch of kclass bracketed by HIP events on
    the library's work stream (direct launches); -> (summed ms, launches)."""
    sim.timing_begin(kclass)
    sim.beam_step(n)
    return sim.timing_end()


def cpu_baseline(wl, n_slices: int):
    """The float64 oracle on the first n_slices slices of one sweep of the
    same workload (full transverse grid, beam restricted to those slices)."""
    import torch
    import qsa_workloads as W
    from oracle import qsa_pic as O
    sub = wl.with_(nxi=n_slices)
    g = O.Grid.of(sub)
    plasma = O.to_torch(W.plasma_template(sub))
    beams = [O.to_torch(b) for b in W.beam(sub)]
    t0 = time.perf_counter()
    src = O.beam_sources(g, beams, [s.Z for s in sub.species])
    O.slice_sweep(g, plasma, src, sub.n_corr, sub.kappa2)
    dt = time.perf_counter() - t0
    return {
        "value": sub.n_plasma * n_slices / dt,
        "unit": "plasma particle-slice updates/s",
        "cores": torch.get_num_threads(),
        "kind": "oracle",
        "sample": (f"first {n_slices} of {wl.nxi} slices of one sweep of {wl.name} "
                   f"({wl.nx}x{wl.ny} grid, {sub.n_plasma} plasma particles/slice, beam "
                   f"cells in those slices only), float64, beam sources included; {dt:.1f} s"),
    }


def adjoint_ratio(steps_in_flight: int):
    """adjoint/forward time on the adjoint workload (128 x 128 x 256, float32,
    20 beam steps, 64 xi bins, plasma checkpoints every 16 slices): the time
    of one qsa_adjoint_sweep (its checkpointed forward pass, the reverse
    pass and the bin gradient) over that of the forward alone (20 beam
    steps and the sweep of the last, steps in flight as in the main run).
    Each is timed on its second call (the first captures graphs and loads
    code)."""
    import numpy as np
    import torch
    import qsa_workloads as W
    import paper_2607_24214_amd as Q
    wl = W.adjoint128()
    steps = wl.steps
    plasma = W.plasma_template(wl)
    beams = W.beam(wl)
    bins = [b["bin"] for b in beams]
    amps = np.ones(wl.n_bins)
    sim = Q.Sim(Q.params_from_workload(wl, precision="f32", pipeline=steps_in_flight, adjoint_steps=steps))
    sim.load_plasma(plasma)
    fwd = []
    for _ in range(2):
        for k, b in enumerate(beams):
            sim.load_beam(k, b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.beam_step(steps)
        sim.slice_sweep()
        torch.cuda.synchronize()
        fwd.append(time.perf_counter() - t0)
    for k, b in enumerate(beams):
        sim.load_beam(k, b)
    adj = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss, grad = sim.adjoint_sweep(steps, amps, bins)
        torch.cuda.synchronize()
        adj.append(time.perf_counter() - t0)
    if not (math.isfinite(loss) and np.all(np.isfinite(grad))):
        raise RuntimeError("adjoint produced non-finite values")
    out = {
        "metric": "adjoint/forward time",
        "value": adj[-1] / fwd[-1],
        "higher_is_better": False,
        "adjoint_ms": 1e3 * adj[-1],
        "forward_ms": 1e3 * fwd[-1],
        "dtype": "f32",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "nxi": wl.nxi, "beam_steps": steps,
                   "bins": wl.n_bins, "checkpoint_every_slices": wl.ckpt_every, "n_corr": wl.n_corr,
                   "forward_steps_in_flight": sim.pipeline},
    }
    del sim
    torch.cuda.empty_cache()
    return out


def scan_rate(n_inst: int, steps: int, warmup: int):
    """Batched parameter scan (float32): the first n_inst instances of the
    64-instance scan (the scan shards by instance: 32 are one GPU's share of
    two) advanced together, one launch per phase and slice for all of them;
    a step is every instance's beam deposit, sweep and beam push."""
    import torch
    import qsa_workloads as W
    import paper_2607_24214_amd as Q
    wls = W.scan_instances()[:n_inst]
    t = time.perf_counter()
    sims = []
    for wl in wls:
        sim = Q.Sim(Q.params_from_workload(wl, precision="f32", pipeline=1))
        sim.load_plasma(W.plasma_template(wl))
        for k, b in enumerate(W.beam(wl)):
            sim.load_beam(k, b)
        sims.append(sim)
    log(f"scan: {n_inst} instances loaded in {time.perf_counter() - t:.1f} s")
    batch = Q.Batch(sims)
    batch.step(warmup)
    batch.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    batch.sync()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    updates = sum(wl.n_plasma * wl.nxi for wl in wls) * steps
    out = {
        "metric": "plasma particle-slice updates/s (push+deposit+solve), batched scan",
        "value": updates / T,
        "unit": "plasma particle-slice updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * T / steps,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic (seeded PCG64 plasma lattice + flat-top beam)",
        "config": {"workload": f"scan of {n_inst} of 64 instances", "instances": n_inst,
                   "plasma_updates_per_step": updates // steps,
                   "beam_particles": sum(wl.n_beam_total for wl in wls),
                   "grids": sorted({(wl.nx, wl.ny) for wl in wls}),
                   "nxi": sorted({wl.nxi for wl in wls})},
    }
    batch.close()
    return out


def diagnostics_rate(sim, wl, rsize):
    """Device diagnostics of the last sweep (windows of 2 c/omega_p): the
    field-moment reduction reads six stored field planes once, the beam
    moments each beam particle's xi, u and w once; wall time per call
    (launches and the call's own synchronization included), against
    copying the same six fields of every slice to the host."""
    import torch
    ws = max(1, int(round(2.0 / wl.dxi)))
    sim.field_moments(ws, on_device=True)
    sim.beam_moments(0, ws, on_device=True)
    reps = 5
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        sim.field_moments(ws, on_device=True)
    tf = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for _ in range(reps):
        sim.beam_moments(0, ws, on_device=True)
    tb = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for name in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        sim.fields(name)
    th = time.perf_counter() - t
    bf = 6 * wl.nxi * wl.nx * wl.ny * rsize
    bb = wl.n_beam_total * (8 + 4 * rsize)
    return {"window_slices": ws,
            "field_moments_ms": 1e3 * tf, "field_moments_GB_s": bf / tf / 1e9,
            "field_moments_frac_hbm": bf / tf / 1e9 / HBM_PEAK_GBS,
            "beam_moments_ms": 1e3 * tb, "beam_moments_GB_s": bb / tb / 1e9,
            "host_copy_of_the_six_fields_ms": 1e3 * th,
            "timing": "wall clock per synchronizing call, 5 calls each, after one untimed call"}


def linear_model_scan():
    """A growth-rate scan for the linear model (Eq. 5): 64 instances (Gamma
    spread over a factor 4 around Gamma0 = 0.05 omega_p, random seeds), xi in
    [0, 40] at 0.02 (2001 points), RK4 with Gamma0 dtau = 0.01 up to
    Gamma0 tau = 8 (800 steps), outputs at every Gamma0 tau = 0.5."""
    import numpy as np
    rng = np.random.default_rng(11)
    n_inst, g0 = 64, 0.05
    gam = g0 * np.exp(rng.uniform(np.log(0.5), np.log(2.0), n_inst))
    xi = np.arange(2001) * 0.02
    seeds = rng.uniform(-1.0, 1.0, (n_inst, xi.size))
    return gam, xi, seeds, 0.01 / g0, np.arange(0, 17) * 0.5 / g0


def linear_model_rate():
    """The batched solver on linear_model_scan(): wall time of the
    synchronized launch."""
    import torch
    import paper_2607_24214_amd as Q
    gam, xi, seeds, dtau, taus = linear_model_scan()
    n_inst = gam.size
    Q.linear_model(gam, seeds, 0.02, taus[:2], dtau)      # first launch
    torch.cuda.synchronize()
    t = time.perf_counter()
    Q.linear_model(gam, seeds, 0.02, taus, dtau)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t
    steps = int(round(taus[-1] / dtau))
    work = n_inst * xi.size * steps
    return {"instances": n_inst, "xi_points": int(xi.size), "rk4_steps": steps, "ms": 1e3 * tg,
            "point_steps_per_s": work / tg}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--pipeline", type=int, default=8, help="beam steps in flight (1 = one at a time)")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time its launch shapes and steps in flight first")
    ap.add_argument("--pre-steps", type=int, default=0,
                    help="untimed beam steps after the warmup (time a more evolved beam)")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--col-threads", type=int, default=0,
                    help="threads per column transform (16, 32, 64; 0 = the library's default)")
    ap.add_argument("--workload", default="cube256")
    ap.add_argument("--cpu-slices", type=int, default=96)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graphs", action="store_true",
                    help="enqueue every launch instead of replaying HIP graphs (for counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 2 GiB three times (scale for HBM counters)")
    ap.add_argument("--breakdown", action="store_true",
                    help="also time every kernel class over one extra group of steps each")
    ap.add_argument("--no-linear-model", action="store_true",
                    help="skip the linear-model solver measurement")
    ap.add_argument("--no-diagnostics", action="store_true",
                    help="skip the device diagnostics measurement")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward time of the 128x128x256 adjoint workload")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only measure the adjoint/forward time (its own JSON line)")
    ap.add_argument("--scan", type=int, default=0,
                    help="only measure batched steps of the first N scan instances (its own JSON line)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the slice sweep runs on a single MI355X; "
              "running on several GPUs is not implemented (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": a.numel() * 8, "launches": 3}), flush=True)
        return
    import qsa_workloads as W
    import paper_2607_24214_amd as Q

    if args.scan:
        print(json.dumps(scan_rate(args.scan, args.steps, args.warmup)), flush=True)
        return
    if args.adjoint_only:
        adj = adjoint_ratio(args.pipeline)
        print(json.dumps(dict(adj, n_gpus=1, data="synthetic (seeded PCG64 plasma lattice + flat-top beam)")),
              flush=True)
        return
    wl = W.CONFIGS[args.workload]().with_(precision=args.precision)
    rsize = 8 if args.precision == "f64" else 4
    log(f"workload {wl.name}: {wl.nx}x{wl.ny}x{wl.nxi}, plasma {wl.n_plasma}/slice, "
        f"beam {wl.n_beam_total}, precision {args.precision}")

    t = time.perf_counter()
    plasma = W.plasma_template(wl)
    beams = W.beam(wl)
    log(f"inputs generated in {time.perf_counter() - t:.1f} s")
    sim = Q.Sim(Q.params_from_workload(wl, precision=args.precision, pipeline=args.pipeline))
    sim.load_plasma(plasma)
    for s, b in enumerate(beams):
        sim.load_beam(s, b)
    del beams
    if args.no_graphs:
        sim.set_graphs(False)
    if args.col_threads:
        sim.set_shapes(0, 0, args.col_threads)
    tuned = None
    if args.autotune:
        t = time.perf_counter()
        best = sim.autotune()
        nt, rt, ct = sim.shapes()
        tuned = {"plasma_threads": nt, "row_threads": rt, "column_threads": ct, "steps_in_flight": sim.pipeline,
                 "best_trial_ms_per_step": best}
        log(f"autotune {time.perf_counter() - t:.1f} s: {tuned}")
    log(f"loaded; workspace {sim.ws_bytes / 2**30:.2f} GiB")

    # warmup
    t = time.perf_counter()
    sim.beam_step(args.warmup)
    sim.sync()
    log(f"warmup {args.warmup} steps: {time.perf_counter() - t:.2f} s")
    if args.pre_steps:
        t = time.perf_counter()
        sim.beam_step(args.pre_steps)
        sim.sync()
        log(f"{args.pre_steps} further untimed steps: {time.perf_counter() - t:.2f} s")

    dominant = "push_pred"
    # the step graphs (a whole group when pipelined) are captured here,
    # outside the timed region
    depth = sim.pipeline
    sim.beam_step(depth)
    sim.sync()
    # timed region: exactly K steps (groups of steps in flight) between synchronizations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.beam_step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if sim.pipeline != depth:
        raise RuntimeError(f"pipelining fell back to depth {sim.pipeline}")
    # the dominant kernel's launch duration: HIP events around each of its
    # launches over the same number of steps, enqueued launch by launch
    dom_ms, dom_n = timed_step(sim, dominant, args.steps)
    timing_note = ("HIP events recorded at the start and end of every launch of the kernel "
                   "(hipExtLaunchKernelGGL on the library's work stream), over "
                   f"{args.steps} steps enqueued launch by launch right after the timed region")
    T = t1 - t0
    ms_step = 1e3 * T / args.steps
    updates = wl.n_plasma * wl.nxi * args.steps
    value = updates / T
    log(f"timed {args.steps} steps: {T:.3f} s, {ms_step:.2f} ms/step, {value:.3e} updates/s")

    # sweep alone (the beam push excluded), for the record: graph captured
    # by the first call, the second is timed
    sim.slice_sweep()
    sim.sync()
    torch.cuda.synchronize()
    t = time.perf_counter()
    sim.slice_sweep()
    torch.cuda.synchronize()
    t_sweep = time.perf_counter() - t

    diag = None
    if not args.no_diagnostics:
        diag = diagnostics_rate(sim, wl, rsize)
        log(f"diagnostics: field moments {diag['field_moments_ms']:.3f} ms "
            f"({diag['field_moments_GB_s']:.0f} GB/s), beam moments {diag['beam_moments_ms']:.3f} ms, "
            f"host copy of the fields {diag['host_copy_of_the_six_fields_ms']:.0f} ms")

    # per-class times over further groups of steps (after the timed region,
    # which they would otherwise move to a later, more evolved beam)
    breakdown = {}
    if args.breakdown:
        for kc in ("push_pred", "push_final", "dep_S", "dep_J", "row_r2c", "col", "row_c2r",
                   "beam_deposit", "beam_push"):
            nst = depth
            ms, n = timed_step(sim, kc, nst)
            breakdown[kc] = {"ms_per_step": ms / nst, "launches": n, "us_per_launch": 1e3 * ms / max(n, 1)}
            log(f"  {kc:13s} {ms / nst:9.2f} ms/step  {n:6d} launches  {1e3 * ms / max(n, 1):8.2f} us/launch")

    avg_s = dom_ms / 1e3 / max(dom_n, 1)
    # one launch advances every step in flight by a slice: algorithmic bytes
    # per launch = per-slice bytes x lane-slices the launches covered / launches
    lane_slices = args.steps * wl.nxi * wl.n_corr
    per_launch = alg_bytes(dominant, wl, rsize) * lane_slices / max(dom_n, 1)
    achieved = per_launch / avg_s / 1e9
    roofline = {
        "kernel": (f"k_plasma_rows<{'double' if rsize == 8 else 'float'}, 2> (predictor: plasma RK2 push "
                   "+ predicted J_perp deposit)"),
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": measured_traffic(wl.name, args.precision, depth) if not tuned else None,
        "avg_launch_us": avg_s * 1e6, "launches_timed": dom_n,
        "timing": timing_note,
        "alg_bytes_per_launch": per_launch,
        "slices_per_launch": lane_slices / max(dom_n, 1),
    }
    linear = None
    if not args.no_linear_model:
        linear = linear_model_rate()
        log(f"linear model: {linear['instances']} instances x {linear['xi_points']} points x "
            f"{linear['rk4_steps']} RK4 steps in {linear['ms']:.1f} ms")
    adjoint = None
    if not args.no_adjoint:
        del sim
        torch.cuda.empty_cache()
        log("adjoint workload ...")
        adjoint = adjoint_ratio(depth)
        log(f"adjoint {adjoint['adjoint_ms']:.0f} ms / forward {adjoint['forward_ms']:.0f} ms "
            f"= {adjoint['value']:.2f}")
    cpu = None
    if not args.no_cpu_baseline:
        log(f"oracle baseline on {args.cpu_slices} slices ...")
        cpu = cpu_baseline(wl, args.cpu_slices)
        log(f"oracle: {cpu['value']:.3e} updates/s on {cpu['cores']} threads")
        if linear is not None:
            # the oracle's solver of the linear model on one instance of the scan
            from oracle import linear_theory as LT
            gam, xi, seeds, dtau, taus = linear_model_scan()
            t = time.perf_counter()
            LT.solve_eq5(float(gam[0]), xi, seeds[0], taus, dtau)
            to = time.perf_counter() - t
            cpu["linear_model"] = {"one_instance_ms": 1e3 * to,
                                   "point_steps_per_s": xi.size * int(round(taus[-1] / dtau)) / to}

    out = {
        "metric": "plasma particle-slice updates/s (push+deposit+solve)",
        "value": value,
        "unit": "plasma particle-slice updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic (seeded PCG64 plasma lattice + flat-top beam)",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "nxi": wl.nxi,
                   "dx": wl.dx, "plasma_per_slice": wl.n_plasma, "beam_particles": wl.n_beam_total,
                   "alpha": wl.species[0].alpha, "gamma_b": wl.gamma_b, "n_corr": wl.n_corr,
                   "steps_in_flight": depth, "autotuned": tuned,
                   "step": "beam source deposit + 512-slice sweep + Boris beam push"},
        "sweep_only": {"ms": 1e3 * t_sweep, "updates_per_s": wl.n_plasma * wl.nxi / t_sweep},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "adjoint": adjoint,
        "diagnostics": diag,
        "linear_model": linear,
    }
    if breakdown:
        out["kernel_breakdown_ms_per_step"] = {k: round(v["ms_per_step"], 3) for k, v in breakdown.items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
