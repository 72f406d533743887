#!/usr/bin/env python
"""Throughput of the QSA particle-in-cell hot path on one MI355X.

The headline workload is the dilute pair beam 512 x 512 x 2048 (dx = dy =
dxi = 0.1 c/omega_p, warm plasma u_th = 1e-3, 2x2 plasma lattice, electron
and positron beams alpha = 1e-4 each, gamma_b = 1e4, 4 particles per cell
per species, u_perp ~ N(0, 1), float32): the largest workload one GPU holds.
A step is one beam step: the beam source deposit of its 4.29e9 particles,
the quasistatic sweep over 2048 slices (K = 3 predictor-corrector
iterations) and the Boris push.  The metric is plasma particle-slice
updates per second over whole steps.  A second copy of its 128 GiB beam
does not fit, so it runs as many beam steps in flight as the device's memory
holds on a lean pipeline that keeps no copy (5; lane k of a group sweeps 8
slices behind lane k - 1 in the same launches).

The 3D workload 256 x 256 x 512 (float64 and float32, 8 beam steps in
flight), the 64 x 128 slab and the 64-instance batched scan are timed too,
as extra entries.

Prints one JSON line with the measured rate, a roofline entry for the
dominant kernel (timed with HIP events on the library's stream) and the
whole path's fraction of the HBM roofline, the float64 oracle timed on a
bounded sample of the same workload on the host cores (and on one core),
and the adjoint/forward time of the gradient workload (128 x 128 x 256,
float32, 20 beam steps, 64 bins).
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# one step at a time, the beam storage is re-sorted by deposit key every this
# many steps (pair 512^2 x 2048 in float32: 1059.5 ms/step never, 1034.0 every
# 4 or 3, 1042.9 every 2, over 10 steps after 2 of warm-up)
RESORT_EVERY = 4
TRAFFIC_FILES = tuple(os.path.join(ROOT, "profiles", f"traffic_push_pred_{w}.json")
                      for w in ("pair512_f32", "cube256_f64", "cube256_f32"))
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
    for f in TRAFFIC_FILES:
        try:
            with open(f) as fh:
                rec = json.load(fh)
        except (OSError, ValueError):
            continue
        if (rec.get("source_sha256") == kernel_source_hash() and rec.get("workload") == workload
                and rec.get("precision") == precision and rec.get("steps_in_flight") == pipeline):
            return rec.get("hbm_bytes_per_launch")
    return None


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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample(wl, n_slices: int):
    """The float64 oracle on the first n_slices slices of one sweep of the
    workload (full transverse grid, beam restricted to those slices);
    -> (seconds, updates)."""
    import qsa_workloads as W
    from oracle import qsa_pic as O
    sub = wl.with_(nxi=n_slices)
    g = O.Grid.of(sub)
    plasma = O.to_torch(W.plasma_template(sub))
    beams = [O.to_torch(b) for b in W.beam(wl, 0, n_slices)]
    t0 = time.perf_counter()
    src = O.beam_sources(g, beams, [s.Z for s in sub.species])
    O.slice_sweep(g, plasma, src, sub.n_corr, sub.kappa2)
    return time.perf_counter() - t0, sub.n_plasma * n_slices


def cpu_baseline(wl, n_slices: int, n_slices_one_core: int):
    """The oracle timed on the host: on all the threads torch uses, and on
    one thread (the paper quotes its QS-PIC run on a single core)."""
    import torch
    dt, upd = _oracle_sample(wl, n_slices)
    threads = torch.get_num_threads()
    out = {
        "value": upd / dt,
        "unit": "plasma particle-slice updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"first {n_slices} of {wl.nxi} slices of one sweep of {wl.name} "
                   f"({wl.nx}x{wl.ny} grid, {wl.n_plasma} plasma particles/slice, beam "
                   f"cells in those slices only), float64, beam sources included; {dt:.1f} s"),
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
        "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
    }
    if n_slices_one_core > 0:
        torch.set_num_threads(1)
        try:
            d1, u1 = _oracle_sample(wl, n_slices_one_core)
        finally:
            torch.set_num_threads(threads)
        out["one_core"] = {"value": u1 / d1, "cores": 1,
                           "sample": f"first {n_slices_one_core} slices, the same way; {d1:.1f} s"}
    return out


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
    from concurrent.futures import ThreadPoolExecutor
    wls = W.scan_instances()[:n_inst]
    t = time.perf_counter()
    sims = [None] * len(wls)

    def make(i):
        # all 64 instances fit one GPU without the packed push fields
        return Q.Sim(Q.params_from_workload(wls[i], precision="f32", pipeline=1, field_pack=False))

    big = [i for i, wl in enumerate(wls) if wl.n_beam_total > 1 << 26]
    small = [i for i in range(len(wls)) if i not in big]
    for i in big:   # generated range by range on host threads
        sims[i] = make(i)
        sims[i].load_plasma(W.plasma_template(wls[i]))
        load_beam_in_ranges(sims[i], wls[i])
    nthr = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 8))
    with ThreadPoolExecutor(nthr) as ex:
        # instances generated on host threads a group at a time (bounded host memory)
        for g0 in range(0, len(small), nthr):
            grp = small[g0:g0 + nthr]
            data = list(ex.map(lambda i: (W.plasma_template(wls[i]), W.beam(wls[i])), grp))
            for i, (pl, beams) in zip(grp, data):
                sims[i] = make(i)
                sims[i].load_plasma(pl)
                for k, b in enumerate(beams):
                    sims[i].load_beam(k, b)
            del data
    torch.cuda.synchronize()
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
    nc = min(wl.nxi, 128)
    t = time.perf_counter()
    for name in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        sim.fields(name, 0, nc)
    th = (time.perf_counter() - t) * wl.nxi / nc
    bf = 6 * wl.nxi * wl.nx * wl.ny * rsize
    bb = wl.n_beam_total * (8 + 4 * rsize)
    return {"window_slices": ws,
            "field_moments_ms": 1e3 * tf, "field_moments_GB_s": bf / tf / 1e9,
            "field_moments_frac_hbm": bf / tf / 1e9 / HBM_PEAK_GBS,
            "beam_moments_ms": 1e3 * tb, "beam_moments_GB_s": bb / tb / 1e9,
            "host_copy_of_the_six_fields_ms": 1e3 * th,
            "timing": ("wall clock per synchronizing call, 5 calls each, after one untimed call; the host "
                       f"copy of the six fields timed on {nc} slices and scaled to {wl.nxi}")}


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


def dirichlet_rate(n_grid: int = 256, n: int = 511):
    """The conducting-wall solver on n_grid grids of n x n interior nodes in
    float32 (a batch of slices of a 512-class box): wall time of the
    synchronized three-launch solve, averaged over 5 after one untimed.
    Algorithmic bytes: the source read and the solution written once (8
    bytes per node); the three passes move each node's value through HBM
    three times (24 bytes)."""
    import torch
    import paper_2607_24214_amd as Q
    f = torch.randn((n_grid, n, n), dtype=torch.float32, device="cuda")
    u = torch.empty_like(f)
    Q.dirichlet_solve(f, 0.1, 0.1, 0.0, out=u)
    torch.cuda.synchronize()
    reps = 5
    t = time.perf_counter()
    for _ in range(reps):
        Q.dirichlet_solve(f, 0.1, 0.1, 0.0, out=u)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t) / reps
    nodes = n_grid * n * n
    return {"grids": n_grid, "nx": n, "ny": n, "dtype": "f32", "ms": ms, "grids_per_s": n_grid / (ms * 1e-3),
            "alg_GB_s": 8.0 * nodes / (ms * 1e-3) / 1e9, "moved_GB_s": 24.0 * nodes / (ms * 1e-3) / 1e9}


def b_alg(wl, rsize: int) -> float:
    """Algorithmic HBM bytes per plasma particle-slice update of the whole
    sweep: the particle state (x, y, u_x, u_y) read and written and its
    weight read once, plus the slice's grid I/O (4 beam source values read,
    6 field values written per cell) shared by the particles of a cell."""
    ppc = wl.plasma_ppc
    grid = (4 + 6) if wl.ny > 1 else (2 + 4)
    state = (5 + 4) if wl.ny > 1 else (3 + 2)
    return state * rsize + grid * rsize / ppc


# Floating-point operations per plasma particle-slice update of the sweep at
# K = 3, counted from the kernels (a division counted as one operation): the
# rho - J_z deposit 12, the J stage (psi gather, G, gamma, three deposits) 40,
# the first predictor pass (two stencils, twelve gathers, the RK2 step, the
# predicted psi and two deposits) 190, each later pass from the RK2 cache 105,
# the final advance 90; plus the spectral solves (about 21 real 2D
# transforms per slice at 2.5 N log2 N each) shared by the particles.
FLOP_PARTICLE = 12 + 40 + 190 + 2 * 105 + 90
FLOP_PEAK_TFS = {"f32": 157.3, "f64": 78.6}


def flop_per_update(wl) -> float:
    n = wl.nx * wl.ny
    fft = 21 * 2.5 * n * math.log2(n)
    return FLOP_PARTICLE + fft / wl.n_plasma


def load_beam_in_ranges(sim, wl, slices_per_range: int = 8):
    """Generate the beam range by range of slices on host threads (numpy
    releases the GIL while it draws and fills arrays) and hand each range to
    the library through a device staging buffer (qsa_load_beam_range), so
    the host never holds the whole beam.  Returns seconds."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import qsa_workloads as W
    nthr = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 8))
    t0 = time.perf_counter()
    keys = ("x", "y", "xi", "ux", "uy", "uz", "w")
    for s in range(len(wl.species)):
        ranges = [(j, min(j + slices_per_range, wl.beam_slices)) for j in range(0, wl.beam_slices, slices_per_range)]
        first = 0
        with ThreadPoolExecutor(nthr) as ex:
            futs = {}
            nxt = 0
            for i in range(len(ranges)):
                while nxt < len(ranges) and nxt < i + 2 * nthr:
                    futs[nxt] = ex.submit(W.beam_species, wl, s, *ranges[nxt])
                    nxt += 1
                b = futs.pop(i).result()
                dev = {k: torch.from_numpy(b[k]).to("cuda") for k in keys}
                sim.load_beam_range(s, first, dev)
                first += int(b["x"].size)
                del b, dev
    sim.sync()
    return time.perf_counter() - t0


def lean_depth(wl, precision: str, most: int = 5, spare_gib: float = 8.0) -> int:
    """Most beam steps in flight (up to `most`) of a lean pipeline (no second
    copy of the beam) whose workspace fits the device's free memory with
    `spare_gib` to spare; 1 (one step at a time) if none does."""
    import ctypes as C
    import torch
    import paper_2607_24214_amd as Q
    free, _ = torch.cuda.mem_get_info()
    lib = Q.lib()
    for n in range(most, 1, -1):
        p = Q.params_from_workload(wl, precision=precision, pipeline=n, lean_pipeline=True)
        need = lib.qsa_workspace_bytes(C.byref(p))
        if need and need + spare_gib * 2**30 <= free:
            return n
    return 1


def run_workload(wl, precision: str, pipeline: int, steps: int, warmup: int, args, with_extras: bool,
                 lean: bool = False):
    """Load a workload, warm up, time exactly `steps` beam steps; then the
    dominant kernel's launches with HIP events, the sweep alone and the
    diagnostics.  Returns the measurement dict."""
    import torch
    import qsa_workloads as W
    import paper_2607_24214_amd as Q
    rsize = 8 if precision == "f64" else 4
    log(f"workload {wl.name}: {wl.nx}x{wl.ny}x{wl.nxi}, plasma {wl.n_plasma}/slice, "
        f"beam {wl.n_beam_total}, precision {precision}, steps in flight {pipeline}")
    lean = pipeline > 1 and lean
    sim = Q.Sim(Q.params_from_workload(wl, precision=precision, pipeline=pipeline, lean_pipeline=lean))
    log(f"workspace {sim.ws_bytes / 2**30:.2f} GiB" + (" (lean pipeline: no second beam copy)" if lean else ""))
    t = time.perf_counter()
    sim.load_plasma(W.plasma_template(wl))
    if wl.n_beam_total > 1 << 28:
        tl = load_beam_in_ranges(sim, wl)
    else:
        for s, b in enumerate(W.beam(wl)):
            sim.load_beam(s, b)
        sim.sync()
        tl = time.perf_counter() - t
    log(f"inputs generated and loaded in {tl:.1f} s")
    if args.no_graphs:
        sim.set_graphs(False)
    if args.no_beside:
        sim.set_beam_beside(False)
    if args.beside_blocks is not None:
        sim.set_beside_blocks(args.beside_blocks)
    resort = (args.resort_every if args.resort_every is not None else RESORT_EVERY) if pipeline == 1 else 0
    if resort:
        sim.set_resort_every(resort)
    if args.col_threads or args.plasma_threads or args.row_threads:
        sim.set_shapes(args.plasma_threads, args.row_threads, args.col_threads)
    tuned = None
    if args.autotune:
        t = time.perf_counter()
        best = sim.autotune()
        nt, rt, ct = sim.shapes()
        tuned = {"plasma_threads": nt, "row_threads": rt, "column_threads": ct, "steps_in_flight": sim.pipeline,
                 "best_trial_ms_per_step": best}
        log(f"autotune {time.perf_counter() - t:.1f} s: {tuned}")
    # warmup (the first step captures the step graph, outside the timed region)
    t = time.perf_counter()
    sim.beam_step(max(warmup, 1))
    sim.sync()
    log(f"warmup {max(warmup, 1)} steps: {time.perf_counter() - t:.2f} s")
    if args.pre_steps:
        t = time.perf_counter()
        sim.beam_step(args.pre_steps)
        sim.sync()
        log(f"{args.pre_steps} further untimed steps: {time.perf_counter() - t:.2f} s")
    depth = sim.pipeline
    # timed region: exactly `steps` beam steps between synchronizations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.beam_step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if sim.pipeline != depth:
        raise RuntimeError(f"pipelining fell back to depth {sim.pipeline}")
    T = t1 - t0
    ms_step = 1e3 * T / steps
    updates = wl.n_plasma * wl.nxi * steps
    value = updates / T
    log(f"timed {steps} steps: {T:.3f} s, {ms_step:.2f} ms/step, {value:.3e} updates/s")
    # the dominant kernel's launch duration: HIP events around each of its
    # launches over further steps, enqueued launch by launch
    dominant = "push_pred"
    n_ev = depth * max(1, min(steps, 16) // depth) if depth > 1 else min(steps, 4)
    dom_ms, dom_n = timed_step(sim, dominant, n_ev)
    timing_note = ("HIP events recorded at the start and end of every launch of the kernel "
                   "(hipExtLaunchKernelGGL on the library's work stream), over "
                   f"{n_ev} steps enqueued launch by launch right after the timed region")
    # the sweep alone (the beam push excluded)
    sim.slice_sweep()
    sim.sync()
    torch.cuda.synchronize()
    t = time.perf_counter()
    sim.slice_sweep()
    torch.cuda.synchronize()
    t_sweep = time.perf_counter() - t
    diag = None
    if with_extras and not args.no_diagnostics:
        diag = diagnostics_rate(sim, wl, rsize)
        log(f"diagnostics: field moments {diag['field_moments_ms']:.3f} ms "
            f"({diag['field_moments_GB_s']:.0f} GB/s), beam moments {diag['beam_moments_ms']:.3f} ms")
    breakdown = {}
    if args.breakdown and with_extras:
        for kc in ("push_pred", "push_final", "dep_S", "dep_J", "row_r2c", "col", "row_c2r",
                   "beam_deposit", "beam_push"):
            ms, n = timed_step(sim, kc, depth)
            breakdown[kc] = {"ms_per_step": ms / depth, "launches": n, "us_per_launch": 1e3 * ms / max(n, 1)}
            log(f"  {kc:13s} {ms / depth:9.2f} ms/step  {n:6d} launches  {1e3 * ms / max(n, 1):8.2f} us/launch")
    del sim
    gc.collect()
    torch.cuda.empty_cache()
    avg_s = dom_ms / 1e3 / max(dom_n, 1)
    # one launch advances every step in flight by a slice: algorithmic bytes
    # per launch = per-slice bytes x lane-slices the launches covered / launches
    lane_slices = n_ev * wl.nxi * wl.n_corr
    per_launch = alg_bytes(dominant, wl, rsize) * lane_slices / max(dom_n, 1)
    achieved = per_launch / avg_s / 1e9
    ba = b_alg(wl, rsize)
    path_gbs = value * ba / 1e9
    roofline = {
        "kernel": (f"k_plasma_rows<{'double' if rsize == 8 else 'float'}, 2> (predictor: plasma RK2 push "
                   "+ predicted J_perp deposit)"),
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": measured_traffic(wl.name, precision, depth) if not tuned else None,
        "avg_launch_us": avg_s * 1e6, "launches_timed": dom_n,
        "timing": timing_note,
        "alg_bytes_per_launch": per_launch,
        "slices_per_launch": lane_slices / max(dom_n, 1),
        "path_alg_bytes_per_update": ba,
        "path_achieved_GB_s": path_gbs,
        "path_frac": path_gbs / HBM_PEAK_GBS,
        "path_flop_per_update": flop_per_update(wl),
        "path_alu_frac": value * flop_per_update(wl) / (FLOP_PEAK_TFS[precision] * 1e12),
    }
    out = {"value": value, "ms_per_step": ms_step, "steps": steps, "warmup": warmup, "dtype": precision,
           "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "nxi": wl.nxi,
                      "dx": wl.dx, "plasma_per_slice": wl.n_plasma, "beam_particles": wl.n_beam_total,
                      "species": [{"Z": sp.Z, "alpha": sp.alpha, "ppc": sp.ppc} for sp in wl.species],
                      "gamma_b": wl.gamma_b, "n_corr": wl.n_corr, "steps_in_flight": depth, "autotuned": tuned,
                      "resort_every": resort, "lean_pipeline": lean,
                      "precision_note": ("float32 particle momenta, fields, spectra and beam state; plasma "
                                         "positions, beam xi and the LDS deposit tiles in float64"
                                         if precision == "f32" else "float64 throughout"),
                      "step": f"beam source deposit + {wl.nxi}-slice sweep + Boris beam push"},
           "sweep_only": {"ms": 1e3 * t_sweep, "updates_per_s": wl.n_plasma * wl.nxi / t_sweep},
           "roofline": roofline, "diagnostics": diag}
    if breakdown:
        out["kernel_breakdown_ms_per_step"] = {k: round(v["ms_per_step"], 3) for k, v in breakdown.items()}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="pair512", choices=sorted(["pair512", "cube256", "slab", "adjoint128"]))
    ap.add_argument("--precision", default=None, choices=["f64", "f32"],
                    help="default: the workload's (float32 for pair512, float64 for cube256)")
    ap.add_argument("--pipeline", type=int, default=None,
                    help="beam steps in flight (1 = one at a time; default for pair512: a lean pipeline as deep "
                         "as the device's memory allows, at most 5; 8 otherwise)")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time its launch shapes and steps in flight first")
    ap.add_argument("--pre-steps", type=int, default=0,
                    help="untimed beam steps after the warmup (time a more evolved beam)")
    ap.add_argument("--row-threads", type=int, default=0,
                    help="threads per row-transform block (0 = the library's default)")
    ap.add_argument("--plasma-threads", type=int, default=0,
                    help="threads per plasma cell-row block (0 = the library's default)")
    ap.add_argument("--col-threads", type=int, default=0,
                    help="threads per column transform (16, 32, 64; 0 = the library's default)")
    ap.add_argument("--cpu-slices", type=int, default=None,
                    help="slices of the oracle sample (default: about 15 s of oracle work)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra entries (the 256^3-class workload in float64 and float32)")
    ap.add_argument("--beside-blocks", type=int, default=None,
                    help="workgroups per launch of the beam work beside the slice loop (0 = the work's)")
    ap.add_argument("--lean", action="store_true",
                    help="steps in flight without a second copy of the beam (with --pipeline > 1; the pair512 "
                         "default is a lean pipeline as deep as memory allows, at most 5)")
    ap.add_argument("--resort-every", type=int, default=None,
                    help="one step at a time: reorder the beam storage by deposit key every n steps (0 = never; "
                         f"default {RESORT_EVERY})")
    ap.add_argument("--no-beside", action="store_true",
                    help="one step at a time: deposit, sweep and push one after the other instead of the "
                         "beam work beside the slice loop")
    ap.add_argument("--no-graphs", action="store_true",
                    help="enqueue every launch instead of replaying HIP graphs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 2 GiB three times (scale for HBM counters)")
    ap.add_argument("--breakdown", action="store_true",
                    help="also time every kernel class over one extra group of steps each")
    ap.add_argument("--no-scan", action="store_true",
                    help="skip the 64-instance batched scan among the extra configurations")
    ap.add_argument("--no-dirichlet", action="store_true",
                    help="skip the conducting-wall (sine-transform) solver measurement")
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

    if args.scan:
        print(json.dumps(scan_rate(args.scan, args.steps, args.warmup)), flush=True)
        return
    if args.adjoint_only:
        adj = adjoint_ratio(args.pipeline or 8)
        print(json.dumps(dict(adj, n_gpus=1, data="synthetic (seeded PCG64 plasma lattice + flat-top beam)")),
              flush=True)
        return
    wl = W.CONFIGS[args.workload]()
    precision = args.precision or wl.precision
    wl = wl.with_(precision=precision)
    if args.pipeline is not None:
        pipeline, lean = args.pipeline, args.lean
    elif args.workload == "pair512":
        # the beam (128 GiB) cannot be held twice: as many lean steps in
        # flight as the device's memory holds
        pipeline = lean_depth(wl, precision)
        lean = pipeline > 1
    else:
        pipeline, lean = 8, args.lean
    head = run_workload(wl, precision, pipeline, args.steps, args.warmup, args, with_extras=True, lean=lean)

    extra = {}
    keys = ("value", "ms_per_step", "steps", "warmup", "dtype", "config", "sweep_only", "roofline")
    if not args.no_extra and args.workload != "cube256":
        cube = W.cube256()
        for prec in ("f64", "f32"):
            e = run_workload(cube.with_(precision=prec), prec, 8, 16, 4, args, with_extras=False)
            extra[f"{cube.name}_{prec}"] = {k: e[k] for k in keys}
    if not args.no_extra and args.workload != "slab":
        # the 64 x 128 slab (float64, 8 steps in flight): launch-bound at
        # 256 plasma particles per slice, reported in absolute terms
        slab = W.CONFIGS["slab"]()
        try:
            e = run_workload(slab, "f64", 8, 48, 8, args, with_extras=False)
            extra[f"{slab.name}_f64"] = {k: e[k] for k in keys}
        except Exception as exc:  # recorded in the line, the headline stands
            log(f"slab workload failed: {exc!r}")
            extra[f"{slab.name}_f64"] = {"error": repr(exc)}
        if not args.no_scan:
            # the 64-instance batched scan (float32), all instances on this GPU
            sc = scan_rate(64, 3, 1)
            log(f"scan64: {sc['ms_per_step']:.1f} ms per batched step, {sc['value']:.3e} updates/s")
            extra["scan64_f32"] = {k: sc[k] for k in ("value", "ms_per_step", "steps", "warmup", "dtype", "config")}
    linear = None
    if not args.no_linear_model:
        linear = linear_model_rate()
        log(f"linear model: {linear['instances']} instances x {linear['xi_points']} points x "
            f"{linear['rk4_steps']} RK4 steps in {linear['ms']:.1f} ms")
    dirichlet = None
    if not args.no_dirichlet:
        dirichlet = dirichlet_rate()
        log(f"dirichlet solve: {dirichlet['grids']} grids of {dirichlet['ny']}x{dirichlet['nx']} in "
            f"{dirichlet['ms']:.2f} ms ({dirichlet['alg_GB_s']:.0f} GB/s algorithmic)")
    adjoint = None
    if not args.no_adjoint:
        log("adjoint workload ...")
        adjoint = adjoint_ratio(8)
        log(f"adjoint {adjoint['adjoint_ms']:.0f} ms / forward {adjoint['forward_ms']:.0f} ms "
            f"= {adjoint['value']:.2f}")
    cpu = None
    if not args.no_cpu_baseline:
        # about 15 s of float64 oracle work on the box's threads and about as
        # much on one (measured on 8 cores: 1.5 us per plasma particle-slice
        # and 0.42 us per beam particle)
        import torch
        nthr = torch.get_num_threads()
        est8 = 1.5e-6 * wl.n_plasma + 0.42e-6 * wl.n_beam_total / max(wl.beam_slices, 1)
        n_sl = args.cpu_slices or max(2, min(wl.nxi, int(15.0 / (est8 * 8.0 / nthr))))
        n_one = max(1, min(wl.nxi, int(15.0 / (est8 * 6.0))))
        log(f"oracle baseline on {n_sl} slices (and {n_one} on one core) ...")
        cpu = cpu_baseline(wl, n_sl, n_one)
        log(f"oracle: {cpu['value']:.3e} updates/s on {cpu['cores']} threads, "
            f"{cpu['one_core']['value']:.3e} on one ({cpu['cpu_model']}, nproc {cpu['nproc']})")
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
        "value": head["value"],
        "unit": "plasma particle-slice updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": precision,
        "data": "synthetic (seeded PCG64 plasma lattice + flat-top beam)",
        "config": head["config"],
        "sweep_only": head["sweep_only"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "extra_configs": extra or None,
        "adjoint": adjoint,
        "diagnostics": head["diagnostics"],
        "linear_model": linear,
        "dirichlet_solve": dirichlet,
    }
    if "kernel_breakdown_ms_per_step" in head:
        out["kernel_breakdown_ms_per_step"] = head["kernel_breakdown_ms_per_step"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
