#!/usr/bin/env python3
"""Throughput of the 2.5D axisymmetric PIC step on one MI355X.

One step = the whole hot path: counting sort (every sort_interval steps),
half Faraday, gather + push + deposit, half Faraday, current filter, Ampere
with walls and lossy layer, surface injection.  Metric: particle-steps/s
(live particles at the start of each step, summed over the timed steps,
over the wall time of the timed steps), inputs resident in HBM.

Workload: the aligned dipole rotator on a 1024 x 1024 log-r, equal-area grid
with 64 particles per cell (about 67M), surface injection on, FP32 particle
state (int32 cell + FP32 offsets) -- and the plain FP64 GPU path on the same
input beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per particle-step of the push+deposit kernel: the
# particle stream read (cell 4, two offsets, three momenta, weight) and
# written back (cell, offsets, momenta); and per cell of the grid, the six
# field components read and three face-charge components written once per step
PUSH_BYTES = {"fp32": (4 + 2 * 4 + 3 * 4 + 4) + (4 + 2 * 4 + 3 * 4), "fp64": (4 + 2 * 8 + 3 * 8 + 8) + (4 + 2 * 8 + 3 * 8)}
CELL_BYTES = {"fp32": 9 * 4, "fp64": 9 * 8}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = [os.path.join(ROOT, "paper_1407_1810_amd", "csrc", f) for f in ("pic_device.h", "pic_kernels.h")]
# committed rocprofv3 summaries (counter passes) of the push in each form
PROFILE = "k_push_dipole_rotator_1024x1024_ppc64.md"
PROFILE_FP64 = "k_push_fp64_dipole_rotator_1024x1024_ppc64.md"
PROFILE_BATCH = "k_push_batched_ensemble_64_runs.md"
PROFILE_STRESS = "k_push_precision_stress_2048x2048_ppc48.md"


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_copy_peak(mib=1024, reps=5) -> float:
    """HBM bandwidth a plain device-to-device copy reaches on this GPU, in
    GB/s (bytes read plus bytes written over the copy's event-timed
    duration): the practical ceiling beside the published peak."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def auto_sort_interval(steps: int, preferred: int = 16) -> int:
    """The sort interval the timed window is built on: the largest divisor of
    `steps` from 8 to `preferred` (so that the window holds whole sort
    intervals and the sort weighs in at its steady share), else `preferred`."""
    for k in range(preferred, 7, -1):
        if steps % k == 0:
            return k
    return preferred


def sync_device():
    """torch's view of the device, synchronised (the library synchronises
    its own stream at the end of every pic_step)."""
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except Exception:
        pass


def roofline(bytes_launch, kernel_ms, kernel, copy_gbs, traffic=None, utilisation=None):
    achieved = bytes_launch / (kernel_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "traffic": traffic, "kernel": kernel, "kernel_ms": kernel_ms, "algorithmic_bytes_per_launch": bytes_launch}
    if copy_gbs:
        out["measured_copy_peak"] = copy_gbs
        out["frac_of_copy"] = achieved / copy_gbs
    if utilisation is not None:
        out["utilisation"] = utilisation
    return out


def run_gpu(cfg, P, precision, steps, warmup, tile, sort_interval, ppt, gauss=True, tag=None):
    """One context on the workload: `warmup` steps, then the timed window of
    `steps` steps replayed from the step graphs (the production path of
    pic_step), bracketed by device synchronisations -- the value -- and then
    a second window of the same length enqueued eagerly between HIP events on
    the context stream, which gives each stage's mean device time and the
    push kernel's duration for the roofline.  Both windows span whole sort
    intervals."""
    from paper_1407_1810_amd.binding import Sim
    tag = tag or precision
    p = cfg["params"]
    n = len(P["x"])
    cap = n + 16 * (1 << 20)
    s = Sim(p, precision=precision, capacity=cap, ids=False, tile=tile, sort_interval=sort_interval, chunk_ppt=ppt)
    t0 = time.perf_counter()
    s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"])
    log(f"[{tag}] loaded {n} particles in {time.perf_counter() - t0:.1f} s")
    s.step(warmup)
    log(f"[{tag}] warmup {warmup} steps done")
    c0 = s.counts()
    sync_device()
    t0 = time.perf_counter()
    s.step(steps)
    sync_device()
    wall = time.perf_counter() - t0
    c1 = s.counts()
    # the same number of steps again, eagerly between HIP events
    s.set_timing(True)
    t1 = time.perf_counter()
    s.step(steps)
    wall_e = time.perf_counter() - t1
    c2 = s.counts()
    st = s.stage_ms()
    s.set_timing(False)
    psteps = c1["particle_steps"] - c0["particle_steps"]
    res = dict(value=psteps / wall, ms_per_step=1e3 * wall / steps, particle_steps=psteps,
               mean_live=psteps / steps, stage_ms=st, live_end=c1["live"], injected=c1["injected"],
               deleted=c1["deleted"], sort_interval=sort_interval,
               eager_ms_per_step=1e3 * wall_e / steps,
               eager_mean_live=(c2["particle_steps"] - c1["particle_steps"]) / steps,
               global_chunks=c2["global_chunks"])
    log(f"[{tag}] {steps} steps: {res['value']:.4e} particle-steps/s, {res['ms_per_step']:.3f} ms/step "
        f"(graph); eager {res['eager_ms_per_step']:.3f} ms/step, stages "
        f"{json.dumps({k: round(v, 4) for k, v in st.items()})}")
    if gauss:
        # the Gauss-law residual (an occasional diagnostic, outside the timed
        # steps): one whole PIC_MOM_GAUSS_RES call -- node charge, filter
        # passes, FP64 flux and residual reductions on the device, the scalars
        # copied to the host -- the second of two calls (the first records the
        # reference)
        for _ in range(2):
            t0 = time.perf_counter()
            g = s.gauss_residual()
            res["gauss_diagnostic_ms"] = 1e3 * (time.perf_counter() - t0)
        res["gauss"] = {k: g[k] for k in ("drift_max", "res_max", "abs_charge_max", "flux_max", "nodes",
                                          "non_finite")}
        log(f"[{tag}] Gauss residual diagnostic: {res['gauss_diagnostic_ms']:.2f} ms per call, {res['gauss']}")
    s.close()
    return res


def run_monopole(steps):
    """The monopole rotator in FP64 from its empty start (512 x 512 cells,
    surface injection only): `steps` steps replayed from the step graphs,
    timed whole -- the particle count grows from zero, so the grid work
    weighs in far more than on the preloaded workloads."""
    from paper_1407_1810_amd import workloads as W
    from paper_1407_1810_amd.binding import Sim
    cfg = W.config(1)
    p = cfg["params"]
    s = Sim(p, precision="fp64", capacity=16 << 20, ids=False, tile=(4, 8), sort_interval=8)
    c0 = s.counts()
    sync_device()
    t0 = time.perf_counter()
    s.step(steps)
    sync_device()
    wall = time.perf_counter() - t0
    c1 = s.counts()
    s.close()
    res = dict(workload=cfg["name"], precision="fp64", steps=steps,
               value=(c1["particle_steps"] - c0["particle_steps"]) / wall, ms_per_step=1e3 * wall / steps,
               particles_end=c1["live"], injected=c1["injected"])
    log(f"[monopole fp64] {steps} steps from an empty start: {res['value']:.4e} particle-steps/s, "
        f"{res['ms_per_step']:.3f} ms/step, {c1['live']} particles at the end")
    return res


def run_batched(n_runs, steps, warmup, tune_steps, seq, ppt=16):
    """The uneven ensemble in FP32: every run autotuned (sort tile and
    interval), then stepped together by one batch (one launch sequence per
    step, replayed from a HIP graph) and, for comparison, one run after the
    other with its own launches."""
    from collections import Counter

    from paper_1407_1810_amd import workloads as W
    from paper_1407_1810_amd.binding import Batch, Sim
    cfg = W.config(4)
    runs = cfg["runs"][:n_runs]
    sims, picks, n0 = [], Counter(), 0
    t0 = time.perf_counter()
    for d in runs:
        p = d["params"]
        P = W.pair_plasma(p, d["pairs_per_cell"], d["theta_T"], d["weight"], d["seed"])
        n = len(P["x"])
        n0 += n
        # room for the surface injection of the tuning, warm-up and timed steps
        # (sized to stay near half the preload over that window)
        s = Sim(p, precision="fp32", capacity=2 * n + (4 << 20), ids=False, chunk_ppt=ppt)
        s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"])
        del P
        best, _ = s.autotune(steps=tune_steps)
        picks[f"{best[0]}x{best[1]}/K{best[2]}"] += 1
        sims.append(s)
    log(f"[batched] {len(sims)} runs, {n0} particles loaded and autotuned in {time.perf_counter() - t0:.1f} s: "
        f"{dict(picks)}")
    b = Batch(sims)
    b.step(warmup)
    ps0 = sum(s.counts()["particle_steps"] for s in sims)
    t0 = time.perf_counter()
    b.step(steps)
    wall = time.perf_counter() - t0
    dev_ms = b.elapsed_ms()
    ps = sum(s.counts()["particle_steps"] for s in sims) - ps0
    live = sum(s.counts()["live"] for s in sims)
    res = dict(value=ps / wall, ms_per_step=1e3 * wall / steps, device_ms_per_step=dev_ms / steps,
               particle_steps=ps, runs=len(sims), particles_start=n0, live_end=live, autotuned=dict(picks),
               steps=steps, warmup=warmup)
    log(f"[batched] {steps} steps: {res['value']:.4e} particle-steps/s, {res['ms_per_step']:.3f} ms/step")
    # a window of the same runs stepped eagerly between HIP events: the push
    # kernel's duration over all runs, for the roofline of the batched form
    ew = min(steps, 32)
    before = [s.counts()["particle_steps"] for s in sims]
    b.set_timing(True)
    b.step(ew)
    st = b.stage_ms()
    b.set_timing(False)
    live_mean = [(s.counts()["particle_steps"] - c) / ew for s, c in zip(sims, before)]
    cells = [d["params"]["nr"] * d["params"]["nth"] for d in runs]
    res["stage_ms"] = {k: round(v, 5) for k, v in st.items()}
    res["eager_steps"] = ew
    res["push_bytes_per_launch"] = sum(PUSH_BYTES["fp32"] * m + CELL_BYTES["fp32"] * c for m, c in zip(live_mean, cells))
    res["push_kernel"] = f"k_push<float,{sims[0].grid.chunk_ppt or 8}>"
    log(f"[batched] eager window of {ew} steps: stages {json.dumps(res['stage_ms'])}")
    if seq:
        wall_s, ps_s = 0.0, 0
        for s in sims:
            c0 = s.counts()["particle_steps"]
            t0 = time.perf_counter()
            s.step(steps)
            wall_s += time.perf_counter() - t0
            ps_s += s.counts()["particle_steps"] - c0
        res["sequential_value"] = ps_s / wall_s
        res["sequential_ms_per_step"] = 1e3 * wall_s / steps
        res["speedup_vs_sequential"] = res["value"] / res["sequential_value"]
        log(f"[batched] sequential: {res['sequential_value']:.4e} particle-steps/s, "
            f"batch speedup {res['speedup_vs_sequential']:.2f}x")
    b.close()
    for s in sims:
        s.close()
    return res


def cpu_baseline(cfg, P, seconds=12.0, max_threads=16):
    """The FP64 oracle on the host cores, same workload, bounded sample:
    the full grid with every 4th pair of the particle set, as many steps as
    fit in about `seconds`."""
    from oracle import oracle as O
    O.build()
    nthreads = max(1, min(max_threads, len(os.sched_getaffinity(0))))
    O.set_threads(nthreads)
    import numpy as np
    o = O.Oracle(cfg["params"])
    npair = len(P["x"]) // 2
    idx = np.arange(0, npair, 4)
    take = np.empty(2 * len(idx), dtype=np.int64)
    take[0::2] = 2 * idx
    take[1::2] = 2 * idx + 1
    o.add_particles(*[P[k][take] for k in ("x", "y", "ur", "ut", "up", "w")])
    m = o.n
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds or steps >= 50:
            break
    v = m * steps / el
    log(f"[cpu oracle] {m} particles x {steps} steps in {el:.1f} s on {nthreads} threads: {v:.3e} particle-steps/s")
    return dict(value=v, unit="particle-steps/s", cores=nthreads, kind="oracle",
                sample=f"FP64 oracle, same 1024x1024 grid and fields, every 4th pair ({m} particles), "
                       f"{steps} steps, {nthreads} threads")


def oracle_timing(seconds=8.0, max_threads=16):
    """The FP64 oracle on the host cores, one thread and all of them, on
    bounded samples of the four single-run workloads: the 64 x 64 plain FP64
    method in full; the 512 x 512 monopole rotator's first steps from its
    empty start (injection only); the 1024 x 1024 dipole rotator with 8 of
    its 32 pairs per cell; the 2048 x 2048 precision stress with 3 of its 24.
    Each entry runs until `seconds` have passed or its step count is done;
    the rate counts the live particles at the start of each step."""
    from oracle import oracle as O
    from paper_1407_1810_amd import workloads as W
    O.build()
    allt = max(1, min(max_threads, len(os.sched_getaffinity(0))))
    plan = [(0, None, 100), (1, None, 200), (2, 8, 50), (3, 3, 20)]
    rows = []
    for k, ppc, max_steps in plan:
        cfg = W.config(k)
        p = cfg["params"]
        pairs = cfg.get("pairs_per_cell", 0) if ppc is None else ppc
        P = W.pair_plasma(p, pairs, cfg["theta_T"], cfg["weight"], cfg["seed"]) if pairs else None
        for threads in sorted({1, allt}):
            O.set_threads(threads)
            o = O.Oracle(p)
            if P is not None:
                o.add_particles(*[P[q] for q in ("x", "y", "ur", "ut", "up", "w")])
            psteps, steps, t0 = 0, 0, time.perf_counter()
            while steps < max_steps and time.perf_counter() - t0 < seconds:
                psteps += o.n
                o.step(1)
                steps += 1
            el = time.perf_counter() - t0
            rows.append(dict(workload=cfg["name"], pairs_per_cell=pairs, threads=threads, steps=steps,
                             particles_end=o.n, seconds=round(el, 2), ms_per_step=1e3 * el / steps,
                             value=psteps / el))
            log(f"[oracle] {cfg['name']} ({pairs} pairs/cell) {threads} threads: {steps} steps, "
                f"{psteps / el:.3e} particle-steps/s")
            del o
    return dict(unit="particle-steps/s", kind="oracle", host_threads=allt, rows=rows)


def profile_figures(name: str) -> dict:
    """'key: value' figures of a committed rocprofv3 summary under profiles/,
    or {} when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- `"):
            k, v = line[3:].split("`", 1)[0], line.split(":", 1)[1].strip().rstrip(".")
            vals[k] = v
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return {}
    return vals


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--fp64-steps", type=int, default=16)
    ap.add_argument("--stress-steps", type=int, default=16)
    ap.add_argument("--parts", type=str, default="fp32,fp64,batched,stress,mono,cpu",
                    help="comma list of fp32, fp64, batched, stress (the 2048^2 workload in FP32), mono (the 512^2 "
                         "monopole rotator in FP64 from its empty start), cpu")
    ap.add_argument("--mono-steps", type=int, default=2000)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-stress", action="store_true")
    ap.add_argument("--tile", type=str, default="4x16")
    ap.add_argument("--sort-interval", type=int, default=0,
                    help="steps between sorts; 0 = the largest divisor of the window from 8 to 16, so that every "
                         "timed window holds whole sort intervals")
    ap.add_argument("--ppt", type=int, default=16, help="particles per thread of a push work-group (4, 8, 16)")
    ap.add_argument("--batched-runs", type=int, default=64)
    ap.add_argument("--batched-ppt", type=int, default=16, help="particles per thread of the batch's push")
    ap.add_argument("--batched-steps", type=int, default=200)
    ap.add_argument("--batched-warmup", type=int, default=50)
    ap.add_argument("--batched-tune-steps", type=int, default=4)
    ap.add_argument("--oracle-timing", action="store_true",
                    help="only time the FP64 oracle on samples of the four single-run workloads (host cores)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.oracle_timing:
        print(json.dumps(oracle_timing()), flush=True)
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration} MiB three times")
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the step is not sharded across "
              f"GPUs", file=sys.stderr)
        sys.exit(2)
    parts = set(args.parts.split(","))
    for flag, part in ((args.no_fp64, "fp64"), (args.no_cpu_baseline, "cpu"), (args.no_batched, "batched"),
                       (args.no_stress, "stress")):
        if flag:
            parts.discard(part)
    # the copy is timed through torch, which must initialise the device before
    # the library's own HIP context exists
    copy_gbs = measured_copy_peak()
    log(f"plain 1 GiB device copy: {copy_gbs:.0f} GB/s")
    from paper_1407_1810_amd import workloads as W
    cfg = W.config(2)
    p = cfg["params"]
    tile = tuple(int(v) for v in args.tile.split("x"))
    cells = p["nr"] * p["nth"]
    P = None
    if parts & {"fp32", "fp64", "cpu"}:
        t0 = time.perf_counter()
        P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
        log(f"generated {len(P['x'])} particles for {cfg['name']} in {time.perf_counter() - t0:.1f} s")
    n = 2 * cfg["pairs_per_cell"] * cells
    k32 = args.sort_interval or auto_sort_interval(args.steps)
    r32 = r64 = rb = rs = None
    if "fp32" in parts:
        r32 = run_gpu(cfg, P, "fp32", args.steps, args.warmup, tile, k32, args.ppt)
    if "fp64" in parts:
        k64 = args.sort_interval or auto_sort_interval(args.fp64_steps)
        r64 = run_gpu(cfg, P, "fp64", args.fp64_steps, min(args.warmup, 2), tile, k64, args.ppt)
    cpu = cpu_baseline(cfg, P) if "cpu" in parts else None
    del P
    if "batched" in parts:
        rb = run_batched(args.batched_runs, args.batched_steps, args.batched_warmup, args.batched_tune_steps, True,
                         args.batched_ppt)
    if "stress" in parts:
        c3 = W.config(3)
        t0 = time.perf_counter()
        P3 = W.pair_plasma(c3["params"], c3["pairs_per_cell"], c3["theta_T"], c3["weight"], c3["seed"])
        log(f"generated {len(P3['x'])} particles for {c3['name']} in {time.perf_counter() - t0:.1f} s")
        k3 = args.sort_interval or auto_sort_interval(args.stress_steps)
        rs = run_gpu(c3, P3, "fp32", args.stress_steps, args.warmup, tile, k3, args.ppt, gauss=False,
                     tag="stress fp32")
        del P3
        rs["workload"] = c3["name"]
        rs["particles"] = 2 * c3["pairs_per_cell"] * c3["params"]["nr"] * c3["params"]["nth"]
        rs["cells"] = c3["params"]["nr"] * c3["params"]["nth"]
    rm = run_monopole(args.mono_steps) if "mono" in parts else None
    out = {
        "metric": "particle-steps/sec (push+deposit+field), FP32 and batched vs FP64 GPU",
        "value": r32["value"] if r32 else None,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"] if r32 else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": f"{p['nr']}x{p['nth']}", "particles": n,
                   "particles_per_cell": 2 * cfg["pairs_per_cell"], "background": p["bg_kind"],
                   "injection": bool(p["inject"]), "n_filt": p["n_filt"], "absorb_cells": p["absorb_cells"],
                   "tile": args.tile, "sort_interval": k32, "particles_per_thread": args.ppt,
                   "precision": "fp32", "timed_path": "graph replay (pic_step)"},
    }
    if r32:
        prof = profile_figures(PROFILE)
        # HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE passes
        # (scaled by a plain copy of known size), valid for this kernel source
        traffic = float(prof["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in prof else None
        util = None
        if "valu_busy" in prof:
            util = {"valu_busy": float(prof["valu_busy"]), "valu_instr_per_particle": float(prof["valu_instr_per_particle"])}
        bl = PUSH_BYTES["fp32"] * r32["eager_mean_live"] + CELL_BYTES["fp32"] * cells
        out["roofline"] = roofline(bl, r32["stage_ms"]["push"], f"k_push<float,{args.ppt}>", copy_gbs, traffic, util)
        out["roofline"]["timed_on"] = "eager window of the same length after the timed steps, HIP events on the context stream"
        out["stage_ms"] = {k: round(v, 5) for k, v in r32["stage_ms"].items()}
        out["eager_ms_per_step"] = r32["eager_ms_per_step"]
        out["gauss_diagnostic_ms"] = r32.get("gauss_diagnostic_ms")
        out["gauss"] = r32.get("gauss")
    if r64:
        prof = profile_figures(PROFILE_FP64)
        traffic = float(prof["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in prof else None
        bl = PUSH_BYTES["fp64"] * r64["eager_mean_live"] + CELL_BYTES["fp64"] * cells
        out["fp64_gpu"] = {
            "value": r64["value"], "ms_per_step": r64["ms_per_step"], "steps": args.fp64_steps,
            "sort_interval": r64["sort_interval"], "stage_ms": {k: round(v, 5) for k, v in r64["stage_ms"].items()},
            "fp32_speedup": (r32["value"] / r64["value"]) if r32 else None,
            "gauss_diagnostic_ms": r64.get("gauss_diagnostic_ms"),
            "roofline": roofline(bl, r64["stage_ms"]["push"], f"k_push<double,{args.ppt}>", copy_gbs, traffic)}
    if rb:
        prof = profile_figures(PROFILE_BATCH)
        traffic = float(prof["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in prof else None
        rb["roofline"] = roofline(rb["push_bytes_per_launch"], rb["stage_ms"]["push"], rb["push_kernel"], copy_gbs,
                                  traffic)
        out["batched_fp32"] = rb
    if rs:
        prof = profile_figures(PROFILE_STRESS)
        traffic = float(prof["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in prof else None
        bl = PUSH_BYTES["fp32"] * rs["eager_mean_live"] + CELL_BYTES["fp32"] * rs["cells"]
        out["stress_fp32"] = {
            "workload": rs["workload"], "particles": rs["particles"], "value": rs["value"],
            "ms_per_step": rs["ms_per_step"], "steps": args.stress_steps, "sort_interval": rs["sort_interval"],
            "stage_ms": {k: round(v, 5) for k, v in rs["stage_ms"].items()},
            "roofline": roofline(bl, rs["stage_ms"]["push"], f"k_push<float,{args.ppt}>", copy_gbs, traffic)}
    if rm:
        out["monopole_fp64"] = rm
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
