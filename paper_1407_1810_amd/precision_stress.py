#!/usr/bin/env python3
"""Precision stress: the FP32 path (int cell + FP32 offset, FP32 fields,
momenta and face charges) against the FP64 GPU path on the same input bits,
over a long run of the 2048 x 2048 dipole rotator (201M particles).

A particle-in-cell plasma is chaotic: two runs that differ only in the
order of floating-point additions separate, and after enough steps their
fields differ by the particle noise itself.  A second FP64 context with a
different sort tile and interval (so a different order of the deposit's
floating-point atomics) measures that floor; the FP32 path is measured
against it.

On a geometric schedule of steps both FP64 contexts and the FP32 one are
read on a probe lattice (every 32nd node in i and j) and compared component
by component -- the six fields and the three filtered face charges --
relative to the FP64 vector field's inf-norm on the lattice (max and RMS).
The Gauss residual (E flux minus the filtered particle charge, FP64 on
every path) is compared with its value at the start, relative to the
absolute charge of the preloaded plasma per node (|w| x particles per cell)
and to the largest E flux of an interior node at that step.  One JSON line per probe, a
summary line at the end.  The FP64 GPU path is the reference because the
CPU oracle cannot run 10^12 particle-steps; both GPU paths are checked
against the oracle at this size, one step at a time, by
tests/test_gpu_fullsize.py.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_1407_1810_amd import workloads as W  # noqa: E402
from paper_1407_1810_amd.binding import COMPS, Sim  # noqa: E402

VEC = {"E": ("Er", "Eth", "Eph"), "B": ("Br", "Bth", "Bph"), "F": ("Fr", "Fth", "Fph")}


def probe(s: Sim, stride: int) -> dict:
    return {c: s.get_field(c)[::stride, ::stride].copy() for c in COMPS}


def compare(p32: dict, p64: dict) -> dict:
    out = {}
    for name, comps in VEC.items():
        scale = max(np.abs(p64[c]).max() for c in comps)
        for c in comps:
            d = np.abs(p32[c] - p64[c])
            out[c] = {"inf": float(d.max() / scale) if scale > 0 else float(d.max()),
                      "rms": float(np.sqrt(np.mean(d * d)) / scale) if scale > 0 else 0.0}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--config", type=int, default=3, help="workload index (3: 2048^2 precision stress)")
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--probes", type=str, default="1,2,5,10,20,50,100,200,500,1000,2000,3000,4000,5000",
                    help="steps at which the contexts are compared")
    ap.add_argument("--stride", type=int, default=32)
    ap.add_argument("--tile", type=str, default="4x8")
    ap.add_argument("--sort-interval", type=int, default=8)
    args = ap.parse_args()
    cfg = W.config(args.config)
    p = cfg["params"]
    P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    n = len(P["x"])
    tile = tuple(int(v) for v in args.tile.split("x"))
    cap = 2 * n + (8 << 20)
    sims = {}
    for name, prec, tl, si in (("fp32", "fp32", tile, args.sort_interval), ("fp64", "fp64", tile, args.sort_interval),
                               ("fp64_alt", "fp64", (8, 8), 4)):
        s = Sim(p, precision=prec, capacity=cap, ids=False, tile=tl, sort_interval=si)
        s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"])
        sims[name] = s
    del P
    qabs = abs(cfg["weight"]) * 2 * cfg["pairs_per_cell"]
    inner = slice(1, p["nr"] - p["absorb_cells"])
    g0 = {}
    for name, s in sims.items():
        G, Q = s.gauss()
        g0[name] = G - Q
    probes = sorted({int(v) for v in args.probes.split(",") if 0 < int(v) <= args.steps} | {args.steps})
    print(json.dumps({"workload": cfg["name"], "particles": n, "steps": args.steps, "probes": probes,
                      "stride": args.stride, "q_inj_over_w": p["q_inj"] / cfg["weight"]}), flush=True)
    wall = {name: 0.0 for name in sims}
    done = 0
    last = {}
    for target in probes:
        k = target - done
        for name, s in sims.items():
            t0 = time.perf_counter()
            s.step(k)
            wall[name] += time.perf_counter() - t0
        done = target
        ref = probe(sims["fp64"], args.stride)
        e32 = compare(probe(sims["fp32"], args.stride), ref)
        e64 = compare(probe(sims["fp64_alt"], args.stride), ref)
        drift, gd = {}, {}
        for name, s in sims.items():
            G, Q = s.gauss()
            gd[name] = (G, Q)
        gscale = float(np.abs(gd["fp64"][0][inner]).max()) or 1.0  # largest interior E flux now
        for name, (G, Q) in gd.items():
            d = float(np.abs((G - Q)[inner] - g0[name][inner]).max())
            drift[name] = {"per_node_charge": d / qabs, "per_flux": d / gscale}
        counts = {name: s.counts()["live"] for name, s in sims.items()}
        last = {"step": done, "live": counts, "gauss_drift": drift,
                "fp32_vs_fp64": {c: [round(e32[c]["inf"], 9), round(e32[c]["rms"], 9)] for c in COMPS},
                "fp64_alt_vs_fp64": {c: [round(e64[c]["inf"], 9), round(e64[c]["rms"], 9)] for c in COMPS}}
        print(json.dumps(last), flush=True)
    ps = {name: s.counts()["particle_steps"] for name, s in sims.items()}
    print(json.dumps({"summary": True, "steps": done, "final": last,
                      "eps32_sqrt_n": float(np.finfo(np.float32).eps * math.sqrt(done)),
                      "rate": {name: ps[name] / wall[name] for name in ps},
                      "fp32_speedup": (ps["fp32"] / wall["fp32"]) / (ps["fp64"] / wall["fp64"])}), flush=True)


if __name__ == "__main__":
    main()
