"""GPU parity at the benchmark sizes, in the launch configuration bench.py
times (sort tile 4 x 16, sort every 16 steps, 16 particles per thread), against
the FP64 oracle running the same step on the host cores:

  * the dipole rotator, 1024 x 1024 cells, 64 particles per cell (67.1M),
    surface injection on: two steps (the first sorts, the second does not),
    every field and every particle compared, FP64 and FP32 -- the FP32 case
    one step at a time from identical input bits (the oracle reloaded from
    the GPU state before each step), as the FP32 tolerance is per step;
  * the plain FP64 method, 64 x 64 cells, 16 pairs per cell, 100 steps;
  * the monopole rotator, 512 x 512, from an empty start: the first 30
    steps of surface injection (FP32 checked one step at a time, at steps
    10, 20 and 30);
  * the four smallest runs of the 64-run ensemble, stepped as one batch;
  * the 2048 x 2048 precision-stress workload (201M particles): FP64 three
    steps, FP32 two steps one at a time (particles compared after the last).

The per-step tolerances are those of the small parity tests (parity_util),
FP32 fields measured against the scale of their vector field (E, B or F:
early in a rotator run the meridional and azimuthal parts are orders of
magnitude below the radial one, and FP32 rounding follows the vector);
over several steps they grow with the step count for FP64 (reordered
floating-point atomics) and stay fixed for FP32.  For FP64 fields the
oracle's own resolution sets the floor: it keeps absolute FP64 grid
coordinates and forms the new ones from r' and cos(theta'), which carries a
rounding of about eps * N / 2 cells per move on an N-cell axis; the face
charges, and the fields they drive, inherit it.  The FP64 field tolerance is
therefore 1e-12 * max(1, N / 256)."""
import os
import sys
import time

import numpy as np
import pytest

from paper_1407_1810_amd import workloads as W
from parity_util import TOL, compare_fields, oracle_from_sim, round_to_storage

pytestmark = pytest.mark.gpu

TILE, SORT_INTERVAL, PPT = (4, 16), 16, 16


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    from paper_1407_1810_amd.binding import gpu_available, lib
    if not gpu_available():
        pytest.skip("no HIP device")
    lib()
    from oracle import oracle as O
    O.set_threads(max(1, min(16, len(os.sched_getaffinity(0)))))


def _by_id(P):
    """Arrays ordered by particle id.  Preloaded ids (top bit clear) are
    placed by direct indexing while none has been deleted, else sorted;
    injected ones (top bit set) follow in id order."""
    ids = P["id"]
    pre = ids < np.uint64(1 << 63)
    n0 = int(pre.sum())
    pid = ids[pre].astype(np.int64)
    direct = n0 == 0 or int(pid.max()) == n0 - 1
    order = None if direct else np.argsort(pid, kind="stable")
    out = {}
    inj = np.argsort(ids[~pre], kind="stable")
    for k, v in P.items():
        a = np.empty_like(v)
        if direct:
            a[pid] = v[pre]
        else:
            a[:n0] = v[pre][order]
        a[n0:] = v[~pre][inj]
        out[k] = a
    return out, n0


def _compare_large(o, s, tol, nth, band):
    Po, no = _by_id(o.particles())
    Ps, ns = _by_id(s.particles())
    assert no == ns and len(Po["x"]) == len(Ps["x"]), (no, ns, len(Po["x"]), len(Ps["x"]))
    assert np.array_equal(Po["id"], Ps["id"])
    if len(Po["x"]) == 0:
        return
    io, jo = np.floor(Po["x"]), np.minimum(np.floor(Po["y"]), nth - 1)
    ig, jg = np.floor(Ps["x"]), np.minimum(np.floor(Ps["y"]), nth - 1)
    dx = np.abs(Po["x"] - np.round(Po["x"]))
    dy = np.abs(Po["y"] - np.round(Po["y"]))
    bad = ((io != ig) & (dx > band)) | ((jo != jg) & (dy > band))
    in_band = int(((io != ig) | (jo != jg)).sum() - bad.sum())
    assert not bad.any(), f"{int(bad.sum())} cell mismatches outside the band"
    same = (io == ig) & (jo == jg)
    ex = np.abs(Po["x"] - Ps["x"])[same].max(initial=0.0)
    ey = np.abs(Po["y"] - Ps["y"])[same].max(initial=0.0)
    umag = np.sqrt(Po["ur"] ** 2 + Po["ut"] ** 2 + Po["up"] ** 2)
    du = np.sqrt((Po["ur"] - Ps["ur"]) ** 2 + (Po["ut"] - Ps["ut"]) ** 2 + (Po["up"] - Ps["up"]) ** 2)
    emom = (du / (umag + 1e-3)).max(initial=0.0)
    _say(f"  particles {len(Po['x'])}: offsets {ex:.2e} {ey:.2e}, momenta {emom:.2e}, in-band cells {in_band}")
    assert ex <= tol["off"] and ey <= tol["off"]
    assert emom <= tol["mom"]
    assert np.abs(Po["w"] - Ps["w"]).max() <= 1e-7 * np.abs(Po["w"]).max()


def _field_tol(prec, p):
    if prec == "fp32":
        return TOL[prec]["field"]
    return TOL[prec]["field"] * max(1.0, max(p["nr"], p["nth"]) / 256.0)


def _pair(p, P, prec, capacity, ids=True):
    from oracle.oracle import Oracle
    from paper_1407_1810_amd.binding import Sim
    o = Oracle(p)
    s = Sim(p, precision=prec, capacity=capacity, tile=TILE, sort_interval=SORT_INTERVAL, chunk_ppt=PPT, ids=ids)
    if P is not None:
        R = round_to_storage(P, prec, p["nth"])
        o.add_particles(R["x"], R["y"], R["ur"], R["ut"], R["up"], R["w"], R["id"])
        del R
        s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
    return o, s


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dipole_rotator_1024_full_size(prec):
    cfg = W.config(2)
    p = cfg["params"]
    t0 = time.time()
    P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    n = len(P["x"])
    _say(f"dipole rotator {prec}: {n} particles generated in {time.time() - t0:.1f} s")
    o, s = _pair(p, P, prec, n + (4 << 20))
    del P
    t = TOL[prec]
    for k in range(2):
        if prec == "fp32" and k > 0:
            o = oracle_from_sim(s, p)
        t0 = time.time()
        s.step(1)
        t1 = time.time()
        o.step(1)
        _say(f" step {k}: gpu {t1 - t0:.2f} s, oracle {time.time() - t1:.1f} s, injected {o.counters()[0]}")
        sc = 1.0 if prec == "fp32" else (k + 1)
        compare_fields(o, s, _field_tol(prec, p) * 2 * sc, vector_scale=prec == "fp32")
        _compare_large(o, s, {kk: v * 2 * sc for kk, v in t.items()}, p["nth"], t["band"] * 2 * sc)
    if prec == "fp64":
        assert s.counts()["injected"] == o.counters()[0]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_precision_stress_2048_window(prec):
    """The 2048 x 2048 precision-stress workload (48 particles per cell,
    201M, injection on), whose long runs set the FP32 path beside the FP64
    GPU path: both checked against the oracle over a short window, FP64 for
    three steps run on, FP32 for two steps each from identical input bits."""
    cfg = W.config(3)
    p = cfg["params"]
    t0 = time.time()
    P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    n = len(P["x"])
    _say(f"precision stress {prec}: {n} particles generated in {time.time() - t0:.1f} s")
    o, s = _pair(p, P, prec, n + (8 << 20))
    del P
    t = TOL[prec]
    steps = 3 if prec == "fp64" else 2
    for k in range(steps):
        if prec == "fp32" and k > 0:
            o = oracle_from_sim(s, p)
        t0 = time.time()
        s.step(1)
        t1 = time.time()
        o.step(1)
        _say(f" step {k}: gpu {t1 - t0:.2f} s, oracle {time.time() - t1:.1f} s, injected {o.counters()[0]}")
        sc = 1.0 if prec == "fp32" else (k + 1)
        compare_fields(o, s, _field_tol(prec, p) * 2 * sc, vector_scale=prec == "fp32")
        if k == steps - 1:
            _compare_large(o, s, {kk: v * 2 * sc for kk, v in t.items()}, p["nth"], t["band"] * 2 * sc)
    if prec == "fp64":
        assert s.counts()["injected"] == o.counters()[0]


def test_plain_fp64_64x64_100_steps():
    cfg = W.config(0)
    p = cfg["params"]
    P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    o, s = _pair(p, P, "fp64", len(P["x"]) + (1 << 16))
    t = TOL["fp64"]
    done = 0
    for k in (1, 9, 90):
        s.step(k)
        o.step(k)
        done += k
        sc = 10.0 * done
        _say(f"plain fp64 after {done} steps")
        compare_fields(o, s, _field_tol("fp64", p) * sc)
        _compare_large(o, s, {kk: v * sc for kk, v in t.items()}, p["nth"], t["band"] * sc)
    assert done == cfg["steps"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_monopole_rotator_512_first_steps(prec):
    cfg = W.config(1)
    p = cfg["params"]
    o, s = _pair(p, None, prec, 16 << 20)
    t = TOL[prec]
    for k in range(3):
        if prec == "fp32":
            # FP32: one step from identical input bits after the unchecked ones
            s.step(9)
            o = oracle_from_sim(s, p)
            s.step(1)
            o.step(1)
        else:
            s.step(10)
            o.step(10)
        sc = 2.0 if prec == "fp32" else 10.0 * (k + 1) * 10
        _say(f"monopole rotator {prec} after {10 * (k + 1)} steps: {o.n} particles")
        compare_fields(o, s, _field_tol(prec, p) * sc, vector_scale=prec == "fp32")
        _compare_large(o, s, {kk: v * sc for kk, v in t.items()}, p["nth"], t["band"] * sc)
    assert o.n > 0
    if prec == "fp64":
        assert s.counts()["injected"] == o.counters()[0]
    assert np.allclose(s.carry(), o.carry(), atol=1e-9 if prec == "fp64" else 1e-3)


def test_smallest_ensemble_runs_as_one_batch():
    from paper_1407_1810_amd.binding import Batch
    runs = W.config(4)["runs"]
    sizes = [d["params"]["nr"] * d["params"]["nth"] * d["pairs_per_cell"] for d in runs]
    pick = [runs[k] for k in np.argsort(sizes, kind="stable")[:4]]
    pairs = []
    for d in pick:
        p = d["params"]
        P = W.pair_plasma(p, d["pairs_per_cell"], d["theta_T"], d["weight"], d["seed"])
        o, s = _pair(p, P, "fp32", 2 * len(P["x"]) + (1 << 20))
        pairs.append((d, o, s))
    b = Batch([s for _, _, s in pairs])
    t = TOL["fp32"]
    for k in range(3):
        if k > 0:
            pairs = [(d, oracle_from_sim(s, d["params"]), s) for d, _, s in pairs]
        b.step(1)
        for d, o, s in pairs:
            o.step(1)
            _say(f"{d['name']} step {k}")
            compare_fields(o, s, _field_tol("fp32", d["params"]) * 5, vector_scale=True)
            _compare_large(o, s, {kk: v * 5 for kk, v in t.items()}, d["params"]["nth"], t["band"] * 5)
