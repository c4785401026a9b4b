"""GPU parity at the benchmark sizes, in the launch configuration bench.py
times (sort tile 4 x 16, sort every 16 steps, 16 particles per thread), against
the FP64 oracle running the same step on the host cores:

  * the dipole rotator, 1024 x 1024 cells, 64 particles per cell (67.1M),
    surface injection on: two steps (the first sorts, the second does not),
    every field and every particle compared;
  * the plain FP64 method, 64 x 64 cells, 16 pairs per cell, 100 steps, one
    step compared at steps 1, 10 and 100;
  * the monopole rotator, 512 x 512, from an empty start: the first 30
    steps of surface injection, one step compared at steps 10, 20 and 30;
  * the four smallest runs of the 64-run ensemble, stepped as one batch;
  * the whole ensemble (64 runs, 320M particles), each run autotuned as the
    benchmark does, then one batched step of every run compared;
  * the 2048 x 2048 precision-stress workload (201M particles): two steps
    (particles compared after the last).

Every compared step starts from identical input bits: before it the oracle
is loaded with the GPU context's state (oracle_from_sim), so each step is
held to the per-step tolerances of the small parity tests (parity_util),
with no factor for the steps run before it.  FP32 fields are gated at 1e-5
of the inf-norm of their vector field (E, B or F: FP32 rounding follows the
vector, which the Cartesian push mixes) and at OWN_TOL_FP32 = 1e-4 of their
own inf-norm where a component is at least 1e-2 of its vector's scale
(early in the monopole rotator E_theta is 1.6e-2 of E_r, and its error
against its own norm is then about 60 times the vector-scale one); both
errors are printed for every component.  FP64 fields are gated at 1e-12 of
their own inf-norm, widened where the oracle's own rounding is larger: the
oracle keeps absolute grid coordinates (a unit in the last place is 1.1e-13
cells at 512), and a nearly radial move deposits meridional face charge in
proportion to its tiny meridional displacement, the difference of two such
coordinates; a
second oracle loaded with every coordinate shifted by one unit in the last
place and stepped beside the first measures that rounding, and the gate is
four times its response (parity_util.shifted_floor).  Momenta are gated
against the largest of the particle's old and new momentum and the largest
term of its update (plus 1e-3).
Multi-step runs are reported, not gated: floating-point atomics reorder
sums."""
import os
import sys
import time

import numpy as np
import pytest

from paper_1407_1810_amd import workloads as W
from parity_util import (OWN_TOL_FP32, TOL, carry_atol, compare_fields, coordinate_gates, momentum_scale,
                         oracle_from_sim, oracles_from_sim, shifted_floor, widen_by_update_terms)

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


def _compare_large(o, s, tol, nth, band, before=None):
    """Particles matched by id; the momentum error is taken against |u| +
    1e-3 with |u| the larger of the oracle's new momentum and, when the
    state before the step is given, the old one and the update's largest
    field term (parity_util.momentum_scale and widen_by_update_terms: a
    particle a strong field stops within the step keeps the rounding of the
    momentum it had, and one at rest in a nearly cancelling field the
    rounding of the field's terms)."""
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
    gx, gy, bx, by = coordinate_gates(o, tol["off"], band)
    bad = ((io != ig) & (dx > bx)) | ((jo != jg) & (dy > by))
    in_band = int(((io != ig) | (jo != jg)).sum() - bad.sum())
    assert not bad.any(), f"{int(bad.sum())} cell mismatches outside the band"
    same = (io == ig) & (jo == jg)
    ex = np.abs(Po["x"] - Ps["x"])[same].max(initial=0.0)
    ey = np.abs(Po["y"] - Ps["y"])[same].max(initial=0.0)
    unew = np.sqrt(Po["ur"] ** 2 + Po["ut"] ** 2 + Po["up"] ** 2)
    umag = unew if before is None else np.maximum(unew, momentum_scale(before, Po["id"]))
    du = np.sqrt((Po["ur"] - Ps["ur"]) ** 2 + (Po["ut"] - Ps["ut"]) ** 2 + (Po["up"] - Ps["up"]) ** 2)
    raised = 0
    if before is not None:
        umag, raised = widen_by_update_terms(o, before, Po["id"], umag, du, tol["mom"])
    rel = du / (umag + 1e-3)
    emom = rel.max(initial=0.0)
    _say(f"  particles {len(Po['x'])}: offsets {ex:.2e} {ey:.2e}, momenta {emom:.2e} (against the new momentum "
         f"alone {(du / (unew + 1e-3)).max(initial=0.0):.2e}; {raised} scaled by the update's field terms), "
         f"in-band cells {in_band}")
    if emom > tol["mom"]:
        for q in np.argsort(rel)[-4:]:
            _say(f"  worst particle id {int(Po['id'][q])}: oracle u ({Po['ur'][q]:.6e}, {Po['ut'][q]:.6e}, "
                 f"{Po['up'][q]:.6e}), gpu u ({Ps['ur'][q]:.6e}, {Ps['ut'][q]:.6e}, {Ps['up'][q]:.6e}), "
                 f"momentum scale {umag[q]:.3e}")
    assert ex <= gx and ey <= gy, (ex, ey, gx, gy)
    assert emom <= tol["mom"]
    assert np.abs(Po["w"] - Ps["w"]).max() <= 1e-7 * np.abs(Po["w"]).max()




def _compare_step(o, s, p, prec, particles=True, o_shift=None, before=None):
    """Fields (and particles) after one step from identical inputs; o_shift
    (FP64) is the oracle stepped from coordinates shifted by one unit in
    the last place, before the particles at the start of the step."""
    t = TOL[prec]
    floor = shifted_floor(o, o_shift) if o_shift is not None else None
    compare_fields(o, s, t["field"], vector_scale=prec == "fp32", own_tol=OWN_TOL_FP32 if prec == "fp32" else None,
                   floor=floor)
    if particles:
        _compare_large(o, s, t, p["nth"], t["band"], before)


def _step_from_gpu_state(s, p, prec, timed=True):
    """The oracle loaded with the GPU state, then both stepped once; for an
    FP64 context also the oracle loaded with shifted coordinates.  Returns
    the oracle, the shifted one and the momenta at the start of the step."""
    o, *rest = oracles_from_sim(s, p, (False, True) if prec == "fp64" else (False,))
    o_shift = rest[0] if rest else None
    before = _momenta(o)
    t0 = time.time()
    s.step(1)
    t1 = time.time()
    o.step(1)
    if timed:
        _say(f"  gpu {t1 - t0:.2f} s, oracle {time.time() - t1:.1f} s, {o.n} particles, injected {o.counters()[0]}")
    if o_shift is not None:
        o_shift.step(1)
    return o, o_shift, before


def _momenta(o):
    """Positions and momenta at the start of a step, by id."""
    P = o.particles()
    return {k: P[k] for k in ("id", "x", "y", "ur", "ut", "up")}


def _sim(p, P, prec, capacity, ids=True):
    """A context in the launch configuration of the benchmark holding P."""
    from paper_1407_1810_amd.binding import Sim
    s = Sim(p, precision=prec, capacity=capacity, tile=TILE, sort_interval=SORT_INTERVAL, chunk_ppt=PPT, ids=ids)
    if P is not None:
        s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
    return s


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dipole_rotator_1024_full_size(prec):
    cfg = W.config(2)
    p = cfg["params"]
    t0 = time.time()
    P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    n = len(P["x"])
    _say(f"dipole rotator {prec}: {n} particles generated in {time.time() - t0:.1f} s")
    s = _sim(p, P, prec, n + (4 << 20))
    del P
    inj = 0
    for k in range(2):
        o, o_shift, before = _step_from_gpu_state(s, p, prec)
        assert s.counts()["injected"] == o.counters()[0] + inj
        inj = s.counts()["injected"]
        _say(f" step {k} (sorts: {k == 0})")
        _compare_step(o, s, p, prec, o_shift=o_shift, before=before)
        del o, o_shift, before


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_precision_stress_2048_window(prec):
    """The 2048 x 2048 precision-stress workload (48 particles per cell,
    201M, injection on), whose long runs set the FP32 path beside the FP64
    GPU path: both checked against the oracle over two steps, each from
    identical input bits (particles compared after the second)."""
    cfg = W.config(3)
    p = cfg["params"]
    t0 = time.time()
    P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    n = len(P["x"])
    _say(f"precision stress {prec}: {n} particles generated in {time.time() - t0:.1f} s")
    s = _sim(p, P, prec, n + (8 << 20))
    del P
    inj = 0
    for k in range(2):
        o, o_shift, before = _step_from_gpu_state(s, p, prec)
        assert s.counts()["injected"] == o.counters()[0] + inj
        inj = s.counts()["injected"]
        _say(f" step {k}")
        _compare_step(o, s, p, prec, particles=k == 1, o_shift=o_shift, before=before)
        del o, o_shift, before


def test_plain_fp64_64x64_100_steps():
    """The plain FP64 method over its 100 steps: one step from identical
    input bits compared at steps 1, 10 and 100; the oracle run alongside
    from the start is reported beside it (not gated)."""
    cfg = W.config(0)
    p = cfg["params"]
    P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    s = _sim(p, P, "fp64", len(P["x"]) + (1 << 16))
    o_run = oracle_from_sim(s, p)
    done = 0
    for k in (1, 10, 100):
        if k - done - 1 > 0:
            s.step(k - done - 1)
            o_run.step(k - done - 1)
        o, o_shift, before = _step_from_gpu_state(s, p, "fp64", timed=False)
        o_run.step(1)
        done = k
        _say(f"plain fp64, step {done}")
        _compare_step(o, s, p, "fp64", o_shift=o_shift, before=before)
        rep = {}
        compare_fields(o_run, s, 1.0, report=rep)
        _say(f"  run alongside from step 0 (reported): worst field {max(rep.values()):.2e}")
    assert done == cfg["steps"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_monopole_rotator_512_first_steps(prec):
    """The monopole rotator from its empty start: one step from identical
    input bits compared at steps 10, 20 and 30 (injected pairs, their Philox
    positions and the injection carry included)."""
    cfg = W.config(1)
    p = cfg["params"]
    s = _sim(p, None, prec, 16 << 20)
    for k in range(3):
        s.step(9)
        o, o_shift, before = _step_from_gpu_state(s, p, prec, timed=False)
        _say(f"monopole rotator {prec} after {10 * (k + 1)} steps: {o.n} particles")
        _compare_step(o, s, p, prec, o_shift=o_shift, before=before)
        assert np.all(np.abs(s.carry() - o.carry()) <= carry_atol(o, p, prec))
    assert o.n > 0


def test_smallest_ensemble_runs_as_one_batch():
    from paper_1407_1810_amd.binding import Batch
    runs = W.config(4)["runs"]
    sizes = [d["params"]["nr"] * d["params"]["nth"] * d["pairs_per_cell"] for d in runs]
    pick = [runs[k] for k in np.argsort(sizes, kind="stable")[:4]]
    pairs = []
    for d in pick:
        p = d["params"]
        P = W.pair_plasma(p, d["pairs_per_cell"], d["theta_T"], d["weight"], d["seed"])
        pairs.append((d, None, _sim(p, P, "fp32", 2 * len(P["x"]) + (1 << 20))))
    b = Batch([s for _, _, s in pairs])
    for k in range(3):
        pairs = [(d, oracle_from_sim(s, d["params"]), s) for d, _, s in pairs]
        b.step(1)
        for d, o, s in pairs:
            before = _momenta(o)
            o.step(1)
            _say(f"{d['name']} step {k}")
            _compare_step(o, s, d["params"], "fp32", before=before)


def test_whole_ensemble_one_batched_step():
    """All 64 runs of the ensemble (320M particles) in the benchmark's
    launch configuration: 16 particles per thread, each run's sort tile and
    interval picked by the autotuner over 4 steps, then the runs stepped
    together as one batch.  After two batched steps, the next batched step
    of every run against its own oracle loaded from that run's state."""
    from collections import Counter

    from paper_1407_1810_amd.binding import Batch, Sim
    runs = W.config(4)["runs"]
    sims, picks = [], Counter()
    t0 = time.time()
    for d in runs:
        p = d["params"]
        P = W.pair_plasma(p, d["pairs_per_cell"], d["theta_T"], d["weight"], d["seed"])
        s = Sim(p, precision="fp32", capacity=2 * len(P["x"]) + (4 << 20), chunk_ppt=PPT)
        s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
        del P
        best, _ = s.autotune(steps=4)
        picks[f"{best[0]}x{best[1]}/K{best[2]}"] += 1
        sims.append(s)
    _say(f"ensemble: {len(sims)} runs, {sum(s.counts()['live'] for s in sims)} particles, loaded and autotuned "
         f"in {time.time() - t0:.0f} s: {dict(picks)}")
    b = Batch(sims)
    b.step(2)
    oracles = [oracle_from_sim(s, d["params"]) for d, s in zip(runs, sims)]
    b.step(1)
    for k, d in enumerate(runs):
        o = oracles[k]
        before = _momenta(o)
        o.step(1)
        _say(f"{d['name']}: {o.n} particles, injected {o.counters()[0]}")
        _compare_step(o, sims[k], d["params"], "fp32", before=before)
        oracles[k] = None
    b.close()
