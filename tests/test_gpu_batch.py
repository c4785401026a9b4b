"""GPU batches: uneven runs stepped together by one launch sequence give, run
by run, what the FP64 oracle gives for each run alone; the captured graph
and the eagerly enqueued step agree; errors name their run."""
import sys

import numpy as np
import pytest

from paper_1407_1810_amd import workloads as W
from parity_util import TOL, compare_fields, compare_particles, make_pair, oracle_from_sim

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    from paper_1407_1810_amd.binding import gpu_available, lib
    if not gpu_available():
        pytest.skip("no HIP device")
    lib()


def _uneven_runs():
    """Three runs that differ in every per-run setting: grid, field kind,
    filter passes, lossy layer, injection, tile and sort interval."""
    out = []
    specs = [
        dict(nr=24, nth=20, pairs_per_cell=2, n_filt=3, absorb_cells=4, bg="monopole", omega_frac=0.3, inject=1,
             seed=11, tile=(4, 4), si=2),
        dict(nr=40, nth=32, pairs_per_cell=3, n_filt=0, absorb_cells=0, bg="dipole", omega_frac=0.2, inject=0,
             seed=12, tile=(8, 8), si=3),
        dict(nr=17, nth=44, pairs_per_cell=1, n_filt=2, absorb_cells=3, bg="dipole", omega_frac=0.25, inject=1,
             seed=13, tile=(2, 8), si=-1),
    ]
    for sp in specs:
        tile, si = sp.pop("tile"), sp.pop("si")
        cfg = W.small_config(**sp)
        p = dict(cfg["params"], q_inj=cfg["params"]["q_inj"] * 0.5, t_spin=4.0)
        P = W.pair_plasma(p, cfg["pairs_per_cell"], 0.2, cfg["weight"], sp["seed"])
        # unpair a quarter so that the plasma field is not zero
        P["x"][1::4] = np.clip(P["x"][1::4] + 0.37, 0.0, p["nr"] - 1e-9)
        out.append((p, P, tile, si))
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_the_oracle_run_by_run(prec):
    from paper_1407_1810_amd.binding import Batch
    pairs = []
    for p, P, tile, si in _uneven_runs():
        o, s = make_pair(p, P, prec, capacity=1 << 18, tile=tile, sort_interval=si)
        pairs.append((p, o, s))
    b = Batch([s for _, _, s in pairs])
    t = TOL[prec]
    injected = [0] * len(pairs)
    for k in range(6):
        _say("batch", prec, "step", k)
        # every step from identical input bits: each oracle reloaded from its run
        if k:
            pairs = [(p, oracle_from_sim(s, p), s) for p, _, s in pairs]
        before = [s.particles() for _, _, s in pairs]
        b.step(1)
        for r, (p, o, s) in enumerate(pairs):
            o.step(1)
            compare_fields(o, s, t["field"])
            compare_particles(o, s, t, p["nth"], t["band"], before=before[r])
            assert s.counts()["step"] == k + 1
            injected[r] += o.counters()[0]
    inj = [s.counts()["injected"] for _, _, s in pairs]
    assert inj[0] > 0 and inj[2] > 0 and inj[1] == 0
    assert inj == injected
    assert b.elapsed_ms() > 0.0
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_with_empty_runs_and_offset_steps(prec):
    """A batch holding a filled run, an empty run that fills by surface
    injection and starts at step index 7 (its sorts, every 3 steps, fall on
    other steps than the first run's, every 2), and an empty run without
    injection (nothing to push or sort at all): each run against its own
    oracle after every step."""
    from paper_1407_1810_amd.binding import Batch
    specs = [
        (dict(nr=24, nth=20, pairs_per_cell=2, n_filt=2, absorb_cells=4, bg="monopole", omega_frac=0.3, inject=1,
              seed=21), True, 2, 0),
        (dict(nr=28, nth=24, pairs_per_cell=0, n_filt=3, absorb_cells=4, bg="monopole", omega_frac=0.3, inject=1,
              seed=22), False, 3, 7),
        (dict(nr=20, nth=16, pairs_per_cell=0, n_filt=1, absorb_cells=3, bg="dipole", omega_frac=0.2, inject=0,
              seed=23), False, 4, 0),
    ]
    runs = []
    for sp, filled, si, step0 in specs:
        cfg = W.small_config(**sp)
        p = dict(cfg["params"], q_inj=cfg["params"]["q_inj"] * 0.5, t_spin=3.0)
        P = None
        if filled:
            P = W.pair_plasma(p, cfg["pairs_per_cell"], 0.2, cfg["weight"], sp["seed"])
            P["x"][1::4] = np.clip(P["x"][1::4] + 0.37, 0.0, p["nr"] - 1e-9)
        o, s = make_pair(p, P, prec, capacity=1 << 18, tile=(4, 4), sort_interval=si, step_index=step0)
        runs.append((p, o, s, step0))
    b = Batch([s for _, _, s, _ in runs])
    t = TOL[prec]
    injected = [0] * len(runs)
    for k in range(7):
        if k:
            runs = [(p, oracle_from_sim(s, p), s, step0) for p, _, s, step0 in runs]
        before = [s.particles() for _, _, s, _ in runs]
        b.step(1)
        for r, (p, o, s, step0) in enumerate(runs):
            o.step(1)
            compare_fields(o, s, t["field"])
            compare_particles(o, s, t, p["nth"], t["band"], before=before[r])
            assert s.counts()["step"] == step0 + k + 1
            injected[r] += o.counters()[0]
    assert runs[1][2].counts()["injected"] > 0
    assert runs[2][2].counts()["live"] == 0
    assert [s.counts()["injected"] for _, _, s, _ in runs] == injected
    b.close()


def test_graph_and_eager_steps_agree():
    """pic_step replays a captured graph; with stage timing on it enqueues
    the same launches one by one.  Both give the same state."""
    from paper_1407_1810_amd.binding import Sim
    p, P, tile, si = _uneven_runs()[0]
    sims = []
    for timing in (False, True):
        s = Sim(p, precision="fp64", capacity=1 << 18, tile=tile, sort_interval=si)
        s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
        s.set_timing(timing)
        s.step(7)
        sims.append(s)
    st = sims[1].stage_ms()
    assert st["total"] > 0.0 and st["push"] > 0.0
    compare_fields(sims[0], sims[1], 1e-12)
    a, c = sims[0].particles(), sims[1].particles()
    ka, kc = np.argsort(a["id"]), np.argsort(c["id"])
    for k in ("x", "y", "ur", "ut", "up", "w"):
        assert np.allclose(a[k][ka], c[k][kc], rtol=0, atol=1e-12 * (1 + np.abs(a[k]).max()))
    assert sims[0].counts() == sims[1].counts()


def test_batch_of_one_equals_the_context_alone():
    from paper_1407_1810_amd.binding import Batch, Sim
    p, P, tile, si = _uneven_runs()[1]
    s1 = Sim(p, precision="fp32", capacity=1 << 18, tile=tile, sort_interval=si)
    s2 = Sim(p, precision="fp32", capacity=1 << 18, tile=tile, sort_interval=si)
    for s in (s1, s2):
        s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
    b = Batch([s2])
    s1.step(5)
    b.step(5)
    compare_fields(s1, s2, 1e-5)
    assert s1.counts() == s2.counts()
    # a member may still be stepped alone between batch steps
    s2.step(1)
    b.step(1)
    assert s2.counts()["step"] == 7


def test_batch_errors_name_the_run():
    from paper_1407_1810_amd.binding import Batch, PicError, Sim
    runs = _uneven_runs()
    p0, P0, _, _ = runs[1]
    p1, _, _, _ = runs[0]
    ok = Sim(p0, precision="fp64", capacity=1 << 16)
    ok.add_particles(P0["x"], P0["y"], P0["ur"], P0["ut"], P0["up"], P0["w"], P0["id"])
    tight = Sim(dict(p1, q_inj=p1["q_inj"] * 1e-3), precision="fp64", capacity=16)
    b = Batch([ok, tight])
    with pytest.raises(PicError) as e:
        b.step(3)
    assert e.value.code == -4 and "run 1" in str(e.value)
    # mixed precisions are refused
    other = Sim(p0, precision="fp32", capacity=16)
    with pytest.raises(PicError) as e:
        Batch([ok, other])
    assert e.value.code == -1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autotune_and_resort_keep_parity(prec):
    """Retiling a live run (pic_set_sort) and autotuning it (which steps it
    under every candidate) leave the trajectory the oracle's; a batch whose
    member was retiled rebuilds its launch plan."""
    from paper_1407_1810_amd.binding import Batch
    runs = _uneven_runs()
    (p0, P0, t0, k0), (p1, P1, t1, k1) = runs[0], runs[1]
    o0, s0 = make_pair(p0, P0, prec, capacity=1 << 18, tile=t0, sort_interval=k0)
    o1, s1 = make_pair(p1, P1, prec, capacity=1 << 18, tile=t1, sort_interval=k1)
    t = TOL[prec]
    best, ns = s0.autotune([(4, 8, 2), (2, 2, 1), (8, 4, 3)], steps=2)
    assert best in [(4, 8, 2), (2, 2, 1), (8, 4, 3)] and ns > 0
    n0 = s0.counts()["step"]
    _say("autotune", prec, best, ns, "steps", n0)
    assert n0 == (1 + 2) + (1 + 2) + (1 + 3)
    # the oracle run alongside over the autotuning's steps: reported, and
    # held only to a gross-error bound (its difference holds the reordered
    # floating-point atomics of every step); the per-step bar follows
    o0.step(n0)
    rep = {}
    compare_fields(o0, s0, 1e-2, report=rep)
    _say(f"  {prec} after autotuning, run alongside from step 0 (reported): worst field {max(rep.values()):.2e}")
    # then every step from identical input bits, retiled and batched
    b = Batch([s0, s1])
    for k in range(4):
        if k == 2:
            s1.set_sort(2, 16, 1)
        o0, o1 = oracle_from_sim(s0, p0), oracle_from_sim(s1, p1)
        before = [s0.particles(), s1.particles()]
        b.step(1)
        for r, (p, o, s) in enumerate(((p0, o0, s0), (p1, o1, s1))):
            o.step(1)
            compare_fields(o, s, t["field"])
            compare_particles(o, s, t, p["nth"], t["band"], before=before[r])
