"""The Gauss-law residual on the GPU (Sec. 2 eq. (maxti), App. B eq.
(multfiltcharge)) against the FP64 oracle, through the C ABI.

G (the closed-surface flux of E out of every dual cell) and Qbar (the
filtered bilinear node charge) are compared element by element with the
oracle's on the same state: particles scattered over a grid wider than 64
cells before any sort (every span of the node-charge kernel too wide for its
LDS window: the global-memory path) and after a sorted step (the LDS path),
with particles on both poles and inside both conductors.  Both sides form
them in FP64 from identical inputs (an FP32 context's E, offsets and weights
are exact in FP64), so the bar is 1e-12 of the quantity's scale in both
precisions.  The device reductions (PIC_MOM_GAUSS_RES) are checked against
the same reductions of the oracle's planes, a non-finite field must come back
as PIC_ENAN, and the drift over 100 steps stays at roundoff in FP64."""
import sys

import numpy as np
import pytest

from paper_1407_1810_amd import workloads as W
from parity_util import oracle_from_sim, random_fields

pytestmark = pytest.mark.gpu

PRECISIONS = ["fp64", "fp32"]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    from paper_1407_1810_amd.binding import gpu_available, lib
    if not gpu_available():
        pytest.skip("no HIP device")
    lib()


def _state(prec, nr=96, nth=80, n_filt=3):
    """A plasma of pairs, a quarter of them unpaired (so that Qbar is not
    zero), particles exactly on both poles and inside both conductors, and
    random E and B; the sort tile is 4 x 4, every step sorts."""
    from oracle.oracle import Oracle
    from paper_1407_1810_amd.binding import Sim
    cfg = W.small_config(nr=nr, nth=nth, pairs_per_cell=2, n_filt=n_filt, absorb_cells=6, theta_T=0.2)
    p = cfg["params"]
    P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    P["x"][1::4] = np.clip(P["x"][1::4] + 0.37, 0.0, p["nr"] - 1e-9)
    n = len(P["x"])
    # poles and conductors: y exactly 0 and nth, x in the ghost rows
    k = np.arange(0, 64)
    P["y"][k[:16]] = 0.0
    P["y"][k[16:32]] = float(nth)
    P["x"][k[32:48]] = -1.0 - 0.5 * np.linspace(0, 1, 16) * (n_filt)
    P["x"][k[48:64]] = nr + 0.25 + 0.5 * np.linspace(0, 1, 16) * (n_filt)
    flds = random_fields(Oracle(p), np.random.default_rng(7), scale=2e-3)
    s = Sim(p, precision=prec, capacity=n + (1 << 16), tile=(4, 4), sort_interval=1)
    s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
    for comp, a in flds.items():
        s.set_field(comp, a)
    return p, s


def _abs_charge(o, p):
    """Unfiltered absolute node charge of the oracle's particles, by the
    oracle's own node-charge routine."""
    P = o.particles()
    rho = None
    for x, y, w in zip(P["x"], P["y"], P["w"]):
        rho = o.node_charge(x, y, abs(w), rho)
    g = o.g
    return rho[g:g + p["nr"] + 1]


def _check_planes(o, s, p, label):
    Go, Qo = o.gauss()
    Gs, Qs = s.gauss()
    gsc = np.abs(Go).max()
    A = _abs_charge(o, p)
    qsc = np.abs(A).max()
    eg = np.abs(Gs - Go).max() / gsc
    eq = np.abs(Qs - Qo).max() / qsc
    _say(f"{label}: G {eg:.2e} of max|G| {gsc:.3e}, Qbar {eq:.2e} of the charge scale {qsc:.3e}")
    assert gsc > 0 and qsc > 0
    assert eg <= 1e-12 and eq <= 1e-12
    # the node charge reaches both poles
    assert np.abs(Qo[:, 0]).max() > 0 and np.abs(Qo[:, -1]).max() > 0
    # the node-charge moment is the second half of the Gauss planes (up to
    # the order of the FP64 atomics that join the spans)
    assert np.abs(s.rho_q() - Qs).max() <= 1e-13 * qsc
    return Go, Qo, A


def _check_reductions(res, Go, Qo, A, p, R0):
    # the nodes below the lossy layer, whose E the layer leaves alone
    rows = slice(1, p["nr"] - p["absorb_cells"])
    R = (Go - Qo)[rows]
    D = R - R0[rows]
    sc_r = max(np.abs(Go[rows]).max(), np.abs(A[rows]).max())
    assert res["nodes"] == (p["nr"] - 1 - p["absorb_cells"]) * (p["nth"] + 1)
    assert res["non_finite"] == 0
    assert res["res_max"] == pytest.approx(np.abs(R).max(), abs=1e-12 * sc_r)
    assert res["res_l2"] == pytest.approx(np.sqrt((R ** 2).sum()), abs=1e-12 * sc_r * np.sqrt(R.size))
    assert res["abs_charge_max"] == pytest.approx(np.abs(A[rows]).max(), rel=1e-12)
    assert res["flux_max"] == pytest.approx(np.abs(Go[rows]).max(), rel=1e-12)
    assert res["drift_max"] == pytest.approx(np.abs(D).max(), abs=1e-12 * sc_r)
    assert res["drift_l2"] == pytest.approx(np.sqrt((D ** 2).sum()), abs=1e-12 * sc_r * np.sqrt(R.size))


@pytest.mark.parametrize("prec", PRECISIONS)
def test_gauss_planes_and_reductions_match_the_oracle(prec):
    p, s = _state(prec)
    # before any step: the generator's shuffled order (global-memory path)
    o = oracle_from_sim(s, p)
    res0 = s.gauss_residual()
    Go, Qo, A = _check_planes(o, s, p, f"{prec} unsorted")
    R0 = Go - Qo
    assert res0["drift_max"] == 0.0 and res0["ref_step"] == 0
    _check_reductions(res0, Go, Qo, A, p, R0)
    # one sorted step (LDS path), then the drift against the first residual
    s.step(1)
    o = oracle_from_sim(s, p)
    Go, Qo, A = _check_planes(o, s, p, f"{prec} sorted")
    res1 = s.gauss_residual()
    _check_reductions(res1, Go, Qo, A, p, R0)
    assert res1["ref_step"] == 0
    _say(f"{prec}: drift after one step {res1['drift_max']:.3e} of the charge scale {res1['abs_charge_max']:.3e}")


def test_non_finite_values_are_reported():
    """A NaN or an infinity in E reaches the flux of its dual cells: the
    device reduction counts it and the call returns PIC_ENAN (after writing
    its output); the luminosity reduction does the same.  Restoring a finite
    field clears the condition."""
    from paper_1407_1810_amd.binding import PicError
    for prec in PRECISIONS:
        p, s = _state(prec, nr=40, nth=32, n_filt=2)
        s.gauss_residual()
        Er = s.get_field("Er")
        bad = Er.copy()
        bad[10, 7] = np.nan
        bad[20, 3] = np.inf
        s.set_field("Er", bad)
        for call in (s.gauss_residual, s.gauss):
            with pytest.raises(PicError) as e:
                call()
            assert e.value.code == -5
        Eth = s.get_field("Eth")
        s.set_field("Er", Er)
        s.set_field("Eth", np.where(np.arange(Eth.shape[0])[:, None] == 12, np.nan, Eth))
        with pytest.raises(PicError) as e:
            s.luminosity()
        assert e.value.code == -5
        s.set_field("Eth", Eth)
        res = s.gauss_residual()
        assert res["non_finite"] == 0 and np.isfinite(s.luminosity()).all()


@pytest.mark.parametrize("prec", PRECISIONS)
def test_gauss_drift_over_100_steps(prec):
    """Charge conservation on the GPU, from the device's own FP64 reduction:
    the residual's drift over 100 steps stays at roundoff against the
    absolute node charge -- FP64 within 1e-12, FP32 within the rounding of
    the FP32-stored E (1e-5)."""
    cfg = W.small_config(nr=40, nth=32, pairs_per_cell=4, n_filt=3, absorb_cells=5, theta_T=0.3)
    p = cfg["params"]
    P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    P["x"][1::2] = np.clip(P["x"][1::2] + 0.37, 0, p["nr"] - 1e-9)
    from paper_1407_1810_amd.binding import Sim
    s = Sim(p, precision=prec, capacity=len(P["x"]) + 10)
    s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
    r0 = s.gauss_residual()
    s.step(100)
    r = s.gauss_residual()
    _say(f"{prec}: drift {r['drift_max']:.3e} (L2 {r['drift_l2']:.3e}), absolute charge {r['abs_charge_max']:.3e}")
    assert r0["drift_max"] == 0.0 and r["ref_step"] == 0
    bound = 1e-12 if prec == "fp64" else 1e-5
    assert r["drift_max"] <= bound * r["abs_charge_max"]
