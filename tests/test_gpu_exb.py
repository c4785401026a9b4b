"""The E x B drift test of Sec. 4.3 on the GPU, as a sweep over omega_c dt:
a test particle at rest on the equator at 3 r0 in the dipole field with the
corotation electric field everywhere (r0 / R_l = 0.05) must drift at the
corotation speed 3 Omega r0 = 0.15 c.  The paper's result: the Vay mover
captures the drift for any omega_c dt, the Boris mover only while the
gyration is resolved and drifts wrongly for omega_c dt >~ 2.  Measured here:
Vay within 2% from omega_c dt = 0.25 to 16 (0.3% from 4 on); Boris within
2.3% up to 2, then 4%, 15% and 49% off at 4, 8 and 16.  Each case is also run by the
oracle on the same input (FP64: the same drift to 1e-9) and in FP32 (a test
particle of weight 1e-30)."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SWEEP = [0.25, 0.5, 1.0, 2.0, 4.0, 8.0, 16.0]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _params(mover, wc_dt):
    nr, nth, ratio = 32, 16, 5.0
    dxi = math.log(ratio) / nr
    r_in = 1.0 / dxi
    c = 0.5 * min(r_in * (math.exp(dxi) - 1.0), r_in * 2.0 / nth)
    p = dict(nr=nr, nth=nth, r_in=r_in, r_out=r_in * ratio, r_kind="log", th_kind="eqarea", c=c, n_filt=0,
             absorb_cells=0, sigma_max=0.0, mover=mover, bg_kind="dipole_corot", B0=1.0)
    p["omega"] = 0.05 * c / r_in
    p["q_over_m"] = wc_dt * c * 27.0 / p["B0"]  # B = B0 / 27 at 3 r0 on the equator
    return p


def _drift(sim, p, w):
    """<v_phi> over 600 steps after 3000, in units of 3 Omega r0."""
    x0 = math.log(3.0) / (math.log(5.0) / p["nr"])
    sim.add_particles([x0], [8.0], [0.0], [0.0], [0.0], [w])
    sim.step(3000)
    acc = []
    for _ in range(600):
        sim.step(1)
        P = sim.particles()
        u = np.array([P["ur"][0], P["ut"][0], P["up"][0]])
        acc.append(P["up"][0] / math.sqrt(1.0 + u @ u) * p["c"])
    return abs(np.mean(acc)) / (3.0 * p["omega"] * p["r_in"])


@pytest.fixture(scope="module")
def sweep():
    from oracle.oracle import Oracle
    from paper_1407_1810_amd.binding import Sim, gpu_available
    if not gpu_available():
        pytest.skip("no HIP device")
    out = {}
    for mover in ("vay", "boris"):
        for wc in SWEEP:
            p = _params(mover, wc)
            g64 = _drift(Sim(p, precision="fp64", capacity=1024), p, 1e-200)
            # an FP32 weight small enough to leave the fields untouched
            g32 = _drift(Sim(p, precision="fp32", capacity=1024), p, 1e-30)
            ora = _drift(Oracle(p), p, 1e-200)
            out[(mover, wc)] = (g64, g32, ora)
            _say(f"{mover:5s} omega_c dt = {wc:5.2f}: drift / corotation  GPU FP64 {g64:.4f}  FP32 {g32:.4f}  "
                 f"oracle {ora:.4f}")
    return out


@pytest.mark.parametrize("wc", SWEEP)
def test_vay_drifts_at_any_omega_c_dt(sweep, wc):
    g64, g32, ora = sweep[("vay", wc)]
    assert g64 == pytest.approx(ora, abs=1e-9)
    assert abs(g64 - 1.0) < 0.03 and abs(g32 - 1.0) < 0.03


def test_boris_fails_once_gyration_is_unresolved(sweep):
    for wc in SWEEP:
        g64, g32, ora = sweep[("boris", wc)]
        assert g64 == pytest.approx(ora, abs=1e-9)
        assert g32 == pytest.approx(g64, abs=0.01)
    err = {wc: abs(sweep[("boris", wc)][0] - 1.0) for wc in SWEEP}
    vay = {wc: abs(sweep[("vay", wc)][0] - 1.0) for wc in SWEEP}
    # resolved gyration: the drift within 3% (both movers read about 2% high
    # at the smallest steps, where 600 steps do not average the gyration
    # out); past omega_c dt = 2 Boris' error grows with the step (measured
    # 4%, 15%, 49% at 4, 8, 16) while Vay's stays below 0.5%
    assert all(err[wc] < 0.03 for wc in SWEEP if wc <= 2.0)
    assert err[4.0] > 3.0 * vay[4.0] and err[4.0] > 0.03
    assert err[8.0] > 0.1 and err[16.0] > 0.3
    assert err[4.0] < err[8.0] < err[16.0]
    assert all(vay[wc] < 0.03 for wc in SWEEP)
    assert all(vay[wc] < 0.005 for wc in SWEEP if wc >= 4.0)
