"""The Michel monopole on the GPU (Sec. 5.4): the 512 x 512 monopole
rotator (r_out = 12 r_in, R_l = 3 r_in, spin-up over 1/Omega, surface
injection sized as in the benchmark workload) run in FP32 and in FP64 (the
workload's own precision) for two rotation periods (about 19,300 steps)
through the library.  Checked inside the light
cylinder, at 0.35, 0.5 and 0.7 R_l:
  * the winding B_phi / B_r = -r sin(theta) / R_l: the median over the
    latitudes away from the poles (the polar eighths excluded) of the ratio
    to Michel's within 8 %;
  * the Poynting luminosity through the sphere within 8 % of
    L_0 = (8 pi / 3) c (B0 r_in^2 / R_l)^2 (Lorentz-Heaviside units; the
    paper quotes about 1 % for its 1024 x 512 run);
  * E_theta = B_phi: the median over the same latitudes of their ratio
    within 12 %.
The equatorial row alone is not gated: it sits in the current sheet, and
its winding and E_theta / B_phi fluctuate by 10-40 % between periods and
between runs that differ only in floating-point order (measured)."""
import math
import sys
import time

import numpy as np
import pytest

from paper_1407_1810_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=["fp32", "fp64"])
def michel_gpu(request):
    from paper_1407_1810_amd.binding import Sim, gpu_available
    if not gpu_available():
        pytest.skip("no HIP device")
    cfg = W.config(1)
    p = cfg["params"]
    prec = request.param
    s = Sim(p, precision=prec, capacity=64 << 20, ids=False, tile=(4, 8), sort_interval=8)
    Rl = p["c"] / p["omega"]
    nsteps = int(2.0 * 2.0 * math.pi / p["omega"])
    t0 = time.time()
    done = 0
    while done < nsteps:
        k = min(2000, nsteps - done)
        s.step(k)
        done += k
        _say(f"michel 512 {prec}: step {done}/{nsteps}, {s.counts()['live']} particles, {time.time() - t0:.0f} s")
    fields = {c: s.get_field(c) for c in ("Er", "Eth", "Eph", "Br", "Bth", "Bph")}
    geo_rb = p["r_in"] * np.exp((np.arange(p["nr"]) + 0.5) * math.log(p["r_out"] / p["r_in"]) / p["nr"])
    geo_rn = p["r_in"] * np.exp(np.arange(p["nr"] + 1) * math.log(p["r_out"] / p["r_in"]) / p["nr"])
    s.close()
    return p, Rl, fields, geo_rb, geo_rn, prec


def _sb(nth):
    yb = np.arange(nth) + 0.5
    return np.sqrt(1.0 - (1.0 - 2.0 * yb / nth) ** 2)


def _metrics(p, Rl, f, rb, rn, frac):
    nth, r0, c = p["nth"], p["r_in"], p["c"]
    sb = _sb(nth)
    i = int(np.searchsorted(rb, frac * Rl))
    ri = rb[i]
    br = p["B0"] * (r0 / ri) ** 2 + 0.5 * (f["Br"][i] + f["Br"][i + 1])
    ratio = f["Bph"][i] / br / (-ri * sb / Rl)
    lat = float(np.median(ratio[nth // 8: -nth // 8]))
    eth_c = 0.5 * (f["Eth"][i] + f["Eth"][i + 1]) - p["B0"] * r0 * (r0 / ri) ** 3 * (p["omega"] / c) * sb
    eph = 0.25 * (f["Eph"][i, :-1] + f["Eph"][i, 1:] + f["Eph"][i + 1, :-1] + f["Eph"][i + 1, 1:])
    bth = 0.5 * (f["Bth"][i, :-1] + f["Bth"][i, 1:])
    L = float((c * (eth_c * f["Bph"][i] - eph * bth) * 2.0 * math.pi * ri * ri * (2.0 / nth)).sum())
    L0 = 8.0 * math.pi / 3.0 * c * (p["B0"] * r0 * r0 / Rl) ** 2
    e_over_b = float(np.median((eth_c / f["Bph"][i])[nth // 8: -nth // 8]))
    return lat, L / L0, e_over_b, float(ratio[nth // 2])


@pytest.mark.parametrize("frac", [0.35, 0.5, 0.7])
def test_michel_inside_the_light_cylinder(michel_gpu, frac):
    p, Rl, f, rb, rn, prec = michel_gpu
    lat, lum, e_over_b, eq = _metrics(p, Rl, f, rb, rn, frac)
    _say(f"{prec}, r = {frac} R_l: winding / Michel median {lat:.4f} (equator {eq:.4f}), L / L0 {lum:.4f}, "
         f"E_theta / B_phi {e_over_b:.4f}")
    assert abs(lat - 1.0) < 0.08
    assert abs(lum - 1.0) < 0.08
    assert abs(e_over_b - 1.0) < 0.12
