"""Pin of the whole oracle step against the paper's monopole test (Sec. 5.4):
a conducting sphere with a monopole field, spun up to Omega and filled by
surface injection, relaxes to Michel's force-free wind, in which the field
lines wind up as B_phi / B_r = -r sin(theta) / R_l and the field is
E_theta = B_phi inside the light cylinder R_l = c / Omega.

The check runs a log-r, equal-area grid (r_out = 12 r_in, R_l = 3 r_in,
spin-up time 1/Omega) for two rotation periods, at 48 x 48 and at 96 x 96
cells.  The paper shows the agreement only in figures (and quotes about 1 %
for the luminosity of its far finer runs), so the bounds are ours, set from
what each resolution reaches: at 0.35, 0.5 and 0.7 R_l the median over the
latitudes away from the poles of the winding's ratio to Michel's and of
E_theta / B_phi, and the Poynting luminosity through spheres at 0.35 and 0.5
R_l against Michel's L_0 = (8 pi / 3) c (B0 r_in^2 / R_l)^2
(Lorentz-Heaviside units).  At 48 x 48 (measured: winding 7-10 % low,
E_theta / B_phi 5-9 % high, L 11-13 % low) within 11 %, 11 % and 14 %; at
96 x 96 (measured: within 0.6 %, 1 % and 1.6 %) within 2.5 %, 2.5 % and 3 %:
the wind converges to Michel's as the grid is refined.
Every term of the step takes part (spin-up fields, injection, push,
deposit, filter, field update, lossy layer); switching the injection off
leaves no wound-up field at all, which the control case checks."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1407_1810_amd import workloads as W


def _run(inject=1, periods=2.0, n=48):
    O.set_threads(max(1, min(8, len(os.sched_getaffinity(0)))))
    d = W._rotator(n, n, "monopole", 0, 0, inject=inject)
    p = d["params"]
    o = O.Oracle(p)
    Rl = p["c"] / p["omega"]
    o.step(int(periods * 2 * math.pi / p["omega"]))
    return o, p, Rl


def _medians(o, p, Rl, frac):
    """Over the latitudes away from the poles (polar eighths excluded): the
    median ratio of the winding B_phi / B_r to Michel's, and of E_theta to
    B_phi, on the cell-centred row of radial half-nodes nearest frac R_l."""
    nth, r0, c = p["nth"], p["r_in"], p["c"]
    rb = o.geometry(1)
    Eth, Br, Bph = o.get_field("Eth"), o.get_field("Br"), o.get_field("Bph")
    yb = np.arange(nth) + 0.5
    sb = np.sqrt(1.0 - (1.0 - 2.0 * yb / nth) ** 2)
    i = int(np.searchsorted(rb, frac * Rl))
    r = rb[i]
    br = p["B0"] * (r0 / r) ** 2 + 0.5 * (Br[i] + Br[i + 1])
    wind = Bph[i] / br / (-r * sb / Rl)
    eth = 0.5 * (Eth[i] + Eth[i + 1]) - p["B0"] * r0 * (r0 / r) ** 3 * (p["omega"] / c) * sb
    q = slice(nth // 8, -nth // 8)
    return float(np.median(wind[q])), float(np.median((eth / Bph[i])[q]))


def _winding(o, p, Rl, frac):
    """B_phi / B_r (total) and E_theta / B_phi on the rows nearest frac R_l."""
    nth, r0 = p["nth"], p["r_in"]
    rb, rn = o.geometry(1), o.geometry(0)
    Bph, Br, Eth = o.get_field("Bph"), o.get_field("Br"), o.get_field("Eth")
    yb = np.arange(nth) + 0.5
    sth = np.sqrt(1.0 - (1.0 - 2.0 * yb / nth) ** 2)
    i = int(np.searchsorted(rb, frac * Rl))
    ri = rb[i]
    br = p["B0"] * (r0 / ri) ** 2 + 0.5 * (Br[i] + Br[i + 1])  # at (i + 1/2, j + 1/2)
    ratio = Bph[i] / br
    michel = -ri * sth / Rl
    k = int(np.searchsorted(rn, ri))
    rk = rn[k]
    # total E_theta at (k, j + 1/2): plasma part plus the vacuum exterior field
    eth = Eth[k] - p["B0"] * r0 * (r0 / rk) ** 3 * (p["omega"] / p["c"]) * sth
    bph = 0.5 * (Bph[k - 1] + Bph[k])
    with np.errstate(divide="ignore", invalid="ignore"):
        return ratio, michel, eth / bph


# grid cells -> bounds on the winding, on E_theta / B_phi and on L / L_0
BOUNDS = {48: (0.11, 0.11, 0.14), 96: (0.025, 0.025, 0.03)}


@pytest.fixture(scope="module", params=[48, 96])
def michel_run(request):
    return _run(n=request.param) + (BOUNDS[request.param],)


@pytest.mark.parametrize("frac", [0.35, 0.5, 0.7])
def test_field_winds_up_as_michel(michel_run, frac):
    o, p, Rl, bounds = michel_run
    wind, e_over_b = _medians(o, p, Rl, frac)
    ratio, michel, _ = _winding(o, p, Rl, frac)
    eq = p["nth"] // 2
    print(f"{p['nr']} cells, r = {frac} R_l: winding / Michel median {wind:.4f} "
          f"(equator {ratio[eq] / michel[eq]:.4f}), E_theta / B_phi median {e_over_b:.4f}")
    assert ratio[eq] < 0.0
    assert abs(wind - 1.0) < bounds[0]
    assert abs(e_over_b - 1.0) < bounds[1]


def _luminosity(o, p, Rl, frac):
    """Poynting flux c (E_th B_ph - E_ph B_th) through the sphere of radial
    half-nodes nearest frac R_l (total fields, cell-centred averages)."""
    nth, r0, c = p["nth"], p["r_in"], p["c"]
    rb = o.geometry(1)
    Eth, Eph = o.get_field("Eth"), o.get_field("Eph")
    Bth, Bph = o.get_field("Bth"), o.get_field("Bph")
    yb = np.arange(nth) + 0.5
    sb = np.sqrt(1.0 - (1.0 - 2.0 * yb / nth) ** 2)
    i = int(np.searchsorted(rb, frac * Rl))
    r = rb[i]
    eth = 0.5 * (Eth[i] + Eth[i + 1]) - p["B0"] * r0 * (r0 / r) ** 3 * (p["omega"] / c) * sb
    eph = 0.25 * (Eph[i, :-1] + Eph[i, 1:] + Eph[i + 1, :-1] + Eph[i + 1, 1:])
    bth = 0.5 * (Bth[i, :-1] + Bth[i, 1:])
    sr = c * (eth * Bph[i] - eph * bth)
    return float((sr * 2.0 * math.pi * r * r * (2.0 / nth)).sum())


def test_luminosity_is_michels(michel_run):
    o, p, Rl, bounds = michel_run
    L0 = 8.0 * math.pi / 3.0 * p["c"] * (p["B0"] * p["r_in"] ** 2 / Rl) ** 2
    for frac in (0.35, 0.5):
        L = _luminosity(o, p, Rl, frac)
        print(f"{p['nr']} cells, r = {frac} R_l: L / L0 = {L / L0:.4f}")
        assert abs(L / L0 - 1.0) < bounds[2]


def test_no_winding_without_plasma():
    """Control: without injection nothing carries current, so B_phi stays
    at the level of the spin-up transient, far below the wound-up field."""
    o, p, Rl = _run(inject=0, periods=0.5, n=32)
    ratio, michel, _ = _winding(o, p, Rl, 0.5)
    eq = p["nth"] // 2
    assert abs(ratio[eq]) < 0.1 * abs(michel[eq])
