"""Seeded synthetic workloads: simulation parameters and initial particles.

This module is shared by the GPU path's tests/bench and by the CPU oracle's
tests.  It only draws inputs (positions, momenta, weights) and chooses
parameter values; it performs none of the method's arithmetic.

Code units (the paper's TRISTAN convention, Table 1 and Sec. 5.4): dt = 1,
lengths are such that the first radial cell at the inner conductor is about
one unit wide, c is the Courant number in length units per step.

Input recipe (all seeded through numpy's Philox bit generator):
  * positions: uniform in each cell, in grid coordinates;
  * pairs: an electron and a positron at the same position (zero net
    charge, so zero initial plasma field is self-consistent);
  * momenta: isotropic Maxwell-Juttner at temperature theta_T, each
    particle independently, by inverse transform of the tabulated CDF;
  * weights: uniform magnitude chosen so that omega_p dt = 0.1 in the
    densest (innermost) cell;
  * q/m chosen so that omega_c dt = 2 at the inner conductor.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["grid_params", "config", "CONFIGS", "pair_plasma", "mj_momenta", "small_config"]


def grid_params(nr: int, nth: int, r_ratio: float, courant: float = 0.5, r_kind: str = "log",
                th_kind: str = "eqarea") -> dict:
    """Conductor radii and light speed for an nr x nth grid spanning
    r_out / r_in = r_ratio.  The radial unit is chosen so that the first
    radial cell is one unit wide; c is `courant` times the smallest cell
    edge at the inner conductor (radial, or the equatorial meridional one)."""
    if r_kind == "log":
        dxi = math.log(r_ratio) / nr
        r_in = 1.0 / dxi
        dr0 = r_in * (math.exp(dxi) - 1.0)
    else:
        r_in = float(nr) / (r_ratio - 1.0)
        dr0 = 1.0
    r_out = r_in * r_ratio
    dth = r_in * (2.0 / nth if th_kind == "eqarea" else math.pi / nth)
    c = courant * min(dr0, dth)
    return dict(nr=nr, nth=nth, r_in=r_in, r_out=r_out, r_kind=r_kind, th_kind=th_kind, c=c)


def _inner_cell_volume(p: dict) -> float:
    """Volume of the smallest (innermost) cell: only used to size weights."""
    if p["r_kind"] == "log":
        r1 = p["r_in"] * (p["r_out"] / p["r_in"]) ** (1.0 / p["nr"])
    else:
        r1 = p["r_in"] + (p["r_out"] - p["r_in"]) / p["nr"]
    dcos = 2.0 / p["nth"] if p["th_kind"] == "eqarea" else 1.0 - math.cos(math.pi / p["nth"])
    return 2.0 * math.pi / 3.0 * (r1 ** 3 - p["r_in"] ** 3) * dcos


def plasma_weight(p: dict, particles_per_cell: float, omega_p_dt: float = 0.1) -> float:
    """|w| such that omega_p^2 = n |w| (q/m) = omega_p_dt^2 in the innermost cell."""
    vol = _inner_cell_volume(p)
    return omega_p_dt ** 2 * vol / (particles_per_cell * p["q_over_m"])


def mj_momenta(rng: np.random.Generator, n: int, theta: float):
    """Isotropic Maxwell-Juttner momenta u = gamma v / c, density
    u^2 exp(-gamma / theta), by inverse transform of a tabulated CDF."""
    umax = math.sqrt((1.0 + 60.0 * theta) ** 2 - 1.0)
    grid = np.linspace(0.0, umax, 40001)
    pdf = grid ** 2 * np.exp(-(np.sqrt(1.0 + grid ** 2) - 1.0) / theta)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
    cdf /= cdf[-1]
    umag = np.interp(rng.random(n), cdf, grid)
    mu = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    st = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return umag * mu, umag * st * np.cos(ph), umag * st * np.sin(ph)


def _pair_chunk(out, lo, hi, p, pairs_per_cell, theta_T, weight, seed, chunk_id, i0, nj):
    """Fill pairs lo..hi-1 (pair index) of the output arrays; the chunk has
    its own Philox key so the result does not depend on how chunks are
    scheduled."""
    rng = np.random.Generator(np.random.Philox(key=[seed, chunk_id + 1]))
    m = hi - lo
    cells = np.arange(lo, hi, dtype=np.int64) // pairs_per_cell
    cells = cells[rng.permutation(m)]
    xp = (i0 + cells // nj) + rng.random(m)
    yp = (cells % nj) + rng.random(m)
    a, b = 2 * lo, 2 * hi
    out["x"][a:b:2] = xp
    out["x"][a + 1:b:2] = xp
    out["y"][a:b:2] = yp
    out["y"][a + 1:b:2] = yp
    if theta_T > 0:
        ur, ut, up = mj_momenta(rng, 2 * m, theta_T)
        out["ur"][a:b] = ur
        out["ut"][a:b] = ut
        out["up"][a:b] = up
    else:
        out["ur"][a:b] = 0.0
        out["ut"][a:b] = 0.0
        out["up"][a:b] = 0.0
    out["w"][a:b:2] = weight
    out["w"][a + 1:b:2] = -weight
    out["id"][a:b] = np.arange(a, b, dtype=np.uint64)


def pair_plasma(p: dict, pairs_per_cell: int, theta_T: float, weight: float, seed: int,
                i_range=None, j_range=None, chunk_pairs: int = 1 << 20, threads: int | None = None) -> dict:
    """Co-located electron/positron pairs (positron first), positions uniform
    in each cell of rows i_range x columns j_range (default: the whole grid),
    momenta Maxwell-Juttner; cell order is shuffled within each chunk of
    `chunk_pairs` pairs.  Returns float64 arrays x, y, ur, ut, up, w and
    uint64 id = array index."""
    import concurrent.futures as cf
    import os
    i0, i1 = i_range if i_range else (0, p["nr"])
    j0, j1 = j_range if j_range else (0, p["nth"])
    ni, nj = i1 - i0, j1 - j0
    npair = ni * nj * pairs_per_cell
    n = 2 * npair
    out = {k: np.empty(n) for k in ("x", "y", "ur", "ut", "up", "w")}
    out["id"] = np.empty(n, dtype=np.uint64)
    if j0 != 0:
        raise ValueError("j_range must start at 0")
    # chunks of whole cells
    per = max(pairs_per_cell, (chunk_pairs // max(pairs_per_cell, 1)) * max(pairs_per_cell, 1))
    bounds = [(lo, min(lo + per, npair)) for lo in range(0, npair, per)]
    if threads is None:
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
    args = [(out, lo, hi, p, pairs_per_cell, theta_T, weight, seed, k, i0, nj) for k, (lo, hi) in enumerate(bounds)]
    if threads == 1 or len(args) == 1:
        for a in args:
            _pair_chunk(*a)
    else:
        with cf.ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda a: _pair_chunk(*a), args))
    return out


def _rotator(nr, nth, bg, pairs_per_cell, steps, absorb_frac=0.1, inject=1, n_filt=3, seed=0,
             r_ratio=12.0, r_lc_over_rin=3.0, wc_dt=2.0, theta_T=0.1, q_inj_scale=1.0):
    p = grid_params(nr, nth, r_ratio)
    p.update(n_filt=n_filt, absorb_cells=max(10, int(round(absorb_frac * nr))), mover="vay",
             bg_kind=bg, B0=1.0, seed=seed)
    p["sigma_max"] = 2.0 / p["absorb_cells"]
    p["q_over_m"] = wc_dt * p["c"] / p["B0"]
    p["omega"] = p["c"] / (r_lc_over_rin * p["r_in"])
    p["t_spin"] = 1.0 / p["omega"]
    ppc = max(2 * pairs_per_cell, 16)
    w = plasma_weight(p, ppc)
    p.update(inject=inject, f_inj=0.5, q_inj=w * q_inj_scale)
    return dict(params=p, pairs_per_cell=pairs_per_cell, theta_T=theta_T, weight=w, steps=steps, seed=seed)


def config(k: int) -> dict:
    """The five benchmark workloads (plain FP64 method, monopole rotator,
    dipole rotator, precision stress, batched ensemble)."""
    if k == 0:
        p = grid_params(64, 64, 10.0)
        p.update(n_filt=3, absorb_cells=10, sigma_max=0.2, mover="vay", bg_kind="monopole", B0=1.0,
                 omega=0.0, t_spin=0.0, inject=0, f_inj=0.0, seed=0)
        p["q_over_m"] = 2.0 * p["c"] / p["B0"]
        w = plasma_weight(p, 32)
        p["q_inj"] = w
        return dict(name="plain_fp64_64x64", params=p, pairs_per_cell=16, theta_T=0.1, weight=w,
                    steps=100, seed=0)
    if k == 1:
        d = _rotator(512, 512, "monopole", 0, 2000)
        _size_injection(d, 2000, target=16_000_000)
        d["name"] = "monopole_rotator_512x512"
        return d
    if k == 2:
        d = _rotator(1024, 1024, "dipole", 32, 1000)
        _size_injection(d, 1000)
        d["name"] = "dipole_rotator_1024x1024_ppc64"
        return d
    if k == 3:
        d = _rotator(2048, 2048, "dipole", 24, 5000)
        _size_injection(d, 5000)
        d["name"] = "precision_stress_2048x2048_ppc48"
        return d
    if k == 4:
        return dict(name="batched_ensemble_64_runs", runs=batched_runs(), steps=200, warmup=50)
    raise KeyError(k)


def table1_monopole(target_particles: float = 2e7, wc_dt: float = 20.0, seed: int = 0) -> dict:
    """The aligned monopole rotator of the paper's Table 1 (Sec. 5.4): 1024 x
    512 cells, log radius from r0 = 256 to e^4 r0 (about 54 r0), equal-area
    theta, light cylinder 5 r0, c = 0.6, two rotation periods (26,808
    steps), Omega spun up over half a period, 3 filter passes, f_inj = 0.5,
    Vay mover, surface injection from an empty start, about 2e7 particles at
    the end.  Not in the table, ours: the lossy layer over the outer 10% of
    the cells (from 36.6 r0, past the 25 r0 the paper plots); omega_c dt = 20
    at the surface, so that the Larmor radius there is below a cell for the
    energies the particles reach (the paper's condition for its Vay mover);
    the injected macro-charge.  The surface-charge estimate of the count
    assumes a field at the star that the plasma never screens; the count
    measured at the end of this run is about 1/30 of it, hence the factor."""
    p = grid_params(1024, 512, math.exp(4.0), courant=0.6)
    p.update(n_filt=3, absorb_cells=102, sigma_max=2.0 / 102, mover="vay", bg_kind="monopole", B0=1.0, seed=seed)
    p["q_over_m"] = wc_dt * p["c"] / p["B0"]
    p["omega"] = p["c"] / (5.0 * p["r_in"])
    period = 2.0 * math.pi / p["omega"]
    p["t_spin"] = 0.5 * period
    w = plasma_weight(p, 16)
    p.update(inject=1, f_inj=0.5, q_inj=w)
    steps = int(round(2.0 * period))
    d = dict(name="table1_monopole_1024x512", params=p, pairs_per_cell=0, theta_T=0.1, weight=w, steps=steps,
             seed=seed)
    _size_injection(d, steps, target=30.0 * target_particles)
    return d


def injection_scale_estimate(p: dict, q: float, window: int) -> float:
    """Order-of-magnitude count of macro-particles a rotator releases from
    its surface over `window` steps with macro-charge q: the surface charge
    scale B0 r_in Omega / c over the sphere 4 pi r_in^2, with Omega rising
    linearly over t_spin.  Used only to size workloads."""
    n1 = 4.0 * np.pi * p["B0"] * p["r_in"] ** 3 * p["omega"] / (p["c"] * q)
    ts = p["t_spin"]
    ramp = window - window * window / (2.0 * ts) if window < ts else window - 0.5 * ts
    return float(n1 * ramp)


def _size_injection(d: dict, window: int, target: float | None = None) -> None:
    """Raise the injected macro-charge of a rotator workload (never below the
    plasma weight) so that the surface-charge estimate over `window` steps
    comes to `target` particles, by default half the preloaded count."""
    p = d["params"]
    n0 = p["nr"] * p["nth"] * 2 * d["pairs_per_cell"]
    want = target if target is not None else 0.5 * n0
    scale = max(1.0, injection_scale_estimate(p, d["weight"], window) / want)
    p["q_inj"] = d["weight"] * scale


def batched_runs(n_runs: int = 64, seed: int = 0, window: int = 350):
    """Uneven rotator runs: square grids 128..512 (steps of 64), Omega in
    [0.1, 0.5] c/R*, r in [1, 4 R_LC], 16..64 particles per cell, monopole and
    dipole alternating; the run index is its seed.  The injected macro-charge
    of each run is raised (never lowered below the plasma weight) until the
    surface-charge estimate over `window` steps is half the preloaded count,
    so that every run stays a preloaded run with injection on top."""
    rng = np.random.Generator(np.random.Philox(seed + 12345))
    runs = []
    for k in range(n_runs):
        n = int(rng.choice(np.arange(128, 513, 64)))
        om = float(rng.uniform(0.1, 0.5))  # in c / R*
        r_lc = 1.0 / om                   # R_LC in R*
        ppc = int(rng.choice([16, 32, 48, 64]))
        bg = "monopole" if k % 2 == 0 else "dipole"
        d = _rotator(n, n, bg, ppc // 2, 0, r_ratio=4.0 * r_lc, r_lc_over_rin=r_lc, seed=k)
        _size_injection(d, window)
        d["name"] = f"run{k}_{bg}_{n}x{n}_ppc{ppc}"
        runs.append(d)
    return runs


def small_config(nr=24, nth=20, pairs_per_cell=3, bg="monopole", omega_frac=0.0, inject=0, n_filt=2,
                 absorb_cells=4, theta_T=0.1, seed=7, r_ratio=6.0, mover="vay", r_kind="log",
                 th_kind="eqarea", wc_dt=2.0):
    """A small grid for oracle pins and GPU parity cases (several tiles and a
    ragged tail for any tile shape the GPU path uses)."""
    p = grid_params(nr, nth, r_ratio, r_kind=r_kind, th_kind=th_kind)
    p.update(n_filt=n_filt, absorb_cells=absorb_cells, sigma_max=2.0 / max(1, absorb_cells), mover=mover,
             bg_kind=bg, B0=1.0, seed=seed)
    p["q_over_m"] = wc_dt * p["c"] / p["B0"]
    p["omega"] = omega_frac * p["c"] / p["r_in"]
    p["t_spin"] = 0.0
    w = plasma_weight(p, max(2 * pairs_per_cell, 2))
    p.update(inject=inject, f_inj=0.5, q_inj=w)
    return dict(name=f"small_{nr}x{nth}", params=p, pairs_per_cell=pairs_per_cell, theta_T=theta_T, weight=w,
                steps=10, seed=seed)


CONFIGS = [0, 1, 2, 3, 4]
