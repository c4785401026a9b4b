"""GPU parity: the HIP library against the FP64 CPU oracle on the same
seeded inputs, through the C ABI.  Every test here needs an MI355X."""
import math
import sys

import numpy as np
import pytest

from paper_1407_1810_amd import workloads as W
from parity_util import (FIELD_COMPS, OWN_TOL_FP32, TOL, carry_atol, compare_fields, compare_particles, make_pair,
                         oracle_from_sim, oracles_from_sim, random_fields, round_to_storage, shifted_floor)

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


def _small(**kw):
    cfg = W.small_config(**kw)
    P = W.pair_plasma(cfg["params"], cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    return cfg, P


@pytest.mark.parametrize("prec", PRECISIONS)
def test_fields_only_one_and_five_steps(prec):
    """Field solver alone (random E, B satisfying the wall/axis conditions,
    lossy layer on, no particles)."""
    cfg = W.small_config(nr=37, nth=29, pairs_per_cell=0, absorb_cells=6)
    p = cfg["params"]
    from oracle.oracle import Oracle
    rng = np.random.default_rng(1)
    flds = random_fields(Oracle(p), rng)
    _say("fields-only", prec)
    o, s = make_pair(p, None, prec, fields=flds)
    for k in range(5):
        if k:
            o = oracle_from_sim(s, p)  # every step from identical input bits
        o.step(1)
        s.step(1)
        compare_fields(o, s, TOL[prec]["field"], comps=FIELD_COMPS)


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("nf", [0, 1, 3, 4, 5, 8])
def test_one_step_with_particles(prec, nf):
    """One full step from identical inputs: fields (E, B and the filtered
    face charges) and every particle, matched by id.  The pass counts reach
    every halo width the filter kernel is built for (2, 3, 4 and 8), up to the
    largest count the library accepts."""
    cfg, P = _small(nr=40, nth=36, pairs_per_cell=4, n_filt=nf, absorb_cells=5, theta_T=0.3)
    p = cfg["params"]
    # unpair half of the particles so that the plasma field is not zero
    P["x"][1::4] = np.clip(P["x"][1::4] + 0.41, 0.0, p["nr"] - 1e-9)
    _say("one-step", prec, nf, len(P["x"]))
    from oracle.oracle import Oracle
    flds = random_fields(Oracle(p), np.random.default_rng(2), scale=3e-3)
    o, s = make_pair(p, P, prec, fields=flds)
    o.step(1)
    s.step(1)
    t = TOL[prec]
    compare_fields(o, s, t["field"])
    compare_particles(o, s, t, p["nth"], t["band"])


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("r_kind,th_kind,mover,bg", [("lin", "lin", "boris", "dipole"), ("log", "lin", "vay", "dipole"),
                                                     ("lin", "eqarea", "boris", "monopole")])
def test_one_step_other_grids_and_boris(prec, r_kind, th_kind, mover, bg):
    """One full step as above on the other mesh options of Sec. 3.2 (uniform
    radius, uniform angle) and with the Boris mover: the push's radius,
    angle and displacement formulas for each option, both hemispheres of
    the uniform-angle mesh, and the second mover."""
    cfg, P = _small(nr=36, nth=40, pairs_per_cell=4, n_filt=2, absorb_cells=5, theta_T=0.3, r_kind=r_kind,
                    th_kind=th_kind, mover=mover, bg=bg)
    p = cfg["params"]
    P["x"][1::4] = np.clip(P["x"][1::4] + 0.41, 0.0, p["nr"] - 1e-9)
    _say("one-step-grid", prec, r_kind, th_kind, mover, bg, len(P["x"]))
    from oracle.oracle import Oracle
    flds = random_fields(Oracle(p), np.random.default_rng(5), scale=3e-3)
    o, s = make_pair(p, P, prec, fields=flds)
    o.step(1)
    s.step(1)
    t = TOL[prec]
    compare_fields(o, s, t["field"])
    compare_particles(o, s, t, p["nth"], t["band"])


@pytest.mark.parametrize("prec", PRECISIONS)
def test_lds_and_global_paths_and_sort(prec):
    """Same result with the chunk staged in LDS (after a sort) and with the
    global-memory path (no sort: chunks of scattered particles)."""
    cfg, P = _small(nr=48, nth=40, pairs_per_cell=6, n_filt=2)
    p = cfg["params"]
    res = {}
    t = TOL[prec]
    for si in (1, -1):
        o, s = make_pair(p, P, prec, sort_interval=si, tile=(4, 4))
        for k in range(3):
            if k > 0:
                o = oracle_from_sim(s, p)
            o.step(1)
            s.step(1)
            compare_fields(o, s, t["field"])
            compare_particles(o, s, t, p["nth"], t["band"])
        res[si] = s.get_field("Er")
    # the two paths after three steps, run on from the same start (reported
    # scale: the reordered floating-point atomics of three steps)
    d = np.abs(res[1] - res[-1]).max() / np.abs(res[1]).max()
    _say(f"{prec}: sorted (LDS) and unsorted (global) paths differ by {d:.2e} after three steps")
    assert d <= 1e3 * t["field"]


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("ppt", [4, 16])
def test_capacity_equal_to_count_ragged_chunks(prec, ppt):
    """Capacity exactly the particle count, which is no multiple of a push
    chunk (256 x particles per thread): the lanes of the last chunk past the
    count load and store in the spare slots past the capacity and leave the
    particles alone.  Sorted (LDS) and unsorted steps against the oracle."""
    cfg, P = _small(nr=40, nth=36, pairs_per_cell=3, n_filt=2, absorb_cells=5, theta_T=0.3)
    p = cfg["params"]
    P["x"][1::4] = np.clip(P["x"][1::4] + 0.41, 0.0, p["nr"] - 1e-9)
    n = len(P["x"])
    assert n % (256 * ppt) != 0
    _say("capacity = count", prec, ppt, n)
    o, s = make_pair(p, P, prec, capacity=n, chunk_ppt=ppt, tile=(4, 4), sort_interval=2)
    t = TOL[prec]
    for k in range(3):
        if k > 0:
            o = oracle_from_sim(s, p)
        o.step(1)
        s.step(1)
        compare_fields(o, s, t["field"])
        compare_particles(o, s, t, p["nth"], t["band"])
    assert s.counts()["live"] == o.n


@pytest.mark.parametrize("prec", PRECISIONS)
def test_luminosity_moment(prec):
    """The device's Poynting luminosity (PIC_MOM_POYNTING) against the
    oracle's on the same state: a spinning monopole with injection, the
    twelfth step taken by both from identical input bits."""
    from parity_util import oracle_from_sim
    cfg, P = _small(nr=40, nth=36, pairs_per_cell=3, n_filt=2, bg="monopole", omega_frac=0.3, inject=1)
    p = dict(cfg["params"], q_inj=cfg["params"]["q_inj"] * 0.5)
    o, s = make_pair(p, P, prec, capacity=1 << 20)
    s.step(11)
    o = oracle_from_sim(s, p)
    s.step(1)
    o.step(1)
    Lg, Lo = s.luminosity(), o.luminosity()
    scale = np.abs(Lo).max()
    _say(f"{prec}: max |L| {scale:.3e}, worst difference {np.abs(Lg - Lo).max() / scale:.2e}")
    assert scale > 0 and Lg.shape == (p["nr"],)
    # L sums products of two fields, each within the per-step field tolerance
    tol = 2 * TOL[prec]["field"]
    assert np.abs(Lg - Lo).max() <= tol * scale


@pytest.mark.parametrize("prec", PRECISIONS)
def test_sort_groups_each_chunk_by_tile(prec):
    """The first sort puts the generator's shuffled particles in tile order:
    with exactly 64 particles per cell, tiles of 1 x 32 cells (one row of
    cells each, so that every tile is full whatever the ghost width) hold
    2048 particles, and each push chunk (16 x 256 particles) covers two tiles
    of one row, which the LDS region holds; a sort that left particles out
    of tile order would send chunks to the global-memory path.  (Once
    particles move, tiles hold unequal counts and a chunk may reach into a
    third or fourth tile; some chunks then take the global path by design.)
    Over three sorted steps no particle is lost or duplicated."""
    from paper_1407_1810_amd.binding import Sim
    cfg, P = _small(nr=96, nth=128, pairs_per_cell=32, n_filt=2, bg="dipole")
    p = cfg["params"]
    s = Sim(p, precision=prec, capacity=len(P["x"]) + (1 << 20), tile=(1, 32), sort_interval=1, chunk_ppt=16)
    s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
    s.step(1)
    assert s.counts()["global_chunks"] == 0
    s.step(2)
    c = s.counts()
    _say(f"{prec}: {c}")
    ids = s.particles()["id"]
    assert len(ids) == c["live"] and len(np.unique(ids)) == len(ids)
    assert c["live"] + c["deleted"] == len(P["x"]) + c["injected"]


def test_sorts_run_on_their_schedule():
    """Only a sort changes the order in which the particles are stored: the
    live particles keep their order through a step that does not sort, and
    after one that does they are in the serpentine tile order of the cells
    they held when the step began.  With a sort interval of 3, sorts come on
    the first step and on every step whose index is a multiple of 3, also
    after the step index is moved, and on the step after particles are added;
    between them the launch sequence leaves the sort kernels out."""
    from paper_1407_1810_amd.binding import Sim
    cfg = W.small_config(nr=24, nth=16, pairs_per_cell=0, n_filt=1, absorb_cells=3, bg="monopole")
    p = cfg["params"]
    G, tr, tt = 2 * p["n_filt"] + 3, 2, 4
    ntj = (p["nth"] + tt - 1) // tt
    rng = np.random.default_rng(5)

    def plasma(n, id0):
        u = rng.normal(0.0, 1.0, (3, n))
        u *= 2.0 / np.linalg.norm(u, axis=0)  # |u| = 2: 0.89 c
        return dict(x=rng.uniform(0.5, p["nr"] - 0.5, n), y=rng.uniform(0.0, p["nth"], n), ur=u[0], ut=u[1],
                    up=u[2], w=np.where(np.arange(n) % 2 == 0, 1.0, -1.0) * cfg["weight"],
                    id=np.arange(id0, id0 + n, dtype=np.uint64))

    def keys(P):
        i = np.floor(P["x"]).astype(np.int64)
        j = np.minimum(np.floor(P["y"]).astype(np.int64), p["nth"] - 1)
        ti, tj = (i + G) // tr, j // tt
        tj = np.where(ti % 2 == 1, ntj - 1 - tj, tj)
        return dict(zip(P["id"].tolist(), (ti * ntj + tj).tolist()))

    P = plasma(3000, 0)
    s = Sim(p, precision="fp64", capacity=10000, sort_interval=3, tile=(tr, tt))
    s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
    reordered = 0

    def one(step, sorts):
        nonlocal reordered
        before = s.particles()
        k = keys(before)
        s.step(1)
        after = s.particles()["id"].tolist()
        alive = set(after)
        kept = [i for i in before["id"].tolist() if i in alive]
        if sorts:
            kk = [k[i] for i in after]
            assert all(a <= b for a, b in zip(kk, kk[1:])), step
            reordered += after != kept
        else:
            assert after == kept, step
        assert s.counts()["step"] == step + 1

    one(0, True)               # the first step sorts
    for st in range(1, 9):
        one(st, st % 3 == 0)
    s.set_step_index(20)       # next sorts at steps 21 and 24
    for st in range(20, 23):
        one(st, st % 3 == 0)
    Q = plasma(200, 5000)
    s.add_particles(Q["x"], Q["y"], Q["ur"], Q["ut"], Q["up"], Q["w"], Q["id"])
    one(23, True)              # sorts because particles arrived
    for st in range(24, 28):
        one(st, st % 3 == 0)
    assert reordered >= 4


@pytest.mark.parametrize("prec", PRECISIONS)
def test_ten_steps_monopole_rotator_with_injection(prec):
    """Ten steps of a small monopole rotator: spin-up, surface injection
    (same pairs, same Philox positions), deletion, lossy layer."""
    cfg = W.small_config(nr=32, nth=24, pairs_per_cell=2, n_filt=3, absorb_cells=5, bg="monopole",
                         omega_frac=0.3, inject=1)
    p = dict(cfg["params"], q_inj=cfg["params"]["q_inj"] * 0.5, t_spin=6.0)
    P = W.pair_plasma(p, 2, 0.2, cfg["weight"], 3)
    o, s = make_pair(p, P, prec, capacity=1 << 20)
    t = TOL[prec]
    injected = 0
    for k in range(10):
        if k > 0:
            o = oracle_from_sim(s, p)
        n0 = s.counts()["injected"]
        o.step(1)
        s.step(1)
        _say("rotator step", k, "n", o.n)
        compare_fields(o, s, t["field"])
        compare_particles(o, s, t, p["nth"], t["band"])
        assert s.counts()["injected"] - n0 == o.counters()[0]
        injected += o.counters()[0]
        assert np.all(np.abs(s.carry() - o.carry()) <= carry_atol(o, p, prec))
    assert injected > 0


def test_edge_cases_poles_conductors_deletion():
    """Particles exactly on the poles, on faces, inside both conductors,
    moving out of the grid (deleted), and zero-weight test particles."""
    cfg = W.small_config(nr=20, nth=16, pairs_per_cell=0, n_filt=2, absorb_cells=3, bg="monopole",
                         omega_frac=0.2)
    p = cfg["params"]
    u = 0.95 / math.sqrt(1 - 0.95 ** 2)
    x = np.array([5.0, 5.5, 7.0, 3.25, -2.5, -2.9, 21.5, 22.9, 0.0, 20.0, 10.0, 10.0])
    y = np.array([0.0, 16.0, 8.0, 0.0, 4.0, 12.0, 3.0, 9.0, 8.0, 8.0, 1e-13, 16.0 - 1e-13])
    ur = np.array([0.0, 0.1, u, -0.3, -u, -u, u, u, -0.2, 0.3, 0.0, 0.0])
    ut = np.array([0.5, -0.5, 0.0, 0.2, 0.0, 0.0, 0.0, 0.0, 0.1, 0.0, -0.7, 0.7])
    up = np.array([0.0, 0.2, 0.0, 0.1, 0.3, 0.0, 0.0, 0.0, 0.0, 0.1, 0.0, 0.0])
    w = np.array([1, -1, 1, -1, 1, -1, 1, -1, 1e-30, -1e-30, 1, -1], dtype=float) * cfg["weight"]
    P = dict(x=x, y=y, ur=ur, ut=ut, up=up, w=w, id=np.arange(len(x), dtype=np.uint64))
    for prec in PRECISIONS:
        o, s = make_pair(p, P, prec)
        deleted = 0
        for k in range(6):
            if k > 0:
                o = oracle_from_sim(s, p)
            d0 = s.counts()["deleted"]
            o.step(1)
            s.step(1)
            t = TOL[prec]
            compare_fields(o, s, t["field"])
            compare_particles(o, s, t, p["nth"], t["band"])
            assert s.counts()["deleted"] - d0 == o.counters()[1]
            deleted += o.counters()[1]
        assert deleted >= 1  # something was deleted


@pytest.mark.parametrize("prec,nr,nth,r_ratio", [("fp64", 64, 8191, math.exp(128 / 8191)),
                                                 ("fp32", 64, 8191, math.exp(128 / 8191)),
                                                 ("fp64", 16000, 4, 6.0)])
def test_largest_grids(prec, nr, nth, r_ratio):
    """The grid extremes the library accepts: 8191 meridional cells (eight
    injection nodes per thread, the longest rows of filter strips and
    tiles, an odd count) on a thin shell whose cells are as wide as they are
    long at the equator, and 16000 radial cells on the fewest meridional
    ones (in FP64 only: its cells are thousands of times wider in theta
    than in r, so a step moves a particle some 3e-5 of a cell meridionally,
    which an FP32 offset (spacing 6e-8 near one half) resolves to about
    2e-3, and the meridional face charge with it: outside the FP32
    tolerance, measured 2e-5 of E's scale and 3e-4 of E_theta's own); a
    rotating dipole with injection (the carry of every
    node drawn in [0, 1), as in a running simulation), unpaired particles,
    two steps, each from identical input bits (the first sorts).  At 8191
    meridional cells a unit in the last place of the oracle's absolute
    coordinate is 9e-13 cells, so the FP64 gate is widened to four times the
    response of an oracle loaded with shifted coordinates (shifted_floor),
    as at the benchmark sizes; FP32 fields are gated as there too, against
    their vector field's scale (and at OWN_TOL_FP32 against their own for
    components at least 1e-2 of it)."""
    cfg, P = _small(nr=nr, nth=nth, pairs_per_cell=2, n_filt=3, absorb_cells=4, theta_T=0.3, inject=1,
                    omega_frac=0.3, bg="dipole", r_ratio=r_ratio)
    p = cfg["params"]
    P["x"][1::4] = np.clip(P["x"][1::4] + 0.37, 0.0, p["nr"] - 1e-9)
    _say("largest grids", prec, nr, nth, len(P["x"]))
    _, s = make_pair(p, P, prec, carry=np.random.default_rng(5).uniform(0.0, 1.0, nth + 1))
    t = TOL[prec]
    injected = 0
    for k in range(2):
        o, *rest = oracles_from_sim(s, p, (False, True) if prec == "fp64" else (False,))
        before = s.particles()
        o.step(1)
        s.step(1)
        for q in rest:
            q.step(1)
        injected += o.counters()[0]
        compare_fields(o, s, t["field"], vector_scale=prec == "fp32", own_tol=OWN_TOL_FP32 if prec == "fp32" else None,
                       floor=shifted_floor(o, rest[0]) if rest else None)
        compare_particles(o, s, t, p["nth"], t["band"], before=before)
        assert np.all(np.abs(s.carry() - o.carry()) <= carry_atol(o, p, prec))
    assert s.counts()["injected"] == injected > 0


def test_error_codes():
    from paper_1407_1810_amd.binding import PicError, Sim
    cfg = W.small_config(nr=16, nth=12, pairs_per_cell=0)
    p = cfg["params"]
    # capacity
    s = Sim(p, precision="fp32", capacity=3)
    with pytest.raises(PicError) as e:
        s.add_particles(np.full(4, 3.5), np.full(4, 2.5), np.zeros(4), np.zeros(4), np.zeros(4), np.ones(4))
    assert e.value.code == -4
    # position outside the grid
    with pytest.raises(PicError) as e:
        s.add_particles([3.5], [-0.5], [0.0], [0.0], [0.0], [1.0])
    assert e.value.code == -1
    # a non-finite weight (it would void the deposit's fixed-point scale) or
    # momentum: refused, nothing appended
    for bad in ([3.5], [2.5], [0.0], [0.0], [0.0], [math.inf]), ([3.5], [2.5], [math.nan], [0.0], [0.0], [1.0]):
        with pytest.raises(PicError) as e:
            s.add_particles(*bad)
        assert e.value.code == -1 and "non-finite" in str(e.value)
    assert s.counts()["live"] == 0
    # CFL: a particle moving more than a cell per step (c > 1 cell per step)
    q = dict(p, c=3.0)
    s2 = Sim(q, precision="fp64", capacity=10)
    s2.add_particles([5.5], [6.0], [50.0], [0.0], [0.0], [0.0])
    with pytest.raises(PicError) as e:
        s2.step(1)
    assert e.value.code == -3
    # invalid descriptor
    with pytest.raises(PicError):
        Sim(dict(p, nth=2), precision="fp64", capacity=10)
    # empty step is fine
    s3 = Sim(p, precision="fp64", capacity=10)
    s3.step(3)
    assert s3.counts()["live"] == 0


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("r_kind,th_kind", [("log", "eqarea"), ("lin", "lin"), ("log", "lin"), ("lin", "eqarea")])
def test_tm_mode_on_gpu(prec, r_kind, th_kind):
    """The TM-mode field test of Sec. 4.1 run through the library in the four
    coordinate systems the paper compares (log or linear radius, equal-area
    or linear theta): the same field as the oracle after the whole run
    (FP64 to 1e-11, FP32 to 2e-5 of the field scale), and close to the
    analytic mode (the oracle's own convergence in all four is pinned by
    test_tm_mode_second_order)."""
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    import test_oracle_pins as T
    roots = T._du1_roots(4)
    N = 48
    r_in, r_out = roots[0], roots[3]
    if r_kind == "log":
        dxi = math.log(r_out / r_in) / N
        dr0 = r_in * (math.exp(dxi) - 1)
    else:
        dr0 = (r_out - r_in) / N
    dth = r_in * (2.0 / N if th_kind == "eqarea" else math.pi / N)
    c0 = 0.4 * min(dr0, dth)
    nsteps = int(math.ceil(1.25 / c0))
    c = 1.25 / nsteps
    p = dict(nr=N, nth=N, r_in=r_in, r_out=r_out, r_kind=r_kind, th_kind=th_kind, c=c, n_filt=0,
             absorb_cells=0, bg_kind="none")
    from oracle.oracle import Oracle
    o = Oracle(p)
    rb = o.geometry(1)
    yh = np.arange(N) + 0.5
    sh = 2.0 / N * np.sqrt(yh * (N - yh)) if th_kind == "eqarea" else np.sin(math.pi * yh / N)

    def bphi(t):
        return -(T._u1(rb) / rb)[:, None] * sh[None, :] * math.cos(c * t)

    o2, s = make_pair(p, None, prec, fields={"Bph": bphi(-0.5)})
    o2.step(nsteps)
    s.step(nsteps)
    tol = 1e-11 if prec == "fp64" else 2e-5
    compare_fields(o2, s, tol, comps=FIELD_COMPS)
    num, ana = s.get_field("Bph"), bphi(nsteps - 0.5)
    wgt = (rb ** 2)[:, None]
    err = math.sqrt((wgt * (num - ana) ** 2).sum() / (wgt * ana ** 2).sum())
    _say(f"{prec} {r_kind}/{th_kind}: L2 error of r B_phi against the analytic mode {err:.2e}")
    assert err < 1e-2
