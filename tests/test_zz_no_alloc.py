"""The entry point that allocates nothing (pic_inject_particles_noalloc)
against pic_inject_particles, through the C ABI: two contexts fed the same
particles, one through each entry point, must hold bit-identical particle
stores (cell, offsets, momenta, weights, ids) after each of two calls in a
row, the second smaller than the first; one step from those stores must give
the same fields and particles (to the per-step tolerance, as the two
contexts' floating-point atomics may add in different orders); a call above
the staging capacity is refused."""
import numpy as np
import pytest

from paper_1407_1810_amd import workloads as W

pytestmark = pytest.mark.gpu

MAX = 65536


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    from paper_1407_1810_amd.binding import gpu_available, lib
    if not gpu_available():
        pytest.skip("no HIP device")
    lib()


def _plasma(p, n, seed):
    rng = np.random.default_rng(seed)
    u = rng.normal(0.0, 0.3, (3, n))
    return dict(x=rng.uniform(0.0, p["nr"], n), y=rng.uniform(0.0, p["nth"], n), ur=u[0], ut=u[1], up=u[2],
                w=np.where(np.arange(n) % 2 == 0, 1.0, -1.0) * rng.uniform(0.5, 1.0, n) * 1e-3,
                id=np.arange(seed << 32, (seed << 32) + n, dtype=np.uint64))


def _same_store(a, b):
    Pa, Pb = a.particles(), b.particles()
    assert len(Pa["x"]) == len(Pb["x"])
    for k in Pa:
        assert np.array_equal(Pa[k], Pb[k]), k


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_injection_matches_the_allocating_one(prec):
    from paper_1407_1810_amd.binding import PicError, Sim
    from parity_util import TOL, compare_fields, compare_particles
    cfg = W.small_config(nr=48, nth=40, pairs_per_cell=0, n_filt=2, absorb_cells=4)
    p = cfg["params"]
    a = Sim(p, precision=prec, capacity=1 << 18, tile=(4, 4), sort_interval=2)
    b = Sim(p, precision=prec, capacity=1 << 18, tile=(4, 4), sort_interval=2)
    for n, seed in ((MAX - 11, 1), (1234, 2)):
        P = _plasma(p, n, seed)
        a.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
        b.add_particles_noalloc(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
        _same_store(a, b)
    assert a.counts()["live"] == MAX - 11 + 1234
    # without ids the slots number the particles in both
    P = _plasma(p, 77, 3)
    a.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"])
    b.add_particles_noalloc(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"])
    _same_store(a, b)
    # one step from the two stores
    a.step(1)
    b.step(1)
    t = TOL[prec]
    compare_fields(a, b, t["field"])
    compare_particles(a, b, t, p["nth"], t["band"])
    # above the staging capacity, or outside the grid: refused, nothing added
    P = _plasma(p, MAX + 1, 4)
    with pytest.raises(PicError) as e:
        b.add_particles_noalloc(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
    assert e.value.code == -1
    with pytest.raises(PicError) as e:
        b.add_particles_noalloc([1.0], [-1.0], [0.0], [0.0], [0.0], [1.0])
    assert e.value.code == -1
    assert b.counts()["live"] == a.counts()["live"]
