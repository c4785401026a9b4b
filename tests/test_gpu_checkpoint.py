"""Checkpoint and resume through the C ABI (pic_save / pic_load): a run
saved after some steps and restored into a fresh context holds the same
bits -- every field plane, every particle slot, the counters, the injection
carry -- and both copies then take the same steps (up to the order of
floating-point atomic additions, as two runs of one context would); a
checkpoint that is not one, or is truncated or corrupt, is refused."""
import os

import numpy as np
import pytest

from paper_1407_1810_amd import workloads as W
from parity_util import compare_fields

pytestmark = pytest.mark.gpu

COMPS = ["Er", "Eth", "Eph", "Br", "Bth", "Bph", "Fr", "Fth", "Fph"]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    from paper_1407_1810_amd.binding import gpu_available, lib
    if not gpu_available():
        pytest.skip("no HIP device")
    lib()


def _rotator(prec):
    from paper_1407_1810_amd.binding import Sim
    cfg = W.small_config(nr=40, nth=36, pairs_per_cell=4, n_filt=2, absorb_cells=6, bg="monopole",
                         omega_frac=0.3, inject=1)
    p = cfg["params"]
    P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    s = Sim(p, precision=prec, capacity=len(P["x"]) + (1 << 21), tile=(4, 4), sort_interval=3, chunk_ppt=8)
    s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
    return s


def _state(s):
    return ({c: s.get_field(c) for c in COMPS}, s.particles(), s.counts(), s.carry())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_save_load_resumes_the_same_run(prec, tmp_path):
    from paper_1407_1810_amd.binding import Sim
    s = _rotator(prec)
    s.step(7) # past a sort, with injection under way
    path = tmp_path / "run.ckpt"
    s.save(path)
    f0, p0, c0, k0 = _state(s)
    assert c0["injected"] > 0 and c0["step"] == 7
    r = Sim.load(path)
    f1, p1, c1, k1 = _state(r)
    for c in COMPS: # the same bits, slot for slot
        assert np.array_equal(f0[c], f1[c]), c
    for k in p0:
        assert np.array_equal(p0[k], p1[k]), k
    assert c0 == c1
    assert np.array_equal(k0, k1)
    assert (r.nr, r.nth) == (s.nr, s.nth)
    s.step(5)
    r.step(5)
    compare_fields(s, r, 1e-12 if prec == "fp64" else 1e-5, vector_scale=prec == "fp32")
    a, b = s.particles(), r.particles()
    ka, kb = np.argsort(a["id"]), np.argsort(b["id"])
    assert np.array_equal(a["id"][ka], b["id"][kb])
    tol = 1e-12 if prec == "fp64" else 1e-5
    for k in ("x", "y", "ur", "ut", "up", "w"):
        assert np.allclose(a[k][ka], b[k][kb], rtol=0, atol=tol * (1 + np.abs(a[k]).max())), k
    assert s.counts()["step"] == r.counts()["step"] == 12


def test_checkpoint_errors(tmp_path):
    import ctypes as C
    from paper_1407_1810_amd.binding import PicError, Sim, lib
    s = _rotator("fp32")
    s.step(2)
    good = tmp_path / "good.ckpt"
    s.save(good)
    L = lib()
    # pic_save on a context without pic_init, pic_load into an initialised one
    h = C.c_void_p()
    assert L.pic_create(C.byref(h), 0, None) == 0
    try:
        assert L.pic_save(h, os.fsencode(str(tmp_path / "x.ckpt"))) == -7
    finally:
        L.pic_destroy(h)
    assert L.pic_load(s._h, os.fsencode(str(good))) == -7
    with pytest.raises(PicError) as e:
        Sim.load(tmp_path / "missing.ckpt")
    assert e.value.code == -1
    junk = tmp_path / "junk.ckpt"
    junk.write_bytes(b"not a checkpoint" * 64)
    with pytest.raises(PicError) as e:
        Sim.load(junk)
    assert e.value.code == -1 and "checkpoint" in str(e.value)
    data = good.read_bytes()
    cut = tmp_path / "cut.ckpt"
    cut.write_bytes(data[: len(data) - 100])
    with pytest.raises(PicError) as e:
        Sim.load(cut)
    assert e.value.code == -1 and "truncated" in str(e.value)
    # a cell index outside the grid.  A context saved before its first step
    # holds exactly its loaded particles; with FP32 storage and ids each
    # slot takes 4 (cell) + 6 x 4 + 8 (id) bytes at the end of the file,
    # cells first.
    t = _rotator("fp32")
    n = t.counts()["live"]
    fresh = tmp_path / "fresh.ckpt"
    t.save(fresh)
    data = bytearray(fresh.read_bytes())
    off = len(data) - n * (4 + 6 * 4 + 8)
    assert Sim.load(fresh).counts()["live"] == n
    data[off:off + 4] = np.uint32((30000 << 16) | 0).tobytes()
    corrupt = tmp_path / "corrupt.ckpt"
    corrupt.write_bytes(bytes(data))
    with pytest.raises(PicError) as e:
        Sim.load(corrupt)
    assert e.value.code == -1 and "out of range" in str(e.value)
