"""The counting sort by tile is stable (a counting sort's scatter keeps the
order of equal keys): after a sorted step the particles of every tile key
hold the order they had in storage, and two contexts built from the same
input hold the same storage order, step after step.  Tiles of 8 x 32 cells
at 32 particles per cell put each key's particles in two or three spans of
4096, so that both the ranks within a span (across its four waves) and the
blocks of consecutive spans (the per-key span lists) are exercised; after a
step a key's particles lie in its own spans and in those of the tiles
around it, at most 27, within the 32 a key's span list holds."""
import sys

import numpy as np
import pytest

from paper_1407_1810_amd import workloads as W

pytestmark = pytest.mark.gpu

TILE = (8, 32)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    from paper_1407_1810_amd.binding import gpu_available, lib
    if not gpu_available():
        pytest.skip("no HIP device")
    lib()


def _keys(p, i, j):
    """Serpentine tile key of each cell (tiles over rows -G..nr+G)."""
    G = 2 * p["n_filt"] + 3
    i = np.asarray(i, dtype=np.int64)
    j = np.minimum(np.asarray(j, dtype=np.int64), p["nth"] - 1)
    ntj = (p["nth"] + TILE[1] - 1) // TILE[1]
    ti, tj = (i + G) // TILE[0], j // TILE[1]
    tj = np.where(ti % 2 == 1, ntj - 1 - tj, tj)
    return ti * ntj + tj


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sort_is_stable_and_deterministic(prec):
    from paper_1407_1810_amd.binding import Sim
    cfg = W.small_config(nr=64, nth=128, pairs_per_cell=16, n_filt=1, absorb_cells=4, bg="dipole", theta_T=0.05)
    p = cfg["params"]
    P = W.pair_plasma(p, cfg["pairs_per_cell"], cfg["theta_T"], cfg["weight"], cfg["seed"])
    # storage order: by tile key, shuffled within each key, so that the
    # first sort meets each key in a few consecutive spans
    k = _keys(p, np.floor(P["x"]), np.floor(P["y"]))
    rng = np.random.default_rng(3)
    order = np.lexsort((rng.random(len(k)), k))
    P = {q: v[order] for q, v in P.items()}
    counts = np.bincount(k)
    _say(f"{prec}: {len(k)} particles, {int((counts > 0).sum())} keys, up to {counts.max()} particles per key")
    sims = [Sim(p, precision=prec, capacity=len(k) + 4096, tile=TILE, sort_interval=1) for _ in range(2)]
    for s in sims:
        s.add_particles(P["x"], P["y"], P["ur"], P["ut"], P["up"], P["w"], P["id"])
    before = [dict(s.particles(), **s.particle_cells()) for s in sims]
    for step in range(3):
        for s in sims:
            s.step(1)
        after = [dict(s.particles(), **s.particle_cells()) for s in sims]
        # the order the sort of this step produced: the ids of the particles
        # that began the step, stable-sorted by the key of their cell then
        ids0 = before[0]["id"]
        kk = _keys(p, before[0]["ci"], before[0]["cj"])
        want = ids0[np.argsort(kk, kind="stable")]
        alive = np.isin(want, after[0]["id"])
        assert np.array_equal(after[0]["id"], want[alive]), step
        assert np.array_equal(after[0]["id"], after[1]["id"]), step
        before = after
    _say(f"{prec}: {sims[0].counts()}")
