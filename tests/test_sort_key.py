"""The sort kernels' tile index floor(x / d) is formed without an integer
division, as trunc((x + 1/2) * r) in FP32 with r = 1/d rounded to FP32 on
the host (TileMap::key).  The exactness argument (the quotient lies at
least 1/(2d) from an integer, the two roundings move it by less) is checked
here exhaustively in FP32 arithmetic over every row or column index the
grids allow and the tile sizes the library accepts."""
import numpy as np


def _tile_index(x, d):
    r = np.float32(1.0) / np.float32(d)
    return ((x.astype(np.float32) + np.float32(0.5)) * r).astype(np.int64)


def test_reciprocal_floor_is_exact():
    x = np.arange(0, 1 << 15, dtype=np.int64)  # nr + 2G stays below 2^15
    for d in list(range(1, 257)) + [300, 511, 512, 1000, 1023, 1024, 2047, 2048, 3000, 4095, 4096]:
        assert np.array_equal(_tile_index(x, d), x // d), d
