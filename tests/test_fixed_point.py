"""Host check of the arithmetic the FP32 deposit relies on (no GPU): each
contribution v, in fixed-point units, is rounded to an integer q by adding
1.5 * 2^52 in FP64, and the 64-bit pattern of that sum, 0x4338 * 2^48 + q,
is accumulated as it is with wrap-around 64-bit integer adds.  The constant
is a multiple of 2^51, so the low 51 bits of the total, sign-extended from
bit 50, are the exact sum of the q while it stays below 2^50 in magnitude:
2^14 contributions (a push chunk of 4096 particles, at most four per entry)
of at most 2^35 + 1/2 each."""
import numpy as np

SHIFT = 6755399441055744.0  # 1.5 * 2^52


def _accumulate(v):
    bits = (np.asarray(v, dtype=np.float64) + SHIFT).view(np.uint64)
    with np.errstate(over="ignore"):
        total = np.add.reduce(bits, dtype=np.uint64)
    low = int(total) & ((1 << 51) - 1)
    return low - (1 << 51) if low >= (1 << 50) else low


def test_constant_is_a_multiple_of_2_51():
    m = int(np.float64(SHIFT).view(np.uint64))
    assert m == 0x4338 << 48
    assert m % (1 << 51) == 0


def test_rounding_to_the_nearest_integer():
    v = np.array([0.4, 0.6, -0.4, -0.6, 2.5, -2.5, 1e10 + 0.25, -(2.0 ** 35)])
    q = (v + SHIFT).view(np.uint64).astype(np.int64) - (0x4338 << 48)
    assert np.array_equal(q, np.rint(v).astype(np.int64))


def test_sum_recovered_at_the_bound():
    rng = np.random.default_rng(7)
    n = 1 << 14
    for v in (np.full(n, 2.0 ** 35), np.full(n, -(2.0 ** 35)),
              rng.uniform(-(2.0 ** 35), 2.0 ** 35, n), rng.normal(0.0, 1e3, n)):
        assert _accumulate(v) == int(np.rint(v).astype(np.int64).sum())


def test_cancelling_pairs_give_exactly_zero():
    rng = np.random.default_rng(3)
    a = rng.uniform(-(2.0 ** 35), 2.0 ** 35, 4096)
    assert _accumulate(np.concatenate([a, -a])) == 0
