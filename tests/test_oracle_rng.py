"""Pins for the oracle's random numbers: Philox4x64-10, the MurmurHash3
finaliser, the Feistel bijection and the block-shift draw.

Philox is checked against numpy's independent implementation. The bijection
is a reading (the paper only asks for "a random permutation of all elements
from a block", Sec. 3.1), so it is pinned by the properties that reading
needs: it is a permutation, it depends on the key, and it looks uniform.
"""
import itertools
import math

import numpy as np
import pytest

MASK64 = (1 << 64) - 1


def numpy_philox_block(ctr, key):
    """Philox4x64-10 of one counter via numpy. numpy advances its 256-bit
    counter before producing a block, so start it one below."""
    c = sum(int(v) << (64 * i) for i, v in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    counter = np.array([(c >> (64 * i)) & MASK64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=counter)
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (5, 0)),
    ((2, 7, 0, 0), (0x5EED, 0)),
    ((0, 12345, 0, 0), (0xFFFFFFFFFFFFFFFF, 0)),
    ((MASK64, MASK64, 3, 9), (0xDEADBEEFCAFEF00D, 0x0123456789ABCDEF)),
    ((1, 1 << 40, 1 << 63, 77), (1, 2)),
])
def test_philox_matches_numpy(ref, ctr, key):
    assert ref.philox4x64_10(ctr, key) == numpy_philox_block(ctr, key)


def test_philox_random_counters_match_numpy(ref):
    rng = np.random.default_rng(11)
    for _ in range(50):
        ctr = [int(v) for v in rng.integers(0, 1 << 63, size=4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 1 << 63, size=2, dtype=np.uint64)]
        assert ref.philox4x64_10(ctr, key) == numpy_philox_block(ctr, key)


def test_draw_is_philox_of_purpose_and_index(ref):
    for seed, purpose, index in [(0x5EED, 0, 0), (0x5EED, 1, 41), (3, 2, 999)]:
        assert ref.draw(seed, purpose, index) == numpy_philox_block((purpose, index, 0, 0), (seed, 0))


def _xorshift_inverse(y, s):
    x = y
    for _ in range(64 // s + 1):
        x = y ^ (x >> s)
    return x & MASK64


def test_fmix64_fixed_point_and_inverse(ref):
    # fmix64 maps 0 to 0 (every step keeps zero).
    assert ref.fmix64(0) == 0
    # It is a bijection of 64-bit words: undo it with the inverse of each step
    # (xor-shift inverse, modular inverse of the published multipliers).
    inv1 = pow(0xff51afd7ed558ccd, -1, 1 << 64)
    inv2 = pow(0xc4ceb53fe1a85ec3, -1, 1 << 64)
    rng = np.random.default_rng(5)
    for v in [1, 2, 0xFFFFFFFFFFFFFFFF, 1 << 63] + [int(x) for x in rng.integers(0, 1 << 63, 200, dtype=np.uint64)]:
        y = ref.fmix64(v)
        x = _xorshift_inverse(y, 33)
        x = (x * inv2) & MASK64
        x = _xorshift_inverse(x, 33)
        x = (x * inv1) & MASK64
        x = _xorshift_inverse(x, 33)
        assert x == v


def test_fmix64_avalanche(ref):
    # Flipping one input bit flips about half of the output bits.
    rng = np.random.default_rng(6)
    flips = []
    for v in rng.integers(0, 1 << 63, 64, dtype=np.uint64):
        v = int(v)
        base = ref.fmix64(v)
        for b in range(64):
            flips.append(bin(base ^ ref.fmix64(v ^ (1 << b))).count("1"))
    assert abs(np.mean(flips) - 32.0) < 0.5


@pytest.mark.parametrize("keyseed", [0, 1, 0x5EED])
def test_bijection_exhaustive_small_n(ref, keyseed):
    for n in list(range(1, 300)) + [511, 512, 513, 1000, 1024, 4095, 4096]:
        rk = ref.draw(keyseed, 1, n)
        table = ref.bijection_table(n, rk)
        assert np.array_equal(np.sort(table), np.arange(n)), n


@pytest.mark.slow
def test_bijection_exhaustive_every_n_to_65536(ref):
    # Every domain size up to 2^16 (grouping tables up to beta = 256 and
    # every grid up to 256 x 256), each with its own keys: the table is a
    # permutation of [0, n).
    for n in range(1, (1 << 16) + 1):
        table = ref.bijection_table(n, ref.draw(0xB1, 3, n))
        assert table.min() == 0 and table.max() == n - 1, n
        seen = np.zeros(n, dtype=bool)
        seen[table] = True
        assert seen.all(), n


@pytest.mark.parametrize("n", [256 * 256, 1 << 18, 1024 * 1024, 1448 * 1448, 1000 * 1001])
def test_bijection_large_n(ref, n):
    rk = ref.draw(7, 0, 0)
    table = ref.bijection_table(n, rk)
    assert table.min() == 0 and table.max() == n - 1
    assert np.unique(table).size == n


def test_bijection_pointwise_matches_table(ref):
    rk = ref.draw(9, 1, 3)
    table = ref.bijection_table(1000, rk)
    for i in [0, 1, 17, 500, 999]:
        assert ref.bijection(1000, rk, i) == table[i]


def test_bijection_depends_on_every_round_key(ref):
    n = 4096
    rk = ref.draw(1, 1, 0)
    base = ref.bijection_table(n, rk)
    for i in range(4):
        other = list(rk)
        other[i] ^= 1 << 5
        assert not np.array_equal(base, ref.bijection_table(n, other))


def test_bijection_looks_uniform(ref):
    # For a uniform random permutation of [0, n): the image of a fixed point
    # is uniform, the mean |pi(i) - i| is (n^2 - 1) / (3n), and the number of
    # fixed points averages 1.
    n, trials = 64, 4000
    images = np.zeros(n, dtype=np.int64)
    fixed = []
    for t in range(trials):
        table = ref.bijection_table(n, ref.draw(123, 1, t))
        images[table[5]] += 1
        fixed.append(int(np.sum(table == np.arange(n))))
    chi2 = float(np.sum((images - trials / n) ** 2 / (trials / n)))
    # 63 degrees of freedom: mean 63, sd ~11.2; allow a wide margin.
    assert chi2 < 63 + 6 * 11.2
    assert abs(np.mean(fixed) - 1.0) < 0.15
    n = 1 << 16
    table = ref.bijection_table(n, ref.draw(77, 1, 1))
    disp = np.abs(table - np.arange(n)).mean()
    assert abs(disp / ((n * n - 1) / (3 * n)) - 1.0) < 0.02


def test_shift_range_and_uniformity(ref):
    w = 37
    counts = np.zeros((2, w), dtype=np.int64)
    for j in range(3700):
        dy, dx = ref.shift(0x5EED, j, w)
        assert 0 <= dy < w and 0 <= dx < w
        counts[0, dy] += 1
        counts[1, dx] += 1
    for row in counts:
        chi2 = float(np.sum((row - 100.0) ** 2 / 100.0))
        assert chi2 < 36 + 6 * math.sqrt(72)


def test_shift_uses_top_bits_of_first_two_words(ref):
    for j, w in [(0, 1024), (5, 64), (17, 1448), (3, 2)]:
        u = numpy_philox_block((2, j, 0, 0), (0x5EED, 0))
        assert ref.shift(0x5EED, j, w) == (((u[0] >> 32) * w) >> 32, ((u[1] >> 32) * w) >> 32)


def test_perms24_is_lexicographic(ref):
    assert [tuple(p) for p in ref.perms24()] == list(itertools.permutations(range(4)))
