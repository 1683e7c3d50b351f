"""Pins for the oracle's target (the low-pass filtered grid of Sec. 3.1) and
for its distance and quantisation.

The blur is a box mean over the window clipped to the grid. It is checked
against closed forms (constants, ramps, the identity at r = 0), against a
float64 brute-force mean over the clipped rectangle within the float32
rounding bound of a sliding sum, and for exact sums on small integers.
"""
import numpy as np
import pytest

EPS32 = 2.0 ** -24


def brute_blur64(G, w, r):
    """Mean over the clipped (2r+1)^2 window, float64, direct sums."""
    d = G.shape[1]
    g = G.astype(np.float64).reshape(w, w, d)
    out = np.empty_like(g)
    for y in range(w):
        y0, y1 = max(0, y - r), min(w - 1, y + r)
        for x in range(w):
            x0, x1 = max(0, x - r), min(w - 1, x + r)
            out[y, x] = g[y0:y1 + 1, x0:x1 + 1].mean(axis=(0, 1))
    return out.reshape(w * w, d)


def test_radius_zero_is_identity(ref):
    G = np.random.default_rng(0).standard_normal((9 * 9, 5)).astype(np.float32)
    assert np.array_equal(ref.blur(G, 9, 0), G)


@pytest.mark.parametrize("w,r", [(8, 1), (16, 3), (16, 15), (16, 40), (33, 7)])
def test_constant_grid(ref, w, r):
    c = np.float32(0.1)
    G = np.full((w * w, 3), c, dtype=np.float32)
    T = ref.blur(G, w, r)
    # Each pass accumulates at most ~(w + r) rounding errors of size
    # ulp(window sum); a missing or doubled window term would be off by
    # c / count >= c / (2r+1)^2.
    bound = 2 * (w + r + 2) * EPS32 * float(c) * 2
    assert np.max(np.abs(T.astype(np.float64) - float(c))) <= bound


@pytest.mark.parametrize("w,r", [(12, 1), (12, 3), (20, 5)])
def test_linear_ramp_interior(ref, w, r):
    # A ramp a*x + b*y + c has its window mean at the window centre wherever
    # the window is not clipped.
    ys, xs = np.mgrid[0:w, 0:w]
    G = np.stack([2 * xs + 3 * ys + 1, xs - ys], axis=-1).reshape(w * w, 2).astype(np.float32)
    T = ref.blur(G, w, r).reshape(w, w, 2)
    inner = slice(r, w - r)
    expect = G.reshape(w, w, 2)[inner, inner].astype(np.float64)
    got = T[inner, inner].astype(np.float64)
    scale = np.abs(G).max()
    assert np.max(np.abs(got - expect)) <= 8 * (w + r) * EPS32 * scale


@pytest.mark.parametrize("w,r,d", [(5, 1, 1), (7, 2, 3), (16, 3, 4), (17, 5, 3), (9, 8, 2), (10, 20, 3)])
def test_matches_float64_brute_force_within_bound(ref, w, r, d):
    rng = np.random.default_rng(w * 100 + r)
    G = rng.uniform(-3, 3, size=(w * w, d)).astype(np.float32)
    T = ref.blur(G, w, r).astype(np.float64)
    T64 = brute_blur64(G, w, r)
    # Sliding-sum error per pass: each of at most w + r + 1 updates rounds a
    # partial sum bounded by (2r+1) max|G|; the result is divided by the
    # count, and the second pass carries the first pass's error through.
    m = float(np.abs(G).max())
    per_pass = (w + r + 2) * EPS32 * m * 2
    assert np.max(np.abs(T - T64)) <= 3 * per_pass


def test_small_integers_horizontal_pass_exact(ref):
    # Integer features in [0, 16): every horizontal sliding sum is an exact
    # integer, so the horizontal pass must equal
    # float32(exact window sum) * float32(1 / count) bit for bit. All rows are
    # equal, so the vertical pass then averages equal values and may only
    # move them by the rounding of its own sliding sum.
    w, r, d = 11, 3, 2
    rng = np.random.default_rng(3)
    row = rng.integers(0, 16, size=(w, d)).astype(np.float32)
    G = np.tile(row, (w, 1))
    T = ref.blur(G, w, r).reshape(w, w, d)
    for x in range(w):
        lo, hi = max(0, x - r), min(w - 1, x + r)
        exact = row[lo:hi + 1].astype(np.int64).sum(axis=0)
        h = exact.astype(np.float32) * (np.float32(1) / np.float32(hi - lo + 1))
        assert np.allclose(T[:, x], h, rtol=(w + 2) * 4 * EPS32, atol=0)
    # Where the vertical window is the whole column of identical values the
    # sums are exact too (small integers times counts stay below 2^24) only
    # when h is an integer; check those columns bit for bit.
    for x in range(w):
        lo, hi = max(0, x - r), min(w - 1, x + r)
        exact = row[lo:hi + 1].astype(np.int64).sum(axis=0)
        cnt = hi - lo + 1
        if np.all(exact % cnt == 0) and cnt in (1, 2, 4):
            assert np.array_equal(T[:, x], (exact // cnt).astype(np.float32) * np.ones((w, 1), np.float32))


def test_transpose_and_flip_symmetry_within_bound(ref):
    w, r, d = 24, 4, 3
    G = np.random.default_rng(8).uniform(-1, 1, size=(w, w, d)).astype(np.float32)
    T = ref.blur(G.reshape(-1, d), w, r).reshape(w, w, d)
    bound = 6 * (w + r + 2) * EPS32
    Tt = ref.blur(np.ascontiguousarray(G.transpose(1, 0, 2)).reshape(-1, d), w, r).reshape(w, w, d)
    assert np.max(np.abs(Tt.transpose(1, 0, 2) - T)) <= bound
    Tf = ref.blur(np.ascontiguousarray(G[::-1, ::-1]).reshape(-1, d), w, r).reshape(w, w, d)
    assert np.max(np.abs(Tf[::-1, ::-1] - T)) <= bound


def test_sliding_order_add_before_subtract(ref):
    # One line where the order of the update matters: with a window of 3
    # at x = 2 the running sum first gains 2^24 then loses 1.
    # Row 0 holds [1, 1, 1, 2^24, 0]; the other rows are zero, r = 1.
    # x=0: s = 1 + 1 = 2; x=1: s = 2 + 1 = 3; x=2: s = 3 + 2^24 = 2^24 + 4
    # (3 + 2^24 rounds to even 2^24 + 4), then minus 1 -> 2^24 + 3 rounds to
    # 2^24 + 4. Subtract-then-add would give 2 + 2^24 exactly.
    w = 5
    G = np.zeros((w * w, 1), dtype=np.float32)
    G[0:5, 0] = [1, 1, 1, 2.0 ** 24, 0]
    # Read the horizontal pass through a vertical pass with r = 1 over rows
    # 0..1 only: T[0][2] = (H[0][2] + H[1][2]) / 2 with H[1] = 0.
    T = ref.blur(G, w, 1).reshape(w, w)
    h_add_first = np.float32(2.0 ** 24 + 4) * (np.float32(1) / np.float32(3))
    assert T[0, 2] == np.float32(h_add_first * np.float32(0.5))


def test_distance_closed_forms(ref):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(59).astype(np.float32)
    assert ref.distance(x, x) == 0.0
    a, b = np.float32(1.75), np.float32(-0.5)
    assert ref.distance([a], [b]) == np.float32(a - b) * np.float32(a - b)


def test_distance_pairwise_tree_order(ref):
    # Squares [1, 0, 2^-24, 2^-24]: the pairwise tree gives
    # (1 + 0) + (2^-24 + 2^-24) = 1 + 2^-23 exactly, while a left-to-right sum
    # (and the interleaved tree (v0+v2)+(v1+v3)) rounds to 1.
    a = np.array([1.0, 0.0, 2.0 ** -12, 2.0 ** -12], dtype=np.float32)
    assert ref.distance(a, np.zeros(4, np.float32)) == np.float32(1.0 + 2.0 ** -23)
    # Padding with zeros to the next power of two changes nothing.
    a3 = np.array([2.0 ** -12, 2.0 ** -12, 1.0], dtype=np.float32)
    assert ref.distance(a3, np.zeros(3, np.float32)) == np.float32(2.0 ** -23) + np.float32(1.0)


@pytest.mark.parametrize("d", [1, 3, 14, 59, 64, 100])
def test_distance_float64_within_pairwise_bound(ref, d):
    rng = np.random.default_rng(d)
    for _ in range(50):
        a = rng.standard_normal(d).astype(np.float32)
        b = rng.standard_normal(d).astype(np.float32)
        exact = float(np.sum((a.astype(np.float64) - b.astype(np.float64)) ** 2))
        got = float(ref.distance(a, b))
        levels = int(np.ceil(np.log2(max(d, 1)))) + 2
        assert abs(got - exact) <= levels * 2 * EPS32 * exact


def test_quantise_is_exact_floor(ref):
    assert ref.quantise(0.75, 2) == 3
    assert ref.quantise(0.75, 0) == 0
    assert ref.quantise(1.5, 40) == 3 << 39
    x = np.float32(0.1)
    assert ref.quantise(x, 61) == int(np.floor(float(x) * 2.0 ** 61))
    assert ref.quantise(5.0, -1) == 2
    assert ref.quantise(0.0, 50) == 0


def test_scale_shift_definition(ref):
    import math
    # Channels spanning [0, 1], [-2, 2] and a constant: D_max = 1 + 16 + 0.
    n = 100
    F = np.zeros((3, n), dtype=np.float32)
    F[0] = np.linspace(0, 1, n)
    F[1] = np.linspace(-2, 2, n)
    F[2] = 7.0
    st, s, dmax = ref.scale_shift(F, "cn")
    assert st == 0 and dmax == 17.0
    m, e = math.frexp(n * 17.0)
    assert s == 61 - e
    st, s, _ = ref.scale_shift(np.ascontiguousarray(F.T), "nc")
    assert s == 61 - e
    const = np.full((2, 16), 3.0, dtype=np.float32)
    assert ref.scale_shift(const)[1] == 0
    bad = F.copy()
    bad[1, 5] = np.nan
    assert ref.scale_shift(bad)[0] == ref.NONFINITE
    bad[1, 5] = np.inf
    assert ref.scale_shift(bad)[0] == ref.NONFINITE


def test_energy_sum_stays_below_2_pow_61(ref):
    # Worst case: every cell as far as possible from its target.
    import synthetic
    w = 32
    F = synthetic.gaussian_attributes(w * w, 4)
    st, s, dmax = ref.scale_shift(F)
    G = ref.gather(F, None)
    for r in (1, 5, 31):
        T = ref.blur(G, w, r)
        assert ref.energy_fixed(G, T, s) < 2 ** 61
