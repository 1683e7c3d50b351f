"""Pins for the oracle's Gaussian-like target filter (BOX3: the box pass
three times per axis, rows then columns; a variant of the paper's Gaussian
filter, Sec. 3.1).

Three box passes of half-width r convolve the grid with the three-fold
convolution of a (2r+1)-wide uniform kernel per axis: a piecewise-quadratic
kernel of support 3r and variance r(r+1). The impulse response in the
interior is checked against that convolution computed with numpy, which
also fixes the pass count (one or two passes give other profiles) and the
normalisation; its second moment against r(r+1); r = 0 and constant grids
against their closed forms; bfloat16 storage against the float32 filter
within the bfloat16 rounding of six passes; and the sort on a 2 x 2 grid,
where every window covers the grid, against the all-arrangements-equal
special case.
"""
import itertools

import numpy as np
import pytest

import synthetic


def triple_box_kernel(r: int) -> np.ndarray:
    u = np.full(2 * r + 1, 1.0 / (2 * r + 1))
    return np.convolve(np.convolve(u, u), u)


def test_radius_zero_is_identity(ref):
    G = np.random.default_rng(3).standard_normal((12 * 12, 4)).astype(np.float32)
    assert np.array_equal(ref.blur(G, 12, 0, filter="box3"), G)


@pytest.mark.parametrize("r", [1, 2, 3, 5])
def test_interior_impulse_response_is_the_triple_box_kernel(ref, r):
    w = 12 * r + 9  # every window of every pass stays inside the grid
    c = w // 2
    G = np.zeros((w * w, 2), dtype=np.float32)
    G[c * w + c, 0] = 1.0
    G[c * w + c, 1] = 4.0
    T = ref.blur(G, w, r, filter="box3").reshape(w, w, 2).astype(np.float64)
    k = triple_box_kernel(r)
    want = np.zeros((w, w))
    lo, hi = c - 3 * r, c + 3 * r + 1
    want[lo:hi, lo:hi] = np.outer(k, k)
    # float32 sliding sums of at most 2r+1 terms, six passes: a few ulps of
    # the largest value.
    assert np.max(np.abs(T[:, :, 0] - want)) < 1e-6 * k.max() ** 2 * 64
    assert np.max(np.abs(T[:, :, 1] - 4.0 * want)) < 4e-6 * k.max() ** 2 * 64
    # One or two passes per axis would not match.
    one = np.zeros((w, w))
    u = np.full(2 * r + 1, 1.0 / (2 * r + 1))
    one[c - r:c + r + 1, c - r:c + r + 1] = np.outer(u, u)
    assert np.max(np.abs(T[:, :, 0] - one)) > 1e-3 * u.max() ** 2


@pytest.mark.parametrize("r", [1, 4, 7])
def test_second_moment_is_r_times_r_plus_one(ref, r):
    w = 8 * r + 11  # every window of every pass stays inside the grid
    c = w // 2
    G = np.zeros((w * w, 1), dtype=np.float32)
    G[c * w + c, 0] = 1.0
    T = ref.blur(G, w, r, filter="box3").reshape(w, w).astype(np.float64)
    row = T.sum(axis=0)  # marginal along x
    x = np.arange(w) - c
    assert row.sum() == pytest.approx(1.0, rel=1e-5)
    assert (row * x).sum() == pytest.approx(0.0, abs=1e-5)
    assert (row * x * x).sum() == pytest.approx(r * (r + 1), rel=1e-5)


@pytest.mark.parametrize("w,r", [(8, 1), (16, 3), (16, 15), (33, 7)])
def test_constant_grid(ref, w, r):
    c = np.float32(0.1)
    G = np.full((w * w, 3), c, dtype=np.float32)
    T = ref.blur(G, w, r, filter="box3")
    # Six passes of the single-pass bound (each within ~(w + r) ulps).
    assert np.max(np.abs(T.astype(np.float64) - 0.1)) < 6 * (w + r + 2) * 2.0 ** -24 * 0.1 * (2 * r + 2)


def test_bfloat16_storage_rounds_every_pass(ref):
    w, r = 24, 2
    G = ref.round_bf16(np.random.default_rng(5).uniform(-4, 4, (w * w, 6)).astype(np.float32))
    T32 = ref.blur(G, w, r, filter="box3").astype(np.float64)
    T16 = ref.blur(G, w, r, storage_bf16=True, filter="box3")
    # Stored values are bfloat16 values.
    assert np.array_equal(ref.round_bf16(T16), T16)
    # Within the rounding of six stored passes (2^-9 relative each) of the
    # float32 filter, and not equal to it.
    scale = np.abs(G).max()
    assert np.max(np.abs(T16 - T32)) < 6 * 2.0 ** -8 * scale
    assert not np.array_equal(T16.astype(np.float64), T32)


def test_sort_2x2_every_arrangement_has_the_same_energy(ref):
    # Every window of a 2 x 2 grid at r = 1 covers its line, so each pass is
    # the line mean and the target is the grid mean: all 24 arrangements have
    # equal float64 energy; the sort still returns an arrangement.
    F = np.random.default_rng(9).standard_normal((3, 4)).astype(np.float32)
    res = ref.sort(F, 2, 11, filter="box3")
    assert res.status == 0
    energies = []
    for p in itertools.permutations(range(4)):
        energies.append(ref.grid_energy_f64(F, np.array(p, dtype=np.int32), 2, 1))
    assert max(energies) - min(energies) <= 1e-12 * max(abs(e) for e in energies)
    assert sorted(res.perm.tolist()) == [0, 1, 2, 3]


@pytest.mark.parametrize("side,d,seed", [(16, 3, 1), (24, 59, 2), (33, 14, 3)])
def test_sort_is_valid_deterministic_and_differs_from_box(ref, side, d, seed):
    n = side * side
    F = synthetic.gaussian_attributes(n, seed)[:d] if d <= 59 else synthetic.random_features(n, d, seed)
    F = np.ascontiguousarray(F)
    a = ref.sort(F, side, 7, filter="box3")
    b = ref.sort(F, side, 7, filter="box3")
    box = ref.sort(F, side, 7)
    assert a.status == 0 and np.array_equal(a.perm, b.perm) and a.reorders == b.reorders
    assert np.array_equal(np.sort(a.perm), np.arange(n, dtype=np.int32))
    assert not np.array_equal(a.perm, box.perm)
    # Level count is the schedule's, whatever the filter.
    assert a.levels == box.levels


def test_unknown_filter_is_rejected(ref):
    import ctypes
    F = np.zeros((3, 16), dtype=np.float32)
    G = np.zeros((16, 3), dtype=np.float32)
    T = np.empty_like(G)
    assert ref.lib().plas_ref_blur_filter(G.ctypes.data_as(ctypes.c_void_p), T.ctypes.data_as(ctypes.c_void_p),
                                          4, 3, 1, 0, 2) == ref.INVALID
    prm = ref._Params(1, 0.95, 10000, 16, 0.0, 0, None, 0, 2)
    perm = np.empty(16, dtype=np.int32)
    res = ref._Result()
    st = ref.lib().plas_ref_sort(F.ctypes.data_as(ctypes.c_void_p), 16, 3, 4, 0, ctypes.byref(prm),
                                 perm.ctypes.data_as(ctypes.c_void_p), ctypes.byref(res))
    assert st == ref.INVALID
