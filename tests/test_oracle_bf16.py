"""Pins for the oracle's bfloat16 storage mode: features and blurred grids
held in bfloat16 (round to nearest, ties to even), all arithmetic in float32.

The rounding is pinned against torch's own float32 -> bfloat16 conversion;
the blur against the float32 blur within the bfloat16 rounding bound; the
sort against the invariants and against the float32 sort's final energy.
"""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")


def torch_bf16(x: np.ndarray) -> np.ndarray:
    return torch.from_numpy(np.asarray(x, np.float32)).to(torch.bfloat16).to(torch.float32).numpy()


def test_round_bf16_matches_torch(ref):
    rng = np.random.default_rng(0)
    vals = np.concatenate([
        rng.standard_normal(2000).astype(np.float32) * 10 ** rng.uniform(-30, 30, 2000).astype(np.float32),
        np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, -3.0e38, 1e-40, -1e-40, 2.0 ** -133], np.float32),
    ])
    # Exact ties: a bfloat16 value plus half of its last place, odd and even.
    base = np.array([1.0, 1.0078125, 3.5, -2.015625, 1e-3], np.float32)
    ulp = np.array([2.0 ** -7, 2.0 ** -7, 2.0 ** -6, 2.0 ** -6, 2.0 ** -17], np.float32)
    ties = (base.astype(np.float64) + ulp.astype(np.float64) / 2).astype(np.float32)
    vals = np.concatenate([vals, ties, -ties]).astype(np.float32)
    got = ref.round_bf16(vals)
    want = torch_bf16(vals)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_round_bf16_is_idempotent_and_keeps_representable_values(ref):
    x = np.random.default_rng(1).standard_normal(500).astype(np.float32)
    once = ref.round_bf16(x)
    assert np.array_equal(ref.round_bf16(once), once)
    assert np.all((once.view(np.uint32) & 0xFFFF) == 0)


@pytest.mark.parametrize("w,r,d", [(8, 1, 3), (17, 4, 5), (32, 31, 4)])
def test_bf16_blur_is_rounded_fp32_blur(ref, w, r, d):
    G = torch_bf16(np.random.default_rng(w + r).uniform(-2, 2, (w * w, d)))
    T16 = ref.blur(G, w, r, storage_bf16=True)
    T32 = ref.blur(G, w, r)
    # Every stored value is a bfloat16 value.
    assert np.all((T16.view(np.uint32) & 0xFFFF) == 0)
    # Each pass rounds once (relative 2^-9), and the second pass sums
    # rounded first-pass values: within a few bfloat16 places of the float32
    # result.
    scale = float(np.abs(G).max())
    assert np.max(np.abs(T16 - T32)) <= 4 * 2.0 ** -8 * scale
    assert np.array_equal(ref.blur(G, w, 0, storage_bf16=True), G)


def test_bf16_sort_sees_rounded_features(ref):
    w = 32
    F = synthetic.gaussian_attributes(w * w, 3)
    res = ref.sort(F, w, 5, storage_bf16=True, energy_cap=100000)
    assert res.status == 0
    assert np.array_equal(np.sort(res.perm), np.arange(w * w))
    # Its energies are those of the rounded features with a bfloat16 target.
    Fr = torch_bf16(F)
    st, E, s, _ = ref.grid_energy(Fr, res.perm, w, 1, storage_bf16=True)
    assert st == 0 and s == res.scale_shift
    # Same as sorting the rounded features in bfloat16 mode.
    again = ref.sort(Fr, w, 5, storage_bf16=True)
    assert np.array_equal(again.perm, res.perm) and again.reorders == res.reorders


def test_bf16_sort_energy_close_to_fp32(ref):
    """The bfloat16 sort's final float64 energy (on the original features, at
    r = 1) averages within 0.5 % of the float32 sort's over seeds; single runs
    differ by heuristic noise of the same size as between float32 seeds."""
    w = 128
    F = synthetic.gaussian_attributes(w * w, 7)
    e32 = [ref.grid_energy_f64(F, ref.sort(F, w, s).perm, w, 1) for s in (1, 2, 3)]
    e16 = [ref.grid_energy_f64(F, ref.sort(F, w, s, storage_bf16=True).perm, w, 1) for s in (1, 2, 3)]
    gap = np.mean(e16) / np.mean(e32) - 1
    assert abs(gap) < 0.005
