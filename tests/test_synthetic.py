"""The seeded input recipes (synthetic/): shapes, layouts, determinism and
the distribution of every channel group of the 3DGS-shaped attributes, the
batch workload's sides, and the random RGB grid of the paper's runtime
experiment (App. C)."""
import numpy as np
import pytest

import synthetic


def test_gaussian_attributes_shape_layouts_and_determinism():
    a = synthetic.gaussian_attributes(1000, 3)
    assert a.shape == (59, 1000) and a.dtype == np.float32 and a.flags.c_contiguous
    b = synthetic.gaussian_attributes(1000, 3, "nc")
    assert b.shape == (1000, 59) and np.array_equal(a.T, b)
    assert np.array_equal(a, synthetic.gaussian_attributes(1000, 3))
    assert not np.array_equal(a, synthetic.gaussian_attributes(1000, 4))
    # n = 0 gives an empty grid.
    assert synthetic.gaussian_attributes(0, 1).shape == (59, 0)
    with pytest.raises(ValueError):
        synthetic.gaussian_attributes(10, 1, "xy")


def test_gaussian_attribute_channel_distributions():
    n = 200_000
    x = synthetic.gaussian_attributes(n, 11, "nc").astype(np.float64)
    off = 0
    groups = {}
    for name, k in synthetic.CHANNELS:
        groups[name] = x[:, off:off + k]
        off += k
    assert off == synthetic.D_3DGS == 59
    # xyz: a mixture of 8 clusters of width 0.3 around centres in [-2, 2]^3.
    xyz = groups["xyz"]
    assert np.all(np.abs(xyz) < 2.0 + 0.3 * 6)
    assert 0.3 < xyz.std(axis=0).min()
    # log-scale N(-4, 0.5^2).
    ls = groups["log_scale"]
    assert abs(ls.mean() + 4.0) < 0.01 and abs(ls.std() - 0.5) < 0.01
    # rotation: unit quaternions, isotropic.
    q = groups["rotation"]
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-6)
    assert np.all(np.abs(q.mean(axis=0)) < 0.01)
    # opacity logit N(0, 2^2).
    op = groups["opacity_logit"]
    assert abs(op.mean()) < 0.02 and abs(op.std() - 2.0) < 0.02
    # SH DC U(-1, 1): mean 0, variance 1/3, bounded.
    dc = groups["sh_dc"]
    assert np.all(np.abs(dc) <= 1.0) and abs(dc.var() - 1.0 / 3.0) < 0.005
    # SH rest N(0, 0.1^2).
    rest = groups["sh_rest"]
    assert abs(rest.mean()) < 0.001 and abs(rest.std() - 0.1) < 0.001


def test_rgb_grid_is_uniform_0_255():
    g = synthetic.random_rgb_grid(512, synthetic.DATA_SEED_RGB)
    assert g.shape == (3, 512 * 512) and g.dtype == np.float32
    assert g.min() >= 0.0 and g.max() < 255.0
    assert abs(g.mean() - 127.5) < 0.5 and abs(g.var() - 255.0 ** 2 / 12) < 60


def test_batch_workload():
    work = synthetic.batch_workload()
    assert len(work) == synthetic.BATCH_GRIDS == 64
    sides = [s for s, _, _ in work]
    lo, hi = synthetic.BATCH_SIDE_RANGE
    assert all(lo <= s <= hi for s in sides)
    assert sum(s * s for s in sides) == 11_833_105
    assert [w[2] for w in work] == [synthetic.SORT_SEED + i for i in range(64)]
    assert len({w[1] for w in work}) == 64
    assert work == synthetic.batch_workload()
    # Log-uniform: about half the sides below the geometric midpoint.
    mid = (lo * hi) ** 0.5
    assert 20 <= sum(s < mid for s in sides) <= 44


def test_random_permutation_and_small_integers():
    p = synthetic.random_permutation(1000, 3)
    assert p.dtype == np.int32 and np.array_equal(np.sort(p), np.arange(1000))
    f = synthetic.small_integer_features(100, 5, 2, high=16)
    assert f.shape == (5, 100) and np.array_equal(f, np.floor(f)) and f.min() >= 0 and f.max() < 16
