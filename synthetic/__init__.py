"""Seeded synthetic inputs for PLAS sorting.

This module only draws random numbers. It holds none of the sort's
arithmetic, so both the CPU oracle tests and the GPU path may use it.

The paper sorts real 3D Gaussian Splatting scenes (Sec. 4) and, for its
runtime experiment, a random 512x512 RGB grid (App. C). Neither the trained
scenes nor the datasets are available, so these generators stand in for
them with the same shapes: N Gaussians with D = 59 attributes each
(position 3, log-scale 3, rotation quaternion 4, opacity logit 1, SH DC 3,
SH rest 45), or a grid of uniform colour values.

All draws use numpy's PCG64 generator in float64 and are cast to float32 at
the end, so the same seed gives the same bytes on every machine that runs
the same numpy.
"""
from __future__ import annotations

import numpy as np

# Channel layout of one 3DGS attribute vector (Sec. 3 of the paper lists the
# attribute kinds; the split below is the standard 3DGS one with degree-3
# spherical harmonics).
CHANNELS = (
    ("xyz", 3),
    ("log_scale", 3),
    ("rotation", 4),
    ("opacity_logit", 1),
    ("sh_dc", 3),
    ("sh_rest", 45),
)
D_3DGS = sum(k for _, k in CHANNELS)  # 59

DATA_SEED_SMALL = 1       # 64 x 64 grid
DATA_SEED_SCENE = 2       # 1024 x 1024 grid
DATA_SEED_PRECISION = 3   # 1448 x 1448 grid
SORT_SEED = 0x5EED
DATA_SEED_BATCH = 4       # the 64-grid batch: sides and per-grid data seeds
DATA_SEED_RGB = 5         # the random 512 x 512 x 3 grid of the runtime experiment
DATA_SEED_GARDEN = 6      # the scene-scale grid of App. C's largest scene
BATCH_GRIDS = 64
BATCH_SIDE_RANGE = (128, 724)
# App. C's largest scene holds 4.37 million Gaussians: a grid of side 2091
# (2091^2 = 4,372,281).
GARDEN_SIDE = 2091
# Channels before the 45 higher spherical-harmonics coefficients: xyz,
# log-scale, rotation, opacity and SH DC (the paper sorts on at most 14).
D_NO_SH_REST = D_3DGS - 45  # 14


def gaussian_attributes(n: int, seed: int, layout: str = "cn") -> np.ndarray:
    """Draw n synthetic 3DGS attribute vectors, D = 59, float32.

    Distributions, in channel order:
      xyz          8 centres ~ U(-2, 2)^3 (drawn first); component ~ U{0..7};
                   xyz = centre + 0.3 * N(0, I3)
      log-scale    N(-4, 0.5^2)
      rotation     q ~ N(0, I4), then q / |q|
      opacity      N(0, 2^2)
      SH DC        U(-1, 1)
      SH rest      N(0, 0.1^2)

    layout "cn" returns [59][n] (channel-major), "nc" returns [n][59].
    """
    if n < 0:
        raise ValueError("n must be non-negative")
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(-2.0, 2.0, size=(8, 3))
    comp = rng.integers(0, 8, size=n)
    xyz = centres[comp] + 0.3 * rng.standard_normal(size=(n, 3))
    log_scale = rng.normal(-4.0, 0.5, size=(n, 3))
    q = rng.standard_normal(size=(n, 4))
    norm = np.sqrt((q * q).sum(axis=1, keepdims=True))
    norm[norm == 0.0] = 1.0
    rot = q / norm
    opacity = rng.normal(0.0, 2.0, size=(n, 1))
    sh_dc = rng.uniform(-1.0, 1.0, size=(n, 3))
    sh_rest = rng.normal(0.0, 0.1, size=(n, 45))
    nc = np.concatenate([xyz, log_scale, rot, opacity, sh_dc, sh_rest], axis=1)
    nc = nc.astype(np.float32)
    if layout == "nc":
        return np.ascontiguousarray(nc)
    if layout == "cn":
        return np.ascontiguousarray(nc.T)
    raise ValueError(f"unknown layout {layout!r}")


def scene_attributes_14(n: int, seed: int) -> np.ndarray:
    """The first 14 channels of gaussian_attributes(n, seed) (every channel
    but the higher SH coefficients), channel-major [14][n]."""
    return np.ascontiguousarray(gaussian_attributes(n, seed, "cn")[:D_NO_SH_REST])


def random_features(n: int, d: int, seed: int, layout: str = "cn",
                    low: float = -1.0, high: float = 1.0) -> np.ndarray:
    """n vectors of d independent U(low, high) float32 values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(low, high, size=(n, d)).astype(np.float32)
    if layout == "nc":
        return np.ascontiguousarray(x)
    if layout == "cn":
        return np.ascontiguousarray(x.T)
    raise ValueError(f"unknown layout {layout!r}")


def random_rgb_grid(side: int, seed: int, layout: str = "cn") -> np.ndarray:
    """A side x side grid of RGB values ~ U(0, 255), as in the paper's
    runtime experiment on a random 512x512x3 grid (App. C)."""
    return random_features(side * side, 3, seed, layout, 0.0, 255.0)


def small_integer_features(n: int, d: int, seed: int, high: int = 16,
                           layout: str = "cn") -> np.ndarray:
    """Integer-valued float32 features in [0, high), for exactness checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.integers(0, high, size=(n, d)).astype(np.float32)
    if layout == "nc":
        return np.ascontiguousarray(x)
    return np.ascontiguousarray(x.T)


def batched_sides(count: int, lo: int, hi: int, seed: int) -> list[int]:
    """Square grid sides drawn log-uniform in [lo, hi] (inclusive), rounded
    to the nearest integer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(np.log(lo), np.log(hi), size=count)
    return [int(min(hi, max(lo, round(float(np.exp(v)))))) for v in u]


def random_permutation(n: int, seed: int) -> np.ndarray:
    """A uniformly random permutation of [0, n) as int32 (for init_perm
    inputs in tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.permutation(n).astype(np.int32)


def batch_workload(count: int = BATCH_GRIDS, lo: int = BATCH_SIDE_RANGE[0], hi: int = BATCH_SIDE_RANGE[1],
                   seed: int = DATA_SEED_BATCH) -> list[tuple[int, int, int]]:
    """The batch of independent grids: (side, data seed, sort seed) per grid,
    sides log-uniform in [lo, hi]; grid i's features are
    gaussian_attributes(side**2, data seed) and its sort seed is
    SORT_SEED + i."""
    sides = batched_sides(count, lo, hi, seed)
    return [(side, seed * 1000 + i, SORT_SEED + i) for i, side in enumerate(sides)]
