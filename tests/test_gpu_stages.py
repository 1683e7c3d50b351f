"""GPU parity of each step of a reorder against the CPU oracle, through the
C ABI stage entry points (include/plas_stages.h). Integer and index results
must be equal; float results must be equal bit for bit (the kernels and the
oracle evaluate the same IEEE float32 operations in the same order)."""
import numpy as np
import pytest

import synthetic
from gpu_util import bits, from_working_layout, require_gpu, to_working_layout

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(ref):
    torch, plas = require_gpu()
    return torch, plas, plas.Context(0), ref


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 17, 256, 257, 1000, 4096, 65536, 1 << 18, 1024 * 1024,
                               1448 * 1448])
def test_bijection(env, n):
    torch, plas, ctx, ref = env
    keys = ref.draw(0x5EED, 0, n)
    got = ctx.stage_bijection(n, keys).cpu().numpy()
    want = ref.bijection_table(n, keys)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("beta", [2, 3, 4, 15, 16, 17, 31, 32, 33, 100, 341, 512, 723])
def test_group_table(env, beta):
    torch, plas, ctx, ref = env
    keys = ref.draw(7, 1, beta)
    packed = ctx.stage_group_table(beta, keys).cpu().numpy().astype(np.int64)
    got = (packed >> 16) * beta + (packed & 0xFFFF)
    assert np.array_equal(got, ref.bijection_table(beta * beta, keys))


BLUR_CASES = [
    # (side, d, r)
    (2, 1, 1), (3, 3, 1), (5, 2, 0), (7, 3, 2), (16, 4, 3), (17, 14, 5), (33, 59, 7), (33, 59, 40),
    (64, 59, 31), (64, 64, 1), (100, 3, 9), (129, 16, 63), (256, 59, 127), (250, 8, 300),
    # float32 radii of the second load stream on small grids (48..192 and
    # past them)
    (97, 59, 48), (301, 59, 192), (301, 59, 193), (150, 32, 75), (77, 4, 60),
    # float32 grids of more than 128 MiB keep the leaving values of
    # 48 <= r <= 192 in registers: both ends, the first radius past them,
    # and cells of 64, 32 and 4 channels
    (800, 59, 48), (800, 59, 192), (800, 59, 193), (1024, 59, 100), (1100, 32, 75), (3000, 4, 60),
    # more than 1024 lines of 64 float32 channels: the 64-row ring (leaving
    # values from the ring up to r = 15, from registers up to r = 64, then
    # from a second load stream)
    (1100, 59, 15), (1100, 59, 16), (1100, 59, 64), (1100, 59, 65),
]


@pytest.mark.parametrize("side,d,r", BLUR_CASES)
def test_blur_bitwise(env, side, d, r):
    torch, plas, ctx, ref = env
    rng = np.random.default_rng(side * 1000 + d * 10 + r)
    G = rng.standard_normal((side * side, d)).astype(np.float32) * rng.uniform(0.01, 10, d).astype(np.float32)
    dp = plas.padded_channels(d)
    T = from_working_layout(ctx.stage_blur(to_working_layout(torch, G, dp), side, r), d)
    want = ref.blur(G, side, r)
    assert np.array_equal(bits(T), bits(want))


# Radius sweeps over the boundaries of the ways a pass gets its leaving
# values, on grids large enough for the register slots (more than 128 MiB):
# with the 128-row ring the ring itself (r <= 47), registers (48..192) and a
# second load stream (r > 192, up to r > w / 2); with the 64-row ring (more
# than 1024 lines) the ring (r <= 15), registers (16..64) and the stream.
SWEEPS = [
    (760, [1, 15, 16, 17, 31, 32, 33, 46, 47, 48, 49, 50, 63, 64, 65, 79, 80, 81, 95, 96, 97, 127, 128, 129,
           175, 176, 177, 190, 191, 192, 193, 194, 255, 300, 379, 380, 759]),
    (1100, [14, 15, 16, 17, 31, 32, 33, 47, 48, 49, 63, 64, 65, 66, 200]),
]


@pytest.mark.parametrize("side,radii", SWEEPS)
def test_blur_radius_sweep_large_grid(env, side, radii):
    torch, plas, ctx, ref = env
    d = 59
    rng = np.random.default_rng(side)
    G = (rng.standard_normal((side * side, d)) * rng.uniform(0.01, 10, d)).astype(np.float32)
    dp = plas.padded_channels(d)
    g = to_working_layout(torch, G, dp)
    for r in radii:
        T = from_working_layout(ctx.stage_blur(g, side, r), d)
        want = ref.blur(G, side, r)
        assert np.array_equal(bits(T), bits(want)), (side, r)


def test_blur_padding_stays_zero(env):
    torch, plas, ctx, ref = env
    G = np.random.default_rng(1).standard_normal((20 * 20, 5)).astype(np.float32)
    T = ctx.stage_blur(to_working_layout(torch, G, 8), 20, 3).cpu().numpy()
    assert np.all(T[:, 5:] == 0.0)


ASSIGN_CASES = [
    # (side, d, beta, r, dy, dx)
    (2, 3, 2, 1, 0, 0), (3, 3, 3, 1, 1, 2), (4, 1, 4, 1, 3, 3), (16, 59, 16, 3, 5, 9),
    (17, 14, 16, 2, 16, 0), (21, 3, 8, 2, 4, 11), (21, 5, 9, 4, 20, 20), (33, 59, 16, 1, 7, 30),
    (64, 59, 32, 31, 13, 50), (64, 64, 16, 5, 0, 63), (100, 16, 33, 32, 99, 1), (128, 59, 16, 1, 77, 3),
]


@pytest.mark.parametrize("side,d,beta,r,dy,dx", ASSIGN_CASES)
def test_assign_bitwise(env, side, d, beta, r, dy, dx):
    torch, plas, ctx, ref = env
    N = side * side
    F = synthetic.gaussian_attributes(N, side + d)[:d] if d <= 59 else \
        synthetic.random_features(N, d, side)
    F = np.ascontiguousarray(F)
    st, s, _ = ref.scale_shift(F)
    P = synthetic.random_permutation(N, side * 7 + d)
    G = ref.gather(F, P)
    T = ref.blur(G, side, r)
    keys = ref.draw(0x5EED, 1, side + beta)
    dp = plas.padded_channels(d)
    g_dev = to_working_layout(torch, G, dp)
    t_dev = to_working_layout(torch, T, dp)
    p_dev = torch.from_numpy(P.copy()).cuda()
    E, moved = ctx.stage_assign(g_dev, t_dev, p_dev, side, beta, dy, dx, keys, s)
    G_ref, P_ref = G.copy(), P.copy()
    E_ref, moved_ref = ref.assign(G_ref, T, P_ref, side, beta, dy, dx, keys, s)
    assert E == E_ref and moved == moved_ref
    assert np.array_equal(p_dev.cpu().numpy(), P_ref)
    assert np.array_equal(bits(from_working_layout(g_dev, d)), bits(G_ref))
    assert np.all(g_dev.cpu().numpy()[:, d:] == 0.0)


@pytest.mark.parametrize("side,d,r", [(16, 59, 2), (33, 3, 5), (64, 14, 1), (200, 59, 20)])
def test_energy(env, side, d, r):
    torch, plas, ctx, ref = env
    F = synthetic.random_features(side * side, d, side, low=-5, high=5)
    st, s, _ = ref.scale_shift(F)
    G = ref.gather(F, synthetic.random_permutation(side * side, 3))
    T = ref.blur(G, side, r)
    dp = plas.padded_channels(d)
    E = ctx.stage_energy(to_working_layout(torch, G, dp), to_working_layout(torch, T, dp), side, s)
    assert E == ref.energy_fixed(G, T, s)
