"""GPU parity of the bfloat16-storage path against the oracle's bfloat16
mode (bit for bit: permutation, trace, energies and every stage), and the
precision gate of the 1448 x 1448 workload: the bfloat16 sort's final
float64 energy within 0.5 % of the float32 sort's on the same GPU."""
import numpy as np
import pytest

import synthetic
from gpu_util import bits, from_working_layout, require_gpu, to_working_layout

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(ref):
    torch, plas = require_gpu()
    return torch, plas, plas.Context(0), ref


def _bf16(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(torch.bfloat16).float().numpy()


@pytest.mark.parametrize("side,d,r", [(7, 3, 2), (17, 14, 5), (33, 59, 7), (64, 59, 31), (100, 3, 9),
                                      (256, 59, 127), (250, 8, 300),
                                      # radii whose leaving values a wave keeps in
                                      # registers (48..128), both ends, one past
                                      (97, 59, 48), (301, 59, 128), (301, 59, 129), (1000, 59, 100),
                                      (150, 32, 75), (77, 8, 60)])
def test_blur_bf16_bitwise(env, side, d, r):
    torch, plas, ctx, ref = env
    rng = np.random.default_rng(side + d + r)
    G = _bf16(torch, rng.standard_normal((side * side, d)) * rng.uniform(0.01, 10, d))
    dp = plas.padded_channels(d)
    T = from_working_layout(ctx.stage_blur(to_working_layout(torch, G, dp, "bf16"), side, r), d)
    want = ref.blur(G, side, r, storage_bf16=True)
    assert np.array_equal(bits(T), bits(want))


@pytest.mark.parametrize("side,d,beta,r,dy,dx", [(16, 59, 16, 3, 5, 9), (21, 5, 9, 4, 20, 20),
                                                 (64, 59, 32, 31, 13, 50), (128, 59, 16, 1, 77, 3)])
def test_assign_bf16_bitwise(env, side, d, beta, r, dy, dx):
    torch, plas, ctx, ref = env
    N = side * side
    F = _bf16(torch, synthetic.gaussian_attributes(N, side + d)[:d])
    st, s, _ = ref.scale_shift(F)
    P = synthetic.random_permutation(N, side)
    G = ref.gather(F, P)
    T = ref.blur(G, side, r, storage_bf16=True)
    keys = ref.draw(0x5EED, 1, side + beta)
    dp = plas.padded_channels(d)
    g_dev = to_working_layout(torch, G, dp, "bf16")
    p_dev = torch.from_numpy(P.copy()).cuda()
    E, moved = ctx.stage_assign(g_dev, to_working_layout(torch, T, dp, "bf16"), p_dev, side, beta, dy, dx,
                                keys, s)
    G_ref, P_ref = G.copy(), P.copy()
    E_ref, moved_ref = ref.assign(G_ref, T, P_ref, side, beta, dy, dx, keys, s)
    assert (E, moved) == (E_ref, moved_ref)
    assert np.array_equal(p_dev.cpu().numpy(), P_ref)
    assert np.array_equal(bits(from_working_layout(g_dev, d)), bits(G_ref))


def _compare(res, perm, want):
    assert res.reorders == want.reorders and res.levels == want.levels
    assert res.energy_fixed == want.energy and res.scale_shift == want.scale_shift
    assert [(t["reorders"], t["energy"], t["moved"]) for t in res.trace] == \
           [(t["reorders"], t["energy"], t["moved"]) for t in want.trace]
    assert np.array_equal(perm, want.perm)


@pytest.mark.parametrize("side,d,layout,seed", [(8, 59, "cn", 1), (17, 14, "nc", 2), (33, 3, "cn", 3),
                                                (64, 59, "cn", synthetic.SORT_SEED)])
def test_small_bf16_sorts_match_oracle(env, side, d, layout, seed):
    torch, plas, ctx, ref = env
    N = side * side
    F = synthetic.gaussian_attributes(N, seed % 97, layout) if d == 59 else \
        synthetic.random_features(N, d, seed, layout, -2, 2)
    perm, res = ctx.sort(torch.from_numpy(F).cuda(), side, seed, layout, storage="bf16")
    want = ref.sort(F, side, seed, layout, storage_bf16=True)
    _compare(res, perm.cpu().numpy(), want)


def test_bf16_input_features(env):
    """bfloat16 features in (as torch.bfloat16) sort like their float32
    values with bfloat16 storage."""
    torch, plas, ctx, ref = env
    side = 32
    F = synthetic.gaussian_attributes(side * side, 4)
    Fb = torch.from_numpy(F).to(torch.bfloat16)
    perm, res = ctx.sort(Fb.cuda(), side, 9, storage="bf16")
    want = ref.sort(Fb.float().numpy(), side, 9, storage_bf16=True)
    _compare(res, perm.cpu().numpy(), want)
    perm32, _ = ctx.sort(Fb.cuda(), side, 9, storage="f32")
    want32 = ref.sort(Fb.float().numpy(), side, 9)
    assert np.array_equal(perm32.cpu().numpy(), want32.perm)


@pytest.mark.parametrize("max_reorders,start_radius", [(4, 0.0), (5, 2.0)])
def test_precision_workload_truncated_matches_oracle(env, max_reorders, start_radius):
    """1448 x 1448, D = 59, bfloat16 storage: the first reorders of the
    coarsest and of the finest levels, bit-exact."""
    torch, plas, ctx, ref = env
    side = 1448
    F = synthetic.gaussian_attributes(side * side, synthetic.DATA_SEED_PRECISION)
    perm, res = ctx.sort(torch.from_numpy(F).cuda(), side, synthetic.SORT_SEED, storage="bf16",
                         max_reorders=max_reorders, start_radius=start_radius)
    want = ref.sort(F, side, synthetic.SORT_SEED, storage_bf16=True, max_reorders=max_reorders,
                    start_radius=start_radius)
    _compare(res, perm.cpu().numpy(), want)


def test_precision_workload_energy_gap(env):
    """Full 1448 x 1448 sorts in float32 and in bfloat16 storage: the final
    float64 energy of the bfloat16 arrangement (on the original features, at
    r = 1) is within 0.5 % of the float32 arrangement's."""
    torch, plas, ctx, ref = env
    side = 1448
    F = synthetic.gaussian_attributes(side * side, synthetic.DATA_SEED_PRECISION)
    f_dev = torch.from_numpy(F).cuda()
    p32, r32 = ctx.sort(f_dev, side, synthetic.SORT_SEED)
    p16, r16 = ctx.sort(f_dev, side, synthetic.SORT_SEED, storage="bf16")
    e32 = ref.grid_energy_f64(F, p32.cpu().numpy(), side, 1)
    e16 = ref.grid_energy_f64(F, p16.cpu().numpy(), side, 1)
    gap = e16 / e32 - 1
    print(f"1448^2 D=59: fp32 {r32.reorders} reorders E64 {e32:.6f}; bf16 {r16.reorders} reorders "
          f"E64 {e16:.6f}; gap {100 * gap:+.3f} %")
    assert abs(gap) < 0.005


@pytest.mark.parametrize("side,d,r", [(16, 59, 1), (64, 14, 3)])
def test_grid_energy_bf16_matches_oracle(env, side, d, r):
    torch, plas, ctx, ref = env
    N = side * side
    F = synthetic.random_features(N, d, side, "cn", -3, 3)
    perm = synthetic.random_permutation(N, side)
    E, s, mean = ctx.grid_energy(torch.from_numpy(F).cuda(), torch.from_numpy(perm).cuda(), side, r,
                                 storage="bf16")
    st, E_ref, s_ref, mean_ref = ref.grid_energy(F, perm, side, r, storage_bf16=True)
    assert (E, s) == (E_ref, s_ref)
