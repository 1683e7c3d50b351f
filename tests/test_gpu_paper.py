"""GPU checks of the paper-comparable experiments (App. C): the VAD quality
measure against the oracle's and its closed forms, the random 512 x 512 x 3
RGB sort against the oracle's stored result (permutation, counts, VAD), and
sorts under other improvement thresholds (the threshold sweep) against the
oracle directly."""
import hashlib
import json
import os

import numpy as np
import pytest

import synthetic
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def env(ref):
    torch, plas = require_gpu()
    return torch, plas, plas.Context(0), ref


def test_vad_hand_example_and_closed_form(env):
    torch, plas, ctx, ref = env
    # 2x2, one channel [[0, 1], [3, 5]]: pairs 1, 2, 3, 4 -> variance 1.25.
    F = torch.tensor([[0.0, 1.0, 3.0, 5.0]], device="cuda")
    assert ctx.vad(F, None, 2) == pytest.approx(1.25, abs=1e-12)
    # Shuffled U(0, a): |X - Y| has variance a^2 / 18.
    G = torch.from_numpy(synthetic.random_rgb_grid(512, 0)).cuda()
    assert abs(ctx.vad(G, None, 512) / (255.0 ** 2 / 18.0) - 1.0) < 0.01


@pytest.mark.parametrize("side,d,layout,with_perm,bf16", [
    (2, 1, "cn", False, False), (7, 3, "nc", True, False), (64, 59, "cn", True, False),
    (100, 3, "cn", True, False), (33, 14, "nc", False, False), (48, 59, "cn", True, True)])
def test_vad_matches_oracle(env, side, d, layout, with_perm, bf16):
    torch, plas, ctx, ref = env
    n = side * side
    F = synthetic.random_features(n, d, side + d, layout, -3.0, 3.0)
    f = torch.from_numpy(F).cuda()
    if bf16:
        f = f.to(torch.bfloat16)
        F = f.float().cpu().numpy()
    perm = synthetic.random_permutation(n, side) if with_perm else None
    got = ctx.vad(f, None if perm is None else torch.from_numpy(perm).cuda(), side, layout)
    want = ref.vad(F, perm, side, layout)
    assert got == pytest.approx(want, rel=1e-10, abs=1e-14)


def test_vad_rejects_a_bad_permutation(env):
    torch, plas, ctx, ref = env
    f = torch.from_numpy(synthetic.random_rgb_grid(8, 1)).cuda()
    perm = torch.arange(64, dtype=torch.int32, device="cuda")
    perm[5] = 6
    with pytest.raises(plas.PlasError) as e:
        ctx.vad(f, perm, 8)
    assert e.value.status == plas.ERR_INVALID_ARGUMENT


def test_rgb_512_sort_matches_stored_oracle_result(env):
    torch, plas, ctx, ref = env
    path = os.path.join(GOLDEN, "sort_512_rgb.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    gold = json.load(open(path))
    side = gold["side"]
    F = synthetic.random_rgb_grid(side, gold["data_seed"])
    f = torch.from_numpy(F).cuda()
    perm, res = ctx.sort(f, side, gold["sort_seed"])
    p = perm.cpu().numpy().astype("<i4")
    assert res.reorders == gold["reorders"] and res.levels == gold["levels"]
    assert res.energy_fixed == int(gold["energy"])
    assert hashlib.sha256(p.tobytes()).hexdigest() == gold["perm_sha256"]
    assert ctx.vad(f, perm, side) == pytest.approx(gold["vad_sorted"], rel=1e-10)
    assert ctx.vad(f, None, side) == pytest.approx(gold["vad_start"], rel=1e-10)


@pytest.mark.parametrize("inv_threshold", [100, 1000, 100000])
def test_threshold_sweep_matches_oracle(env, inv_threshold):
    torch, plas, ctx, ref = env
    side = 64
    F = synthetic.random_rgb_grid(side, 7)
    perm, res = ctx.sort(torch.from_numpy(F).cuda(), side, 3, inv_threshold=inv_threshold)
    want = ref.sort(F, side, 3, inv_threshold=inv_threshold)
    assert want.status == 0
    assert res.reorders == want.reorders and res.energy_fixed == want.energy
    assert np.array_equal(perm.cpu().numpy(), want.perm)
