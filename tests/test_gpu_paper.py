"""GPU checks of the paper-comparable experiments (App. C): the VAD quality
measure against the oracle's and its closed forms, the random 512 x 512 x 3
RGB sort against the oracle's stored result (permutation, counts, VAD), and
sorts under other improvement thresholds (the threshold sweep) against the
oracle directly."""
import ctypes
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


@pytest.mark.parametrize("name", ["sort_512_rgb", "sort_512_rgb_box3"])
def test_rgb_512_sort_matches_stored_oracle_result(env, name):
    torch, plas, ctx, ref = env
    path = os.path.join(GOLDEN, f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    gold = json.load(open(path))
    side = gold["side"]
    F = synthetic.random_rgb_grid(side, gold["data_seed"])
    f = torch.from_numpy(F).cuda()
    perm, res = ctx.sort(f, side, gold["sort_seed"], filter=gold.get("filter", "box"))
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


# The Gaussian-like target filter (three box passes per axis): whole sorts
# against the oracle's, bit for bit, in both storages and layouts.
@pytest.mark.parametrize("side,d,layout,storage,seed", [
    (64, 3, "cn", "f32", 1), (48, 59, "cn", "f32", 2), (40, 59, "cn", "bf16", 3), (33, 14, "nc", "f32", 4),
    (2, 3, "cn", "f32", 5), (17, 1, "cn", "f32", 6)])
def test_box3_filter_sort_matches_oracle(env, side, d, layout, storage, seed):
    torch, plas, ctx, ref = env
    n = side * side
    if d == 3:
        F = synthetic.random_rgb_grid(side, seed) if layout == "cn" else None
    else:
        F = synthetic.gaussian_attributes(n, seed, layout)[:d] if layout == "cn" else \
            synthetic.random_features(n, d, seed, layout, -2.0, 2.0)
    if F is None:
        F = synthetic.random_features(n, d, seed, layout, 0.0, 255.0)
    F = np.ascontiguousarray(F)
    perm, res = ctx.sort(torch.from_numpy(F).cuda(), side, seed, layout, storage=storage, filter="box3",
                         profile=True)
    want = ref.sort(F, side, seed, layout, storage_bf16=(storage == "bf16"), filter="box3")
    assert want.status == 0
    assert res.reorders == want.reorders and res.levels == want.levels
    assert res.energy_fixed == want.energy and res.scale_shift == want.scale_shift
    assert [(t["r"], t["reorders"], t["energy"], t["moved"]) for t in res.trace] == \
           [(t["r"], t["reorders"], t["energy"], t["moved"]) for t in want.trace]
    assert np.array_equal(perm.cpu().numpy(), want.perm)
    # Six blur passes per timed reorder.
    assert res.blur_launches == 6 * res.assign_launches


def test_box3_filter_truncated_at_the_coarsest_levels(env):
    """256 x 256, D = 59: the first 24 reorders (radius 127 and below, six
    passes of windows up to 255 cells) against the oracle."""
    torch, plas, ctx, ref = env
    side = 256
    F = synthetic.gaussian_attributes(side * side, 12)
    perm, res = ctx.sort(torch.from_numpy(F).cuda(), side, 9, filter="box3", max_reorders=24)
    want = ref.sort(F, side, 9, filter="box3", max_reorders=24)
    assert res.reorders == want.reorders == 24 and res.energy_fixed == want.energy
    assert np.array_equal(perm.cpu().numpy(), want.perm)


def test_box3_filter_in_batches_and_servers(env):
    """A batch and a server with the filter give each sort's single-sort
    result, bit for bit; unknown filters are rejected."""
    torch, plas, ctx, ref = env
    sides, seeds = [16, 24, 33], [1, 2, 3]
    feats = [torch.from_numpy(synthetic.gaussian_attributes(s * s, 40 + s)).cuda() for s in sides]
    alone = [ctx.sort(f, s, seed, filter="box3") for f, s, seed in zip(feats, sides, seeds)]
    for graph in (False, True):
        perms, results, _ = ctx.sort_batch(feats, sides=sides, seeds=seeds, filter="box3", graph=graph)
        for (p1, r1), p, r in zip(alone, perms, results):
            assert torch.equal(p1, p) and r1.reorders == r.reorders and r1.energy_fixed == r.energy_fixed
    srv = plas.Server(ctx, memory_budget=1 << 30, filter="box3")
    ids = [srv.submit(f, s, seed) for f, s, seed in zip(feats, sides, seeds)]
    done = {}
    for _ in range(100000):
        running, waiting = srv.step()
        for job, st, p, r in srv.poll():
            assert st == plas.OK
            done[job] = (p, r)
        if len(done) == len(ids):
            break
    for job, (p1, r1) in zip(ids, alone):
        p, r = done[job]
        assert torch.equal(p1, p) and r1.reorders == r.reorders
    srv.close()
    out = torch.empty(64, dtype=torch.int32, device="cuda")
    f = torch.from_numpy(synthetic.gaussian_attributes(64, 1)).cuda()
    bad = plas._sort_params()
    bad.filter = 2
    assert plas.library().plas_sort(ctx._h, ctypes.c_void_p(f.data_ptr()), 64, 59, 8, plas.LAYOUT_CN, 0,
                                    ctypes.byref(bad), ctypes.c_void_p(out.data_ptr()), None) == \
        plas.ERR_INVALID_ARGUMENT
