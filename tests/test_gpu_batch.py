"""GPU parity of batched sorts (plas_sort_batch): every sort of a batch must
equal, bit for bit, the same sort run alone through plas_sort (itself equal
to the oracle, and checked against it here on the small cases) -- the
permutation, reorder and level counts, integer energy and per-level trace --
whatever runs beside it, with direct launches or graph replay, under any
launch shapes of the tuning table."""
import numpy as np
import pytest

import synthetic
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(ref):
    torch, plas = require_gpu()
    return torch, plas, plas.Context(0), ref


def _same(res_a, perm_a, res_b, perm_b):
    assert res_a.reorders == res_b.reorders
    assert res_a.levels == res_b.levels
    assert res_a.energy_fixed == res_b.energy_fixed
    assert res_a.scale_shift == res_b.scale_shift
    assert len(res_a.trace) == len(res_b.trace)
    for a, b in zip(res_a.trace, res_b.trace):
        assert (a["r"], a["beta"], a["reorders"], a["energy"], a["moved"]) == \
               (b["r"], b["beta"], b["reorders"], b["energy"], b["moved"])
    assert np.array_equal(perm_a, perm_b)


# (side, d, layout, storage, seed): mixed channel counts, layouts and storages
MIXED = [(2, 3, "cn", "f32", 1), (3, 59, "cn", "bf16", 2), (5, 14, "nc", "f32", 3), (16, 59, "cn", "f32", 4),
         (17, 64, "nc", "bf16", 5), (31, 8, "cn", "f32", 6), (48, 59, "cn", "bf16", 7), (64, 59, "cn", "f32", 8),
         (40, 1, "cn", "f32", 9), (33, 32, "nc", "bf16", 10)]


def _mixed_inputs(torch):
    feats = []
    for side, d, layout, storage, seed in MIXED:
        n = side * side
        F = synthetic.gaussian_attributes(n, seed, layout) if d == 59 else \
            synthetic.random_features(n, d, seed, layout, -2.0, 2.0)
        feats.append((F, torch.from_numpy(F).cuda()))
    return feats


@pytest.fixture(scope="module")
def mixed_alone(env):
    torch, plas, ctx, ref = env
    feats = _mixed_inputs(torch)
    alone = []
    for (side, d, layout, storage, seed), (_, f) in zip(MIXED, feats):
        perm, res = ctx.sort(f, side, seed, layout, storage=storage)
        alone.append((perm.cpu().numpy(), res))
    return feats, alone


@pytest.mark.parametrize("graph,rps,tune", [
    (False, 0, None),
    (True, 0, None),
    (False, 5, None),
    (True, 7, None),  # rounded up to 8 with graph replay
    (False, 3, [dict(side_lo=2, side_hi=20, blur_waves_per_block=1, assign_blocks=1),
                dict(side_lo=21, side_hi=100, blur_waves_per_block=2, assign_blocks=3)]),
    (True, 0, [dict(side_lo=2, side_hi=100, blur_waves_per_block=1, assign_blocks=2)]),
])
def test_mixed_batch_equals_single_sorts(env, mixed_alone, graph, rps, tune):
    torch, plas, ctx, ref = env
    feats, alone = mixed_alone
    perms, results, b = ctx.sort_batch(
        [f for _, f in feats], sides=[m[0] for m in MIXED], seeds=[m[4] for m in MIXED],
        layouts=[m[2] for m in MIXED], storages=[m[3] for m in MIXED], graph=graph,
        reorders_per_sync=rps, tune=tune)
    assert b.sorts == len(MIXED)
    if graph:
        assert b.graph_builds >= 1
    for (pa, ra), pb, rb in zip(alone, perms, results):
        _same(ra, pa, rb, pb.cpu().numpy())


def test_batch_matches_oracle_directly(env, mixed_alone):
    torch, plas, ctx, ref = env
    feats, _ = mixed_alone
    pick = [0, 2, 3, 5, 8]
    perms, results, _ = ctx.sort_batch(
        [feats[i][1] for i in pick], sides=[MIXED[i][0] for i in pick], seeds=[MIXED[i][4] for i in pick],
        layouts=[MIXED[i][2] for i in pick], storages=[MIXED[i][3] for i in pick], graph=True)
    for i, perm, res in zip(pick, perms, results):
        side, d, layout, storage, seed = MIXED[i]
        want = ref.sort(feats[i][0], side, seed, layout, storage_bf16=(storage == "bf16"))
        assert want.status == 0
        assert res.reorders == want.reorders and res.energy_fixed == want.energy
        assert np.array_equal(perm.cpu().numpy(), want.perm)


def test_init_perm_and_truncation_in_a_batch(env):
    torch, plas, ctx, ref = env
    sides = [24, 40, 57]
    feats = [torch.from_numpy(synthetic.gaussian_attributes(s * s, 20 + s)).cuda() for s in sides]
    inits = [torch.from_numpy(synthetic.random_permutation(s * s, s)).cuda() for s in sides]
    for max_reorders in (0, 11):
        perms, results, _ = ctx.sort_batch(feats, sides=sides, seeds=[5, 6, 7], init_perms=inits,
                                           max_reorders=max_reorders, graph=True)
        for f, s, seed, init, perm, res in zip(feats, sides, [5, 6, 7], inits, perms, results):
            p1, r1 = ctx.sort(f, s, seed, init_perm=init, max_reorders=max_reorders)
            _same(r1, p1.cpu().numpy(), res, perm.cpu().numpy())
            if max_reorders:
                assert res.reorders == max_reorders


def test_batch_of_medium_grids_full_sorts(env):
    """Eight grids of the batch workload's distribution, 128 .. 256, whole sorts."""
    torch, plas, ctx, ref = env
    work = synthetic.batch_workload(8, 128, 256, 7)
    feats = [torch.from_numpy(synthetic.gaussian_attributes(s * s, ds)).cuda() for s, ds, _ in work]
    perms, results, b = ctx.sort_batch(feats, sides=[w[0] for w in work], seeds=[w[2] for w in work],
                                       graph=True)
    for (s, ds, seed), f, perm, res in zip(work, feats, perms, results):
        p1, r1 = ctx.sort(f, s, seed)
        _same(r1, p1.cpu().numpy(), res, perm.cpu().numpy())
    assert b.reorder_slots >= max(r.reorders for r in results)


def test_full_batch_workload_truncated(env):
    """The 64-grid batch workload (sides 128 .. 724), first 40 reorders of
    every sort, graph replay, against single truncated sorts."""
    torch, plas, ctx, ref = env
    work = synthetic.batch_workload()
    feats = [torch.from_numpy(synthetic.gaussian_attributes(s * s, ds)).cuda() for s, ds, _ in work]
    perms, results, b = ctx.sort_batch(feats, sides=[w[0] for w in work], seeds=[w[2] for w in work],
                                       graph=True, max_reorders=40)
    assert b.sorts == 64
    for i in range(0, 64, 5):
        s, ds, seed = work[i]
        p1, r1 = ctx.sort(feats[i], s, seed, max_reorders=40)
        _same(r1, p1.cpu().numpy(), results[i], perms[i].cpu().numpy())


def test_profile_and_stats(env):
    torch, plas, ctx, ref = env
    sides = [32, 48]
    feats = [torch.from_numpy(synthetic.gaussian_attributes(s * s, s)).cuda() for s in sides]
    perms, results, b = ctx.sort_batch(feats, sides=sides, seeds=[1, 2], profile=True, graph=True)
    assert b.graph_builds == 0  # profiling runs direct launches
    # The controller step runs at the end of the assignment: no time of its own.
    assert b.step_ms == 0 and b.blur_ms > 0 and b.assign_ms > 0
    assert b.chunks >= 1 and b.reorder_slots == 32 * b.chunks
    assert max(r.total_ms for r in results) <= b.total_ms + 1e-6
    for f, s, seed, perm, res in zip(feats, sides, [1, 2], perms, results):
        p1, r1 = ctx.sort(f, s, seed)
        _same(r1, p1.cpu().numpy(), res, perm.cpu().numpy())


def test_autotune_table_covers_the_batch_and_keeps_results(env):
    torch, plas, ctx, ref = env
    sides = [20, 23, 45, 90]
    feats = [torch.from_numpy(synthetic.gaussian_attributes(s * s, 100 + s)).cuda() for s in sides]
    table = ctx.autotune_batch(feats, sides=sides, seeds=[1, 2, 3, 4], graph=True)
    assert table
    for s in sides:
        e = [t for t in table if t["side_lo"] <= s <= t["side_hi"]]
        assert e, s
        assert e[0]["blur_waves_per_block"] in (1, 2, 4) and e[0]["assign_blocks"] >= 0
    perms, results, _ = ctx.sort_batch(feats, sides=sides, seeds=[1, 2, 3, 4], tune=table, graph=True)
    for f, s, seed, perm, res in zip(feats, sides, [1, 2, 3, 4], perms, results):
        p1, r1 = ctx.sort(f, s, seed)
        _same(r1, p1.cpu().numpy(), res, perm.cpu().numpy())


def test_batch_errors(env):
    torch, plas, ctx, ref = env
    f = torch.from_numpy(synthetic.gaussian_attributes(64, 1)).cuda()
    out = torch.empty(64, dtype=torch.int32, device="cuda")
    with pytest.raises(plas.PlasError) as e:
        ctx.sort_batch([f, f], sides=[8, 8], out=out)
    assert e.value.status == plas.ERR_INVALID_ARGUMENT
    with pytest.raises(plas.PlasError) as e:
        ctx.sort_batch([f], sides=[8], tune=[dict(side_lo=1, side_hi=100, blur_waves_per_block=3)])
    assert e.value.status == plas.ERR_INVALID_ARGUMENT
    bad = f.clone()
    bad[2, 7] = float("nan")
    with pytest.raises(plas.PlasError) as e:
        ctx.sort_batch([f, bad], sides=[8, 8])
    assert e.value.status == plas.ERR_NONFINITE
    with pytest.raises(plas.PlasError) as e:
        ctx.sort_batch([f], sides=[7])
    assert e.value.status == plas.ERR_INVALID_ARGUMENT
    # The context still sorts afterwards, alone and in batches.
    perms, results, _ = ctx.sort_batch([f], sides=[8], seeds=[3])
    p1, r1 = ctx.sort(f, 8, 3)
    _same(r1, p1.cpu().numpy(), results[0], perms[0].cpu().numpy())
    _, _, b = ctx.sort_batch([], sides=[])
    assert b.sorts == 0


def test_full_batch_workload_whole_sorts(env):
    """The 64-grid batch workload (sides 128 .. 724), whole sorts with graph
    replay: every grid equals its plain sort (permutation, reorders, levels,
    energy and per-level trace)."""
    torch, plas, ctx, ref = env
    work = synthetic.batch_workload()
    feats = [torch.from_numpy(synthetic.gaussian_attributes(s * s, ds)).cuda() for s, ds, _ in work]
    perms, results, b = ctx.sort_batch(feats, sides=[w[0] for w in work], seeds=[w[2] for w in work],
                                       graph=True)
    assert b.sorts == 64
    for i, (s, ds, seed) in enumerate(work):
        p1, r1 = ctx.sort(feats[i], s, seed)
        _same(r1, p1.cpu().numpy(), results[i], perms[i].cpu().numpy())
