"""Checkpoint and resume of a sort on the GPU: a sort stopped after k
reorders and resumed from its checkpoint (its permutation as the start)
ends exactly as the uninterrupted sort; the checkpoint equals the
oracle's stop state field by field; and a GPU sort resumed from the
oracle's stop state ends as the oracle's uninterrupted sort."""
import ctypes

import numpy as np
import pytest

import synthetic
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(ref):
    torch, plas = require_gpu()
    return torch, plas, plas.Context(0), ref


def _stitched(ctx, f, side, seed, stops, **kw):
    perm, ck, trace = None, None, []
    for k in list(stops) + [0]:
        perm, res = ctx.sort(f, side, seed, max_reorders=k, init_perm=perm, resume=ck, **kw)
        first = 0 if ck is None else ck.levels_done
        trace = trace[:first] + res.trace[first:]
        ck = res.checkpoint
    return perm, res, trace


def _key(trace):
    return [(t["r"], t["beta"], t["reorders"], t["energy"], t["moved"]) for t in trace]


@pytest.mark.parametrize("side,d,storage,filt,seed", [
    (48, 59, "f32", "box", 1), (40, 59, "bf16", "box", 2), (33, 3, "f32", "box3", 3), (64, 14, "f32", "box", 4)])
def test_stop_and_resume_equals_uninterrupted(env, side, d, storage, filt, seed):
    torch, plas, ctx, ref = env
    F = np.ascontiguousarray(synthetic.gaussian_attributes(side * side, seed)[:d])
    f = torch.from_numpy(F).cuda()
    full_perm, full = ctx.sort(f, side, seed, storage=storage, filter=filt)
    assert full.checkpoint.done and full.checkpoint.reorders == full.reorders
    starts = np.cumsum([0] + [t["reorders"] for t in full.trace])[:-1]
    for stops in ([1], [int(starts[len(starts) // 2])], [full.reorders - 1], [5, 40, int(starts[-1]) + 1]):
        perm, res, trace = _stitched(ctx, f, side, seed, stops, storage=storage, filter=filt)
        assert torch.equal(perm, full_perm), stops
        assert res.reorders == full.reorders and res.energy_fixed == full.energy_fixed
        assert res.levels == full.levels and _key(trace) == _key(full.trace), stops


def test_checkpoint_equals_the_oracle_stop_state(env):
    torch, plas, ctx, ref = env
    side, seed = 40, 7
    F = np.ascontiguousarray(synthetic.gaussian_attributes(side * side, seed))
    f = torch.from_numpy(F).cuda()
    for k in (1, 3, 17, 60, 150):
        perm, res = ctx.sort(f, side, seed, max_reorders=k)
        want = ref.sort(F, side, seed, max_reorders=k)
        c, s = res.checkpoint, want.state
        assert np.array_equal(perm.cpu().numpy(), want.perm)
        assert (c.done, c.reorders, c.shift_draws, c.level, c.levels_done, c.dy, c.dx, c.has_prev,
                c.just_shifted, c.energy_prev, c.energy_last, c.level_reorders, c.level_moved) == \
               (s.done, s.k, s.j, s.level, s.levels_run, s.dy, s.dx, s.has_prev, s.just_shifted,
                s.E_prev, s.E_last, s.level_reorders, s.level_moved), k


def test_resume_from_the_oracle_stop_state(env):
    torch, plas, ctx, ref = env
    side, seed = 36, 8
    F = np.ascontiguousarray(synthetic.gaussian_attributes(side * side, seed))
    full = ref.sort(F, side, seed)
    stopped = ref.sort(F, side, seed, max_reorders=full.reorders // 2)
    s = stopped.state
    c = plas.Checkpoint()
    c.struct_size = ctypes.sizeof(plas.Checkpoint)
    c.done, c.reorders, c.shift_draws, c.level, c.levels_done = s.done, s.k, s.j, s.level, s.levels_run
    c.dy, c.dx, c.has_prev, c.just_shifted = s.dy, s.dx, s.has_prev, s.just_shifted
    c.energy_prev, c.energy_last, c.level_reorders, c.level_moved = s.E_prev, s.E_last, s.level_reorders, \
        s.level_moved
    init = torch.from_numpy(stopped.perm.copy()).cuda()
    perm, res = ctx.sort(torch.from_numpy(F).cuda(), side, seed, init_perm=init, resume=c)
    assert np.array_equal(perm.cpu().numpy(), full.perm)
    assert res.reorders == full.reorders and res.energy_fixed == full.energy


def test_resume_errors_and_finished_sorts(env):
    torch, plas, ctx, ref = env
    side, seed = 24, 9
    f = torch.from_numpy(synthetic.gaussian_attributes(side * side, seed)).cuda()
    perm, res = ctx.sort(f, side, seed, max_reorders=10)
    ck = res.checkpoint
    with pytest.raises(plas.PlasError) as e:
        ctx.sort(f, side, seed, resume=ck)  # no init_perm
    assert e.value.status == plas.ERR_INVALID_ARGUMENT
    bad = plas.Checkpoint.from_buffer_copy(ck)
    bad.level = 10_000
    with pytest.raises(plas.PlasError) as e:
        ctx.sort(f, side, seed, init_perm=perm, resume=bad)
    assert e.value.status == plas.ERR_INVALID_ARGUMENT
    bad = plas.Checkpoint.from_buffer_copy(ck)
    bad.struct_size = 8
    with pytest.raises(plas.PlasError) as e:
        ctx.sort(f, side, seed, init_perm=perm, resume=bad)
    assert e.value.status == plas.ERR_INVALID_ARGUMENT
    # A stop at the same k again changes nothing; a finished sort stays finished.
    p2, r2 = ctx.sort(f, side, seed, init_perm=perm, resume=ck, max_reorders=10)
    assert torch.equal(p2, perm) and r2.reorders == 10
    full_perm, full = ctx.sort(f, side, seed)
    p3, r3 = ctx.sort(f, side, seed, init_perm=full_perm, resume=full.checkpoint)
    assert torch.equal(p3, full_perm) and r3.reorders == full.reorders and r3.checkpoint.done
    # Batches start from their items.
    prm = plas._sort_params()
    prm.resume = ctypes.pointer(ck)
    items = (plas.BatchItem * 1)()
    out = torch.empty(side * side, dtype=torch.int32, device="cuda")
    items[0].features, items[0].n, items[0].d, items[0].side = f.data_ptr(), side * side, 59, side
    items[0].perm_out = out.data_ptr()
    cfg = plas._batch_config(False, 0, False, None)[0]
    assert plas.library().plas_sort_batch(ctx._h, items, 1, ctypes.byref(prm), ctypes.byref(cfg), None) == \
        plas.ERR_INVALID_ARGUMENT


def test_batch_checkpoints_equal_single_sort_checkpoints(env):
    torch, plas, ctx, ref = env
    sides, seeds = [24, 33, 40], [11, 12, 13]
    feats = [torch.from_numpy(synthetic.gaussian_attributes(s * s, s)).cuda() for s in sides]
    for max_reorders in (7, 0):
        perms, results, _ = ctx.sort_batch(feats, sides=sides, seeds=seeds, max_reorders=max_reorders)
        for f, s, seed, perm, res in zip(feats, sides, seeds, perms, results):
            p1, r1 = ctx.sort(f, s, seed, max_reorders=max_reorders)
            assert torch.equal(p1, perm)
            a, b = r1.checkpoint, res.checkpoint
            assert bytes(a) == bytes(b), (s, max_reorders)
            assert a.done == (max_reorders == 0)


def test_profiled_resume_counts_only_the_reorders_it_ran(env):
    torch, plas, ctx, ref = env
    side, seed = 32, 21
    f = torch.from_numpy(synthetic.gaussian_attributes(side * side, seed)).cuda()
    perm, res = ctx.sort(f, side, seed, max_reorders=50)
    p2, r2 = ctx.sort(f, side, seed, init_perm=perm, resume=res.checkpoint, profile=True)
    ran = r2.reorders - 50
    # Every 32nd reorder slot of this call is timed.
    assert r2.assign_launches == (ran + 31) // 32 and r2.blur_launches == 2 * r2.assign_launches
