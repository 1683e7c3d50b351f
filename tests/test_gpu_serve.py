"""GPU tests of the sort server (plas_server_*): jobs submitted while others
run are admitted at reorder boundaries as memory frees up, and every job's
result equals, bit for bit, the same sort run alone (plas_sort)."""
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
    assert [t["energy"] for t in res_a.trace] == [t["energy"] for t in res_b.trace]
    assert np.array_equal(perm_a, perm_b)


JOBS = [  # (side, storage, data seed, sort seed)
    (16, "f32", 1, 11), (40, "bf16", 2, 12), (96, "f32", 3, 13), (23, "bf16", 4, 14),
    (64, "f32", 5, 15), (130, "bf16", 6, 16), (31, "f32", 7, 17), (77, "bf16", 8, 18),
]


def _features(torch, side, seed):
    return torch.from_numpy(synthetic.gaussian_attributes(side * side, seed)).cuda()


@pytest.mark.parametrize("graph,rps", [(False, 0), (True, 0), (True, 3)])
def test_jobs_joining_a_running_batch_equal_alone(env, graph, rps):
    torch, plas, ctx, ref = env
    feats = [_features(torch, s, ds) for s, _, ds, _ in JOBS]
    srv = plas.Server(ctx, 1 << 34, graph=graph, reorders_per_sync=rps)
    done = {}
    ids = {}
    # Jobs arrive in three waves, each while the earlier ones are running.
    waves = [[0, 1, 2], [3, 4], [5, 6, 7]]
    steps = 0
    for wave in waves:
        for i in wave:
            side, storage, _, seed = JOBS[i]
            ids[srv.submit(feats[i], side, seed, storage=storage)] = i
        for _ in range(3):
            srv.step()
            steps += 1
            for job, status, perm, res in srv.poll():
                assert status == plas.OK
                done[ids[job]] = (perm, res)
    while len(done) < len(JOBS):
        running, waiting = srv.step()
        steps += 1
        assert steps < 100000
        for job, status, perm, res in srv.poll():
            assert status == plas.OK
            done[ids[job]] = (perm, res)
    assert srv.step() == (0, 0)
    srv.close()
    for i, (side, storage, _, seed) in enumerate(JOBS):
        p1, r1 = ctx.sort(feats[i], side, seed, storage=storage)
        perm, res = done[i]
        _same(r1, p1.cpu().numpy(), res, perm.cpu().numpy())
        assert res.total_ms > 0


def test_admission_follows_the_memory_budget(env):
    torch, plas, ctx, ref = env
    sides = [48, 48, 48, 200]
    feats = [_features(torch, s, 30 + i) for i, s in enumerate(sides)]
    one = plas.job_footprint(48, 59)
    srv = plas.Server(ctx, one + one // 2)  # room for one 48 x 48 job at a time
    for i, s in enumerate(sides):
        srv.submit(feats[i], s, 40 + i)
    max_running = 0
    finished = []
    order = []
    while len(finished) < len(sides):
        running, waiting = srv.step()
        max_running = max(max_running, running)
        for job, status, perm, res in srv.poll():
            assert status == plas.OK
            finished.append((job, perm, res))
            order.append(job)
    srv.close()
    # One job at a time, first come first served; the 200 x 200 job is
    # larger than the budget and still runs once it is alone.
    assert max_running == 1
    assert order == [0, 1, 2, 3]
    assert plas.job_footprint(200, 59) > one + one // 2
    for (job, perm, res), s, f, seed in zip(finished, sides, feats, [40, 41, 42, 43]):
        p1, r1 = ctx.sort(f, s, seed)
        _same(r1, p1.cpu().numpy(), res, perm.cpu().numpy())


def test_a_bad_job_fails_alone(env):
    torch, plas, ctx, ref = env
    good = _features(torch, 24, 50)
    bad = _features(torch, 24, 51)
    bad[3, 5] = float("inf")
    srv = plas.Server(ctx, 1 << 32)
    a = srv.submit(good, 24, 1)
    b = srv.submit(bad, 24, 2)
    results = {}
    for _ in range(100000):
        srv.step()
        for job, status, perm, res in srv.poll():
            results[job] = (status, perm, res)
        if len(results) == 2:
            break
    srv.close()
    assert results[b][0] == plas.ERR_NONFINITE and results[b][1] is None
    assert results[a][0] == plas.OK
    p1, r1 = ctx.sort(good, 24, 1)
    _same(r1, p1.cpu().numpy(), results[a][2], results[a][1].cpu().numpy())


def test_other_calls_between_steps(env):
    torch, plas, ctx, ref = env
    f1, f2 = _features(torch, 56, 60), _features(torch, 36, 61)
    srv = plas.Server(ctx, 1 << 32, graph=True)
    j1 = srv.submit(f1, 56, 7)
    srv.step()
    # A plain sort and a batch on the same context while the server runs.
    p_alone, r_alone = ctx.sort(f2, 36, 8)
    perms, results, _ = ctx.sort_batch([f2], sides=[36], seeds=[8], graph=True)
    _same(r_alone, p_alone.cpu().numpy(), results[0], perms[0].cpu().numpy())
    got = None
    for _ in range(100000):
        srv.step()
        for job, status, perm, res in srv.poll():
            got = (perm, res)
        if got is not None:
            break
    srv.close()
    p1, r1 = ctx.sort(f1, 56, 7)
    _same(r1, p1.cpu().numpy(), got[1], got[0].cpu().numpy())
