"""GPU tests of the sort server (plas_server_*): jobs submitted while others
run are admitted at reorder boundaries as memory frees up, and every job's
result equals, bit for bit, the same sort run alone (plas_sort) and the CPU
oracle's sort -- for small mixed jobs and for jobs of the serving
configuration (sides 256 .. 1024, float32 and bfloat16 storage)."""
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


def test_small_jobs_match_the_oracle(env):
    """The served small jobs (the mix above, direct launches) against the CPU
    oracle itself: permutation, reorders and integer energy."""
    torch, plas, ctx, ref = env
    feats = [synthetic.gaussian_attributes(s * s, ds) for s, _, ds, _ in JOBS]
    srv = plas.Server(ctx, 1 << 34)
    ids = {srv.submit(torch.from_numpy(F).cuda(), side, seed, storage=storage): i
           for i, (F, (side, storage, _, seed)) in enumerate(zip(feats, JOBS))}
    done = _drain(plas, srv, ids, len(JOBS))
    for i, (side, storage, _, seed) in enumerate(JOBS):
        perm, res = done[i]
        want = ref.sort(feats[i], side, seed, storage_bf16=(storage == "bf16"))
        assert want.status == 0
        assert res.reorders == want.reorders and res.energy_fixed == want.energy, (side, storage)
        assert np.array_equal(perm.cpu().numpy(), want.perm), (side, storage)


def _drain(plas, srv, ids, count, submit_later=()):
    """Steps the server until `count` jobs finished; jobs in submit_later
    ((step, features, side, seed, storage, index) tuples) are submitted at
    their step, while the others run."""
    done = {}
    later = sorted(submit_later, key=lambda t: t[0])
    steps = 0
    while len(done) < count:
        while later and later[0][0] <= steps:
            _, f, side, seed, storage, i = later.pop(0)
            ids[srv.submit(f, side, seed, storage=storage)] = i
        srv.step()
        steps += 1
        assert steps < 100000
        for job, status, perm, res in srv.poll():
            assert status == plas.OK
            done[ids[job]] = (perm, res)
    assert srv.step() == (0, 0)
    srv.close()
    return done


def _serving_jobs(count=6, seed=71):
    """Jobs of the serving workload's distribution: sides log-uniform in
    [256, 1024], float32 and bfloat16 storage alternating."""
    sides = synthetic.batched_sides(count, 256, 1024, seed)
    return [(side, "f32" if i % 2 == 0 else "bf16", seed * 1000 + i, synthetic.SORT_SEED + i)
            for i, side in enumerate(sides)]


def _submit_in_two_waves(srv, jobs, feats):
    ids = {}
    half = len(jobs) // 2
    for i in range(half):
        side, storage, _, seed = jobs[i]
        ids[srv.submit(feats[i], side, seed, storage=storage)] = i
    later = [(2 + i, feats[i], jobs[i][0], jobs[i][3], jobs[i][1], i) for i in range(half, len(jobs))]
    return ids, later


def test_serving_config_jobs_equal_alone(env):
    """Whole sorts of jobs from the serving configuration (sides 256 .. 1024,
    float32 / bfloat16), half of them admitted while the others run: each
    equals the same sort run alone."""
    torch, plas, ctx, ref = env
    jobs = _serving_jobs()
    assert {s for _, s, _, _ in jobs} == {"f32", "bf16"} and max(j[0] for j in jobs) >= 512
    feats = [_features(torch, side, ds) for side, _, ds, _ in jobs]
    srv = plas.Server(ctx, 1 << 36, graph=True)
    ids, later = _submit_in_two_waves(srv, jobs, feats)
    done = _drain(plas, srv, ids, len(jobs), later)
    for i, (side, storage, _, seed) in enumerate(jobs):
        p1, r1 = ctx.sort(feats[i], side, seed, storage=storage)
        perm, res = done[i]
        _same(r1, p1.cpu().numpy(), res, perm.cpu().numpy())


@pytest.mark.parametrize("params", [dict(max_reorders=3), dict(start_radius=3.0, max_reorders=4)])
def test_serving_config_jobs_match_the_oracle(env, params):
    """The same serving-configuration jobs, served in a mix, checked against
    the CPU oracle over the first reorders of the coarsest level and of the
    finest levels (a sort started at radius 3)."""
    torch, plas, ctx, ref = env
    jobs = _serving_jobs()
    host = [synthetic.gaussian_attributes(side * side, ds) for side, _, ds, _ in jobs]
    feats = [torch.from_numpy(F).cuda() for F in host]
    srv = plas.Server(ctx, 1 << 36, graph=True, **params)
    ids, later = _submit_in_two_waves(srv, jobs, feats)
    done = _drain(plas, srv, ids, len(jobs), later)
    for i, (side, storage, _, seed) in enumerate(jobs):
        perm, res = done[i]
        want = ref.sort(host[i], side, seed, storage_bf16=(storage == "bf16"), **params)
        assert want.status == 0
        assert res.reorders == want.reorders == params["max_reorders"]
        assert res.energy_fixed == want.energy, (side, storage)
        assert np.array_equal(perm.cpu().numpy(), want.perm), (side, storage)
