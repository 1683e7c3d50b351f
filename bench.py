#!/usr/bin/env python3
"""Benchmark of the PLAS sort on one MI355X.

Default workload ("scene"): one plain float32 sort of a 1024 x 1024 grid
(N = 1,048,576) of D = 59 synthetic 3DGS-shaped attribute vectors,
channel-major (~247 MB), data seed 2, sort seed 0x5EED. A step is one whole
sort (ingest, every reorder of every radius level, output) with the features
already resident in device memory. Prints one JSON line.

"precision" workload: 1448 x 1448 (N = 2,096,704), D = 59, data seed 3, the
working grids stored in bfloat16; the same input is also sorted in float32
on the same GPU and both are reported.

"batch" workload: 64 independent grids, sides log-uniform in [128, 724]
(sum N = 11,833,105), D = 59 float32, sorted together by plas_sort_batch
with graph replay and a measured tuning table; a step is the whole batch.
The same grids sorted one after another by plas_sort are reported beside it.

"serve" workload: a Poisson stream (mean 20 jobs/s) of sort jobs, sides
log-uniform in [256, 1024], D = 59, float32 or bfloat16 storage (50/50),
served by a continuous-batching plas_server; latency percentiles and
throughput of a finite trace, and of a second trace at 0.8 x the measured
capacity.

"paper" workload: the paper's runtime experiment (App. C), a random
512 x 512 grid of U(0, 255) RGB values (data seed 5): throughput, reorders
and VAD beside the paper's figures, a sweep of the improvement threshold
(1/M for M = 10^2 .. 10^5), a sweep of the grid side (128 .. 2048), and the
same grid sorted with the Gaussian-like target filter (box3).

"garden" workload: the scene scale of App. C's largest scene (4.37 M
Gaussians, the Garden scene), a synthetic 2091 x 2091 grid (data seed 6)
sorted with D = 59 and with its first 14 channels (every attribute but the
higher SH coefficients), beside the paper's report that this scene sorts in
under a minute (context).

The default run also appends a compact "precision" record after its timed
region: the 1448^2 sort in bfloat16 and in float32 storage, and the float64
energy gap between the two arrangements.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload scene|precision|batch|serve|paper|garden]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD's published peak
KERNEL_SOURCE = os.path.join(ROOT, "paper_2312_13299_amd", "csrc", "plas_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash() -> str:
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed PMC measurement of
    `workload` (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter
    reads for a plain copy of known size), or None if there is none or it was
    taken on other kernel code."""
    path = os.path.join(PROFILES, f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else int(k["hbm_bytes_per_launch"])


def pmc_command(counter: str, out_dir: str, workload: str) -> str:
    """The rocprofv3 run whose per-dispatch `counter` values a traffic record
    is built from (one counter per run, the copy probe included)."""
    return (f"rocprofv3 --pmc {counter} -T --kernel-include-regex 'k_blur|k_assign|elementwise' -d {out_dir} "
            f"-o run -f csv -- python3 bench.py --workload {workload} --steps 1 --warmup 0 --no-cpu-baseline "
            f"--no-fp32-compare --no-precision --copy-probe")


def traffic_record(workload: str, fetch_dir: str, write_dir: str) -> dict:
    """HBM bytes per launch of the blur pass and the assignment from two
    rocprofv3 --pmc runs of this script (pmc_command): FETCH_SIZE and
    WRITE_SIZE in KiB per dispatch, each divided by what the same counter
    reads for the copy probe (2^26 floats read and written by one
    elementwise kernel). Blur launches queued after the end of a sort
    return at once and are left out."""
    import csv
    import glob

    def per_kernel(d, counter):
        vals = {}
        for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] != counter:
                        continue
                    k = r["Kernel_Name"]
                    key = ("blur_pass" if "k_blur" in k else "assign" if "k_assign" in k
                           else "copy" if "elementwise" in k else None)
                    if key is not None:
                        vals.setdefault(key, []).append(float(r["Counter_Value"]))
        return vals

    fv, wv = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    copy_bytes = (1 << 26) * 4
    # The probe's first kernel fills its source (writes only): take the copies.
    copies = [v for v in fv["copy"] if v > 1024]
    ff = sum(copies) / len(copies) * 1024 / copy_bytes
    wf = sum(wv["copy"]) / len(wv["copy"]) * 1024 / copy_bytes
    rec = {"workload": f"plas_sort ({workload} workload, one full sort)",
           "kernel_source_sha256": kernel_source_hash(),
           "copy_probe": {"bytes_read": copy_bytes, "bytes_written": copy_bytes,
                          "fetch_counter_factor": round(ff, 4), "write_counter_factor": round(wf, 4)},
           "commands": {"fetch": pmc_command("FETCH_SIZE", fetch_dir, workload),
                        "write": pmc_command("WRITE_SIZE", write_dir, workload),
                        "record": f"python3 bench.py --workload {workload} --write-traffic {fetch_dir} {write_dir}"},
           "kernels": {}}
    for k in ("blur_pass", "assign"):
        fs = [v for v in fv[k] if v > 1024]
        ws = [v for v in wv.get(k, []) if v > 0]
        n = min(len(fs), len(ws)) if k == "blur_pass" else len(fs)
        fm = sum(fs) / len(fs)
        wm = sum(ws) / len(ws) if ws else 0.0
        rec["kernels"][k] = {"launches": n, "fetch_kib_raw": round(fm, 1), "write_kib_raw": round(wm, 1),
                             "hbm_bytes_per_launch": int(fm * 1024 / ff + wm * 1024 / wf)}
    return rec


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_roofline(res, n: int, d: int, elem: int) -> dict:
    """Achieved algorithmic bandwidth of the blur pass and of the assignment
    kernel, from HIP-event times of the launches of the profiled sorts.
    elem: bytes per stored channel value (4 float32, 2 bfloat16)."""
    blur_bytes = n * 2 * d * elem                      # read + write one grid per pass
    moved = sum(t["moved"] for t in res.trace) / max(res.reorders, 1)
    assign_bytes = n * 2 * d * elem + moved * (d * elem + 2 * 4)  # read grid+target; write moved cells + perm
    out = {}
    if res.blur_launches:
        avg = res.blur_ms / res.blur_launches
        out["blur_pass"] = dict(avg_ms=avg, bytes=blur_bytes, gbs=blur_bytes / (avg * 1e-3) / 1e9)
    if res.assign_launches:
        avg = res.assign_ms / res.assign_launches
        out["assign"] = dict(avg_ms=avg, bytes=assign_bytes, gbs=assign_bytes / (avg * 1e-3) / 1e9,
                             moved_per_reorder=moved)
    return out


def cpu_baseline(F, side: int, seed: int, trace, sample_reorders: int, bands: int = 4) -> dict:
    """The oracle's throughput on the whole sort, estimated from short runs.

    trace: the full sort's levels as (phi, reorders) pairs. The schedule is
    cut into `bands` runs of consecutive levels; one oracle sort per band
    starts at the radius of the band's middle level (start_radius) and stops
    after sample_reorders / bands reorders. Each band's reorders are priced
    at its sample's time per reorder."""
    import oracle
    levels = [(float(phi), int(k)) for phi, k in trace]
    full = sum(k for _, k in levels)
    bands = max(1, min(bands, len(levels)))
    per_band = max(1, sample_reorders // bands)
    threads = oracle.set_threads(0)
    est = 0.0
    parts = []
    t_all = 0.0
    ran = 0
    for b in range(bands):
        lo, hi = b * len(levels) // bands, (b + 1) * len(levels) // bands
        phi = levels[(lo + hi - 1) // 2][0]
        t0 = time.perf_counter()
        res = oracle.sort(F, side, seed, start_radius=phi, max_reorders=per_band)
        dt = time.perf_counter() - t0
        if res.status != 0:
            raise RuntimeError(f"oracle failed: {res.status}")
        per = dt / max(res.reorders, 1)
        band_reorders = sum(k for _, k in levels[lo:hi])
        est += per * band_reorders
        t_all += dt
        ran += res.reorders
        parts.append(f"phi {phi:.1f}: {per:.3f} s x {band_reorders}")
    n = side * side
    # The same oracle on one thread, on a shorter sample from the start of
    # the sort (the result does not depend on the thread count).
    one_reorders = max(1, sample_reorders // 12)
    oracle.set_threads(1)
    t1 = time.perf_counter()
    one = oracle.sort(F, side, seed, max_reorders=one_reorders)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    first = oracle.sort(F, side, seed, max_reorders=one_reorders)
    if one.status != 0 or not (one.perm == first.perm).all():
        raise RuntimeError("oracle result depends on the thread count")
    t2 = time.perf_counter()
    oracle.sort(F, side, seed, max_reorders=one_reorders)
    per_all_cores = (time.perf_counter() - t2) / max(one_reorders, 1)
    return {
        "value": n / est,
        "unit": "Gaussians/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"CPU oracle on the same {side}x{side} D={F.shape[0]} input: {ran} reorders in "
                   f"{t_all:.1f} s, {bands} runs started at levels spread over the schedule, each pricing "
                   f"its band of levels ({'; '.join(parts)}); value = N / {est:.0f} s for the "
                   f"{full} reorders of the full sort"),
        "one_thread": {"seconds_per_reorder": round(dt1 / max(one.reorders, 1), 4), "sample_reorders": one.reorders,
                       "speedup_of_all_cores": round(dt1 / max(one.reorders, 1) / per_all_cores, 2)},
    }


def energy_f64(torch, f, perm, side: int, r: int = 1) -> float:
    """Mean over cells of the squared distance of the arranged features to
    their clipped (2r+1)^2 window mean, in float64 on the device (direct
    window sums, no quantisation): the measure the bfloat16 storage gate
    compares. f: [d][n] float32 features, perm: int32[n] (gather form)."""
    G = f.double()[:, perm.long()].reshape(f.shape[0], side, side)

    def box(x, axis):
        c = torch.cumsum(x, dim=axis)
        z = torch.zeros_like(x.narrow(axis, 0, 1))
        c = torch.cat([z, c], dim=axis)
        idx = torch.arange(side, device=x.device)
        hi = torch.clamp(idx + r, max=side - 1) + 1
        lo = torch.clamp(idx - r, min=0)
        return c.index_select(axis, hi) - c.index_select(axis, lo), (hi - lo).double()

    sy, cy = box(G, 1)
    s2, cx = box(sy, 2)
    T = s2 / (cy.view(1, side, 1) * cx.view(1, 1, side))
    return float(((G - T) ** 2).sum(dim=0).mean().item())


def precision_record(torch, plas, synthetic, ctx) -> dict:
    """The bfloat16 storage gate in a few seconds: the 1448^2 D=59 sort in
    bfloat16 and in float32 storage on the same input, and the float64
    energy of both arrangements at r = 1 (on the original features)."""
    side = 1448
    n = side * side
    f = torch.from_numpy(synthetic.gaussian_attributes(n, synthetic.DATA_SEED_PRECISION)).cuda()
    out = {"workload": f"plas_sort_{side}x{side}_d59", "data_seed": synthetic.DATA_SEED_PRECISION}
    for storage in ("bf16", "f32"):
        ctx.sort(f, side, synthetic.SORT_SEED, storage=storage, max_reorders=1)  # sizes the workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        perm, res = ctx.sort(f, side, synthetic.SORT_SEED, storage=storage)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[storage] = {"ms": round(dt * 1e3, 1), "gaussians_per_s": round(n / dt, 1),
                        "reorders": res.reorders, "energy_f64_r1": round(energy_f64(torch, f, perm, side), 6)}
    out["bf16_speedup"] = round(out["f32"]["ms"] / out["bf16"]["ms"], 3)
    out["energy_gap_pct"] = round(100 * (out["bf16"]["energy_f64_r1"] / out["f32"]["energy_f64_r1"] - 1), 4)
    out["gate_pct"] = 0.5
    return out


def percentile(values, q: float) -> float:
    """Nearest-rank percentile."""
    import math
    v = sorted(values)
    return v[max(0, min(len(v) - 1, math.ceil(q / 100.0 * len(v)) - 1))]


def run_batch_workload(args, torch, plas, synthetic) -> int:
    work = synthetic.batch_workload()
    sides = [w[0] for w in work]
    seeds = [w[2] for w in work]
    t0 = time.perf_counter()
    feats = [torch.from_numpy(synthetic.gaussian_attributes(s * s, ds)).cuda() for s, ds, _ in work]
    n_total = sum(s * s for s in sides)
    d = feats[0].shape[0]
    log(f"batch inputs: {len(work)} grids, sum N {n_total}, {time.perf_counter() - t0:.1f} s")
    ctx = plas.Context(0)
    tune = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tune = ctx.autotune_batch(feats, sides=sides, seeds=seeds, graph=True)
        log(f"autotune: {len(tune)} buckets in {time.perf_counter() - t0:.1f} s: {tune}")
    for i in range(args.warmup):
        ctx.sort_batch(feats, sides=sides, seeds=seeds, graph=True, tune=tune, max_reorders=16)
    # Per-kernel times: a profiled batch of the first 200 reorders (every
    # sort still runs then), direct launches timed with HIP events.
    prof_reorders = 200
    _, _, bp = ctx.sort_batch(feats, sides=sides, seeds=seeds, tune=tune, profile=True,
                              max_reorders=prof_reorders)
    torch.cuda.synchronize()
    results = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        perms, results, b = ctx.sort_batch(feats, sides=sides, seeds=seeds, graph=True, tune=tune)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = n_total * args.steps / elapsed
    log(f"batch: {elapsed / args.steps:.2f} s per batch, {b.graph_builds} graphs, {b.launches} launches")
    # The same batch with the default launch shapes (no tuning table), to
    # measure what the autotuner adds.
    default_shapes = None
    if tune is not None:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        perms_d, results_d, _ = ctx.sort_batch(feats, sides=sides, seeds=seeds, graph=True)
        torch.cuda.synchronize()
        t_default = time.perf_counter() - t0
        same_d = sum(int(torch.equal(a, c) and ra.reorders == rc.reorders)
                     for a, c, ra, rc in zip(perms, perms_d, results, results_d))
        default_shapes = {"value": round(n_total / t_default, 1), "seconds": round(t_default, 3),
                          "autotune_speedup": round(t_default / (elapsed / args.steps), 3),
                          "identical_to_tuned": f"{same_d}/{len(work)}"}
        log(f"default launch shapes: {default_shapes}")
        del perms_d, results_d
    # The same grids one after another through plas_sort.
    t0 = time.perf_counter()
    same = 0
    for f, s, seed, perm, res in zip(feats, sides, seeds, perms, results):
        p1, r1 = ctx.sort(f, s, seed)
        same += int(torch.equal(p1, perm) and r1.reorders == res.reorders and r1.energy_fixed == res.energy_fixed)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    blur_bytes = n_total * 2 * d * 4
    blur_avg = bp.blur_ms / (2 * prof_reorders)
    assign_avg = bp.assign_ms / prof_reorders
    line = {
        "metric": "Gaussians sorted/s, 64-grid batch D=59",
        "value": round(value, 1), "unit": "Gaussians/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plas_sort_batch_64_grids_128_724_d59_f32", "grids": len(work),
                   "sum_n": n_total, "d": d, "side_min": min(sides), "side_max": max(sides),
                   "graph": True, "tune": tune,
                   "reorders_min": min(r.reorders for r in results),
                   "reorders_max": max(r.reorders for r in results)},
        "vs_single_sorts": {"value": round(n_total / t_plain, 1), "seconds": round(t_plain, 3),
                            "speedup": round(t_plain / (elapsed / args.steps), 3),
                            "identical": f"{same}/{len(work)}"},
        "default_launch_shapes": default_shapes,
        "roofline": {
            "bound": "hbm", "kernel": "blur_pass (batched, all 64 grids)",
            "achieved": round(blur_bytes / (blur_avg * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(blur_bytes / (blur_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
            "per_launch_bytes": blur_bytes, "avg_launch_ms": round(blur_avg, 5),
            "sample": f"first {prof_reorders} reorders of the batch, direct launches timed with HIP events",
            "assign_avg_ms": round(assign_avg, 5),
        },
    }
    print(json.dumps(line), flush=True)
    return 0


def run_serve_workload(args, torch, plas, synthetic) -> int:
    import numpy as np
    ctx = plas.Context(0)
    d = 59

    def make_trace(count, rate, seed):
        rng = np.random.Generator(np.random.PCG64(seed))
        gaps = rng.exponential(1.0 / rate, size=count)
        arrivals = np.cumsum(gaps) - gaps[0]
        sides = synthetic.batched_sides(count, 256, 1024, seed + 1)
        storages = ["f32" if v < 0.5 else "bf16" for v in rng.uniform(size=count)]
        feats = [torch.from_numpy(synthetic.gaussian_attributes(s * s, seed * 1000 + i)).cuda()
                 for i, s in enumerate(sides)]
        return [dict(arrival=float(a), side=s, storage=st, features=f, seed=synthetic.SORT_SEED + i)
                for i, (a, s, st, f) in enumerate(zip(arrivals, sides, storages, feats))]

    def serve(trace, budget, check):
        """Serves the trace in real time; returns latency and throughput
        statistics, and checks the served results of the jobs at positions
        `check` (after the trace) against the same sorts run alone."""
        srv = plas.Server(ctx, budget, graph=True)
        pending = sorted(trace, key=lambda j: j["arrival"])
        ids = {}
        finish = {}
        kept = {}
        max_running = 0
        t0 = time.perf_counter()
        nxt = 0
        while len(finish) < len(trace):
            now = time.perf_counter() - t0
            while nxt < len(pending) and pending[nxt]["arrival"] <= now:
                j = pending[nxt]
                ids[srv.submit(j["features"], j["side"], j["seed"], storage=j["storage"])] = nxt
                nxt += 1
            running, waiting = srv.step()
            max_running = max(max_running, running)
            for job, status, perm, res in srv.poll():
                if status != plas.OK:
                    raise RuntimeError(f"job {job} failed with status {status}")
                finish[ids[job]] = time.perf_counter() - t0
                if ids[job] in check:
                    kept[ids[job]] = (perm, res)
            if running == 0 and waiting == 0 and nxt < len(pending):
                time.sleep(max(0.0, pending[nxt]["arrival"] - (time.perf_counter() - t0)))
        srv.close()
        lat = [finish[i] - pending[i]["arrival"] for i in range(len(pending))]
        n = sum(j["side"] ** 2 for j in pending)
        makespan = max(finish.values()) - pending[0]["arrival"]
        same = 0
        for i, (perm, res) in kept.items():
            j = pending[i]
            p1, r1 = ctx.sort(j["features"], j["side"], j["seed"], storage=j["storage"])
            same += int(torch.equal(p1, perm) and r1.reorders == res.reorders and
                        r1.energy_fixed == res.energy_fixed)
        return dict(jobs=len(pending), p50_ms=round(percentile(lat, 50) * 1e3, 1),
                    p90_ms=round(percentile(lat, 90) * 1e3, 1), p99_ms=round(percentile(lat, 99) * 1e3, 1),
                    max_ms=round(max(lat) * 1e3, 1),
                    gaussians_per_s=round(n / makespan, 1), makespan_s=round(makespan, 3),
                    offered_jobs_per_s=round(len(pending) / max(pending[-1]["arrival"], 1e-9), 2),
                    max_running=max_running, sum_n=n,
                    identical_to_alone=f"{same}/{len(kept)}")

    budget = 64 << 30
    jobs = args.jobs or 100
    # Served results checked against the same sorts run alone: every tenth
    # job of each trace.
    check = set(range(0, jobs, 10))
    t0 = time.perf_counter()
    trace = make_trace(jobs, 20.0, 11)
    log(f"trace 1: {jobs} jobs generated in {time.perf_counter() - t0:.1f} s")
    # Warm-up: one small served job.
    warm = make_trace(1, 20.0, 99)
    serve(warm, budget, set())
    r1 = serve(trace, budget, check)
    log(f"trace 1 (20 jobs/s): {r1}")
    mean_n = np.mean([j["side"] ** 2 for j in trace])
    rate2 = 0.8 * r1["gaussians_per_s"] / mean_n
    del trace
    torch.cuda.empty_cache()
    trace2 = make_trace(jobs, rate2, 12)
    r2 = serve(trace2, budget, check)
    log(f"trace 2 ({rate2:.2f} jobs/s): {r2}")
    line = {
        "metric": "served p50/p99 latency and Gaussians/s, Poisson 20 jobs/s, sides 256..1024, D=59",
        "value": r1["gaussians_per_s"], "unit": "Gaussians/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(r1["makespan_s"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 or bf16 storage (50/50), f32 arithmetic", "data": "synthetic",
        "config": {"workload": "plas_server_poisson_20_sides_256_1024_d59", "jobs": jobs,
                   "memory_budget_bytes": budget, "graph": True},
        "p50_ms": r1["p50_ms"], "p99_ms": r1["p99_ms"],
        "note": ("percentiles are nearest-rank over the trace's jobs; the 20 jobs/s stream offers "
                 "more work than one GPU sorts, so its latencies grow along the trace, and the "
                 "second trace runs at 0.8 x the capacity measured on the first"),
        "trace_20_per_s": r1,
        "trace_0p8_capacity": dict(r2, rate_jobs_per_s=round(rate2, 3)),
    }
    print(json.dumps(line), flush=True)
    return 0


# The paper's runtime experiment (App. C): PLAS on an RTX 4090 sorts a
# random 512 x 512 x 3 grid in 5.7 s with 8015 reorders, to a VAD of 4.02
# (shuffled: 3607.45), with a Gaussian filter and its own random numbers.
PAPER_RGB = {"seconds": 5.7, "reorders": 8015, "vad_sorted": 4.02, "vad_shuffled": 3607.45,
             "gaussians_per_s": 512 * 512 / 5.7, "hardware": "NVIDIA RTX 4090"}


def run_paper_workload(args, torch, plas, synthetic) -> int:
    ctx = plas.Context(0)

    def timed_sort(f, side, reps, **kw):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            perm, res = ctx.sort(f, side, synthetic.SORT_SEED, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return perm, res, best

    side = 512
    f = torch.from_numpy(synthetic.random_rgb_grid(side, synthetic.DATA_SEED_RGB)).cuda()
    for _ in range(args.warmup):
        ctx.sort(f, side, synthetic.SORT_SEED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        perm, res = ctx.sort(f, side, synthetic.SORT_SEED)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = side * side * args.steps / elapsed
    vad_sorted, vad_start = ctx.vad(f, perm, side), ctx.vad(f, None, side)
    sweep_m = []
    for m in (100, 1000, 10000, 100000):
        p, r, dt = timed_sort(f, side, 1, inv_threshold=m)
        sweep_m.append(dict(threshold=1.0 / m, reorders=r.reorders, seconds=round(dt, 4),
                            vad=round(ctx.vad(f, p, side), 4)))
        log(f"threshold 1/{m}: {sweep_m[-1]}")
    sweep_side = []
    for sd in (128, 256, 512, 1024, 2048):
        g = torch.from_numpy(synthetic.random_rgb_grid(sd, synthetic.DATA_SEED_RGB)).cuda()
        p, r, dt = timed_sort(g, sd, 1)
        sweep_side.append(dict(side=sd, n=sd * sd, reorders=r.reorders, levels=r.levels, seconds=round(dt, 4),
                               gaussians_per_s=round(sd * sd / dt, 1), vad=round(ctx.vad(g, p, sd), 4)))
        log(f"side {sd}: {sweep_side[-1]}")
        del g
    # The Gaussian-like target filter (three box passes per axis) on the same
    # grid: the paper's filter family, three times the blur work.
    p3, r3, dt3 = timed_sort(f, side, max(1, args.steps), filter="box3")
    box3 = dict(filter="box3", reorders=r3.reorders, levels=r3.levels, seconds=round(dt3, 4),
                gaussians_per_s=round(side * side / dt3, 1), vad=round(ctx.vad(f, p3, side), 4))
    log(f"box3 filter: {box3}")
    line = {
        "metric": "Gaussians sorted/s, random 512^2 RGB grid (App. C runtime experiment)",
        "value": round(value, 1), "unit": "Gaussians/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": round(value / PAPER_RGB["gaussians_per_s"], 3),
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plas_sort_512x512_rgb_u0_255", "side": side, "d": 3,
                   "data_seed": synthetic.DATA_SEED_RGB, "sort_seed": synthetic.SORT_SEED},
        "reorders": res.reorders, "levels": res.levels,
        "vad_sorted": round(vad_sorted, 4), "vad_start": round(vad_start, 2),
        "paper": dict(PAPER_RGB, note="context: another GPU, a Gaussian filter and another RNG"),
        "threshold_sweep": sweep_m, "side_sweep": sweep_side, "filter_box3": box3,
    }
    print(json.dumps(line), flush=True)
    return 0


def run_garden_workload(args, torch, plas, synthetic) -> int:
    """Scene scale: the sort of a 2091 x 2091 grid (4,372,281 Gaussians, the
    size of App. C's largest scene), with D = 59 and with 14 channels."""
    ctx = plas.Context(0)
    side = args.side or synthetic.GARDEN_SIDE
    n = side * side
    runs = {}
    for label, make in (("d59", synthetic.gaussian_attributes), ("d14", synthetic.scene_attributes_14)):
        f = torch.from_numpy(make(n, synthetic.DATA_SEED_GARDEN)).cuda()
        for _ in range(args.warmup):
            ctx.sort(f, side, synthetic.SORT_SEED, max_reorders=8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            perm, res = ctx.sort(f, side, synthetic.SORT_SEED)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        runs[label] = {"d": int(f.shape[0]), "seconds": round(dt, 3), "gaussians_per_s": round(n / dt, 1),
                       "reorders": res.reorders, "levels": res.levels, "energy_mean": res.energy}
        log(f"{side}^2 {label}: {runs[label]}")
        del f, perm
        torch.cuda.empty_cache()
    line = {
        "metric": f"Gaussians sorted/s at {side}^2 D=59 (scene scale)",
        "value": runs["d59"]["gaussians_per_s"], "unit": "Gaussians/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(runs["d59"]["seconds"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"plas_sort_{side}x{side}_d59_and_d14", "side": side, "n": n,
                   "data_seed": synthetic.DATA_SEED_GARDEN, "sort_seed": synthetic.SORT_SEED},
        "runs": runs,
        "paper": {"scene": "Garden", "gaussians": 4_370_000, "time": "under a minute (the paper's report, paraphrased)",
                  "note": "context: another GPU, the paper's filter and channel weights"},
    }
    print(json.dumps(line), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("scene", "precision", "batch", "serve", "paper", "garden"),
                    default="scene")
    ap.add_argument("--jobs", type=int, default=0, help="serve: jobs per trace (default 100)")
    ap.add_argument("--no-autotune", action="store_true", help="batch: use the default launch shapes")
    ap.add_argument("--side", type=int, default=0, help="grid side (default: the workload's)")
    ap.add_argument("--cpu-sample-reorders", type=int, default=120,
                    help="reorders of the CPU oracle sample (about 10-15 s on 16 host cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-compare", action="store_true",
                    help="precision workload: skip the float32 sort of the same input")
    ap.add_argument("--max-reorders", type=int, default=0,
                    help="stop each sort after this many reorders (profiling runs only; "
                         "the JSON line is then not the workload's throughput)")
    ap.add_argument("--no-precision", action="store_true",
                    help="scene workload: skip the appended 1448^2 bfloat16 / float32 record")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain elementwise copy of 256 MiB (read and write 2^26 "
                         "floats) to calibrate HBM byte counters")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="scene / precision workload: write profiles/hbm_traffic_<name>.json from the "
                         "output folders of the two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) and exit")
    args = ap.parse_args()
    if args.write_traffic:
        if args.workload not in ("scene", "precision"):
            print("--write-traffic applies to the scene and precision workloads", file=sys.stderr)
            return 2
        name = "sort_1448_d59_bf16" if args.workload == "precision" else "sort_1024_d59"
        rec = traffic_record(args.workload, *args.write_traffic)
        with open(os.path.join(PROFILES, f"hbm_traffic_{name}.json"), "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec, indent=1))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the PLAS sort of one grid is a single-device "
              f"workload here (asked for --gpus {args.gpus})", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2312_13299_amd as plas
    import synthetic

    if args.workload == "batch":
        return run_batch_workload(args, torch, plas, synthetic)
    if args.workload == "serve":
        return run_serve_workload(args, torch, plas, synthetic)
    if args.workload == "paper":
        return run_paper_workload(args, torch, plas, synthetic)
    if args.workload == "garden":
        return run_garden_workload(args, torch, plas, synthetic)
    precision = args.workload == "precision"
    side = args.side or (1448 if precision else 1024)
    data_seed = synthetic.DATA_SEED_PRECISION if precision else synthetic.DATA_SEED_SCENE
    storage = "bf16" if precision else "f32"
    n = side * side
    seed = synthetic.SORT_SEED
    F = synthetic.gaussian_attributes(n, data_seed)
    d = F.shape[0]
    workload = f"sort_{side}_d{d}" + ("_bf16" if precision else "")
    f_dev = torch.from_numpy(F).cuda()
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx = plas.Context(0)
    torch.cuda.synchronize()

    if args.copy_probe:
        src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy probe: 3 launches, each reads {src.numel() * 4} B and writes {dst.numel() * 4} B")
        del src, dst
    for i in range(args.warmup):
        _, res = ctx.sort(f_dev, side, seed, out=perm, max_reorders=args.max_reorders, storage=storage)
        log(f"warmup {i}: {res.reorders} reorders, {res.levels} levels, {res.total_ms:.1f} ms")
    torch.cuda.synchronize()

    # Timed region: K whole sorts. The library times the blur and assignment
    # launches of every 32nd reorder with HIP events on its stream
    # (profile=True).
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, res = ctx.sort(f_dev, side, seed, out=perm, profile=True, max_reorders=args.max_reorders,
                          storage=storage)
        results.append(res)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for i, res in enumerate(results):
        log(f"step {i}: {res.reorders} reorders, {res.total_ms:.1f} ms, blur {res.blur_ms:.1f} ms, "
            f"assign {res.assign_ms:.1f} ms")
    res = results[-1]
    # Sum the event times over all timed steps.
    agg = plas.SortResult(reorders=sum(r.reorders for r in results), levels=res.levels,
                          energy_fixed=res.energy_fixed, scale_shift=res.scale_shift,
                          energy=res.energy, trace=[t for r in results for t in r.trace],
                          blur_ms=sum(r.blur_ms for r in results),
                          blur_launches=sum(r.blur_launches for r in results),
                          assign_ms=sum(r.assign_ms for r in results),
                          assign_launches=sum(r.assign_launches for r in results))
    kern = kernel_roofline(agg, n, d, 2 if precision else 4)
    dominant = max(kern, key=lambda k: kern[k]["avg_ms"] * (2 if k == "blur_pass" else 1))
    roof = {
        "bound": "hbm",
        "kernel": dominant,
        "achieved": round(kern[dominant]["gbs"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(kern[dominant]["gbs"] / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(dominant, workload),
        "per_launch_bytes": int(kern[dominant]["bytes"]),
        "avg_launch_ms": round(kern[dominant]["avg_ms"], 5),
        "timed_launches": int(agg.blur_launches if dominant == "blur_pass" else agg.assign_launches),
        "sample": "every 32nd reorder of the timed sorts, HIP events on the library's stream",
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
    }
    # Practical streaming ceiling, outside the timed region: a device copy of
    # one working grid's bytes (read + write), timed with HIP events.
    grid_bytes = n * 64 * (2 if precision else 4)
    src = torch.empty(grid_bytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * grid_bytes * 10 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src, dst
    roof["copy_gbs"] = round(copy_gbs, 1)
    roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
    # The whole sort's algorithmic bytes per reorder (two blur passes, the
    # assignment's reads and its moved-cell writes) over the wall time.
    e = 2 if precision else 4
    moved = sum(t["moved"] for t in res.trace) / max(res.reorders, 1)
    per_reorder = 3 * n * 2 * d * e + moved * (d * e + 8)
    path_gbs = per_reorder * res.reorders * args.steps / elapsed / 1e9
    roof["whole_sort"] = {"bytes_per_reorder": int(per_reorder), "achieved": round(path_gbs, 1),
                          "frac": round(path_gbs / HBM_PEAK_GBS, 4)}
    ms_per_step = elapsed / args.steps * 1e3
    value = n * args.steps / elapsed
    line = {
        "metric": (f"Gaussians sorted/s at {side}^2 D={d}, bfloat16 storage" if precision
                   else f"Gaussians sorted/s at {side}^2 D={d}"),
        "value": round(value, 1),
        "unit": "Gaussians/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 storage, f32 arithmetic" if precision else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"plas_sort_{side}x{side}_d{d}_{storage}",
            "profile_name": workload,
            "side": side, "n": n, "d": d, "layout": "channel-major", "storage": storage,
            "data_seed": data_seed, "sort_seed": seed,
            "reorders": res.reorders, "levels": res.levels,
            "energy_mean": res.energy,
        },
        # Per level: radius r, reorders, and the mean squared distance to the
        # target after the level's last reorder (energy * 2^-s / N).
        "level_energy": [[t["r"], t["reorders"], round(t["energy"] * 2.0 ** -res.scale_shift / n, 6)]
                         for t in res.trace],
        "roofline": roof,
    }
    if precision and not args.no_fp32_compare:
        # The plain float32 sort of the same input on the same GPU, and the
        # energy of both arrangements (library grid-energy query at r = 1,
        # float32 storage, on the original features).
        perm16 = perm.clone()
        ctx.sort(f_dev, side, seed, max_reorders=1)  # sizes the float32 workspace
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        perm32, res32 = ctx.sort(f_dev, side, seed, max_reorders=args.max_reorders)
        torch.cuda.synchronize()
        t32 = time.perf_counter() - t0
        _, _, e16 = ctx.grid_energy(f_dev, perm16, side, 1)
        _, _, e32 = ctx.grid_energy(f_dev, perm32, side, 1)
        line["vs_fp32_sort"] = {
            "fp32_value": round(n / t32, 1),
            "fp32_ms_per_step": round(t32 * 1e3, 3),
            "fp32_reorders": res32.reorders,
            "speedup": round(value * t32 / n, 3),
            "energy_r1_bf16": e16, "energy_r1_fp32": e32,
            "energy_gap_pct": round(100 * (e16 / e32 - 1), 4),
        }
    if args.max_reorders:
        line["config"]["max_reorders"] = args.max_reorders
        line["note"] = "truncated profiling run, not the workload's throughput"
    if not args.no_cpu_baseline and not args.max_reorders and not precision:
        line["cpu_baseline"] = cpu_baseline(F, side, seed, [(t["phi"], t["reorders"]) for t in res.trace],
                                           args.cpu_sample_reorders)
    if not precision and not args.no_precision and not args.max_reorders and not args.side:
        del f_dev, perm
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        line["precision"] = precision_record(torch, plas, synthetic, ctx)
        log(f"precision record in {time.perf_counter() - t0:.1f} s: {line['precision']}")
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
