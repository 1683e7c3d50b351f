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

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload scene|precision]
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


def cpu_baseline(F, side: int, seed: int, reorders_full: int, sample_reorders: int) -> dict:
    import oracle
    threads = oracle.set_threads(0)
    t0 = time.perf_counter()
    res = oracle.sort(F, side, seed, max_reorders=sample_reorders)
    dt = time.perf_counter() - t0
    if res.status != 0:
        raise RuntimeError(f"oracle failed: {res.status}")
    per_reorder = dt / max(res.reorders, 1)
    est = per_reorder * reorders_full
    n = side * side
    return {
        "value": n / est,
        "unit": "Gaussians/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"CPU oracle on the same {side}x{side} D={F.shape[0]} input, stopped after "
                   f"{res.reorders} reorders in {dt:.1f} s; value = N / ({per_reorder:.3f} s per reorder "
                   f"x {reorders_full} reorders of the full sort)"),
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("scene", "precision"), default="scene")
    ap.add_argument("--side", type=int, default=0, help="grid side (default: the workload's)")
    ap.add_argument("--cpu-sample-reorders", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-compare", action="store_true",
                    help="precision workload: skip the float32 sort of the same input")
    ap.add_argument("--max-reorders", type=int, default=0,
                    help="stop each sort after this many reorders (profiling runs only; "
                         "the JSON line is then not the workload's throughput)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain elementwise copy of 256 MiB (read and write 2^26 "
                         "floats) to calibrate HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the PLAS sort of one grid is a single-device "
              f"workload here (asked for --gpus {args.gpus})", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2312_13299_amd as plas
    import synthetic

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

    # Timed region: K whole sorts. The library times its blur and assignment
    # launches with HIP events on its stream (profile=True).
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
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
    }
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
        line["cpu_baseline"] = cpu_baseline(F, side, seed, res.reorders, args.cpu_sample_reorders)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
