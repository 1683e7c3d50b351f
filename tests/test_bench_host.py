"""Host logic of bench.py, on the CPU: the one-GPU refusal, the algorithmic
byte counts behind the roofline, the committed traffic records, and the
nearest-rank percentile used for serving latencies."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


class _Res:
    def __init__(self, reorders, moved_per_level, blur_ms, blur_launches, assign_ms, assign_launches):
        self.reorders = reorders
        self.trace = [{"moved": m} for m in moved_per_level]
        self.blur_ms, self.blur_launches = blur_ms, blur_launches
        self.assign_ms, self.assign_launches = assign_ms, assign_launches


def test_kernel_roofline_bytes_and_rates():
    n, d = 1024 * 1024, 59
    # 100 reorders, 2,000,000 cells moved in all; 200 blur launches of 0.1 ms,
    # 100 assignment launches of 0.2 ms.
    res = _Res(100, [1_500_000, 500_000], 20.0, 200, 20.0, 100)
    k = bench.kernel_roofline(res, n, d, 4)
    blur_bytes = n * 2 * d * 4  # read and write one grid, 59 float32 channels
    assert k["blur_pass"]["bytes"] == blur_bytes == 494_927_872
    assert k["blur_pass"]["avg_ms"] == pytest.approx(0.1)
    assert k["blur_pass"]["gbs"] == pytest.approx(blur_bytes / 1e-4 / 1e9)
    moved = 2_000_000 / 100
    assert k["assign"]["moved_per_reorder"] == pytest.approx(moved)
    assert k["assign"]["bytes"] == pytest.approx(n * 2 * d * 4 + moved * (d * 4 + 8))
    assert k["assign"]["avg_ms"] == pytest.approx(0.2)
    # bfloat16 storage halves the bytes per channel.
    assert bench.kernel_roofline(res, n, d, 2)["blur_pass"]["bytes"] == blur_bytes // 2
    # No timed launches, no entry.
    assert bench.kernel_roofline(_Res(0, [], 0.0, 0, 0.0, 0), n, d, 4) == {}


def test_committed_traffic_records():
    for workload in ("sort_1024_d59", "sort_1448_d59_bf16"):
        path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
        rec = json.load(open(path))
        if rec["kernel_source_sha256"] != bench.kernel_source_hash():
            # Counters taken on other kernel code are not used: bench.py
            # then reports traffic as null.
            for kernel in ("blur_pass", "assign"):
                assert bench.measured_traffic(kernel, workload) is None
            continue
        for kernel in ("blur_pass", "assign"):
            v = bench.measured_traffic(kernel, workload)
            assert v == rec["kernels"][kernel]["hbm_bytes_per_launch"]
            # Both kernels read a whole grid (268 MB in either storage) and
            # the blur writes one: well above 256 MB per launch.
            assert v > 256 * 1024 * 1024
    assert bench.measured_traffic("blur_pass", "no_such_workload") is None
    assert bench.measured_traffic("no_such_kernel", "sort_1024_d59") is None


def test_percentile_nearest_rank():
    v = [5.0, 1.0, 4.0, 2.0, 3.0]
    assert bench.percentile(v, 50) == 3.0
    assert bench.percentile(v, 99) == 5.0
    assert bench.percentile(v, 0) == 1.0
    assert bench.percentile(list(range(1, 101)), 99) == 99
    assert bench.percentile([7.0], 50) == 7.0


def test_cpu_baseline_on_a_small_grid():
    import synthetic
    F = synthetic.gaussian_attributes(64 * 64, 1)
    trace = [(phi, 6) for phi in (31.0, 20.0, 9.0, 4.0, 2.0, 1.0)]
    b = bench.cpu_baseline(F, 64, 0x5EED, trace, 24)
    assert b["kind"] == "oracle" and b["unit"] == "Gaussians/s" and b["cores"] >= 1
    assert b["value"] > 0 and "24 reorders in" in b["sample"] and "for the 36 reorders" in b["sample"]
    # Bands of levels 0-0, 1-2, 3-3, 4-5 start at their middle levels.
    for phi in ("31.0", "20.0", "4.0", "2.0"):
        assert f"phi {phi}:" in b["sample"]
    assert b["one_thread"]["sample_reorders"] == 2 and b["one_thread"]["seconds_per_reorder"] > 0


@pytest.mark.parametrize("side,d,r", [(2, 3, 1), (7, 59, 1), (16, 14, 2), (33, 5, 1)])
def test_energy_f64_matches_the_oracle_definition(ref, side, d, r):
    """bench.energy_f64 (prefix sums in float64 on torch) against the
    oracle's float64 energy (direct window sums) of the same arrangement."""
    import numpy as np
    import torch
    import synthetic
    n = side * side
    F = synthetic.random_features(n, d, 3 + side, "cn", -2.0, 2.0)
    perm = synthetic.random_permutation(n, side)
    got = bench.energy_f64(torch, torch.from_numpy(F), torch.from_numpy(perm), side, r)
    want = ref.grid_energy_f64(F, perm, side, r)
    assert got == pytest.approx(want, rel=1e-12, abs=1e-15)


def _counter_csv(path, rows):
    import csv
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_record_scales_by_the_copy_probe(tmp_path):
    """The traffic record divides each counter by what it reads for the copy
    probe: a FETCH_SIZE that reports half the copy's 256 MiB and a WRITE_SIZE
    that reports all of it give factors 0.5 and 1, and a blur pass that
    fetches 100 MiB and writes 50 MiB by those counters moves 250 MiB."""
    mib = 1024  # KiB
    fetch = tmp_path / "f"
    write = tmp_path / "w"
    copy = "void at::native::elementwise_kernel<...>"
    _counter_csv(str(fetch), [
        (copy, "FETCH_SIZE", 0.5),                      # the probe's fill: ignored
        (copy, "FETCH_SIZE", 128 * mib), (copy, "FETCH_SIZE", 128 * mib),
        ("k_blur_staged<...>", "FETCH_SIZE", 100 * mib), ("k_blur_staged<...>", "FETCH_SIZE", 100 * mib),
        ("k_blur_staged<...>", "FETCH_SIZE", 0.25),     # a pass queued after the end of the sort
        ("k_assign<...>", "FETCH_SIZE", 200 * mib),
    ])
    _counter_csv(str(write), [
        (copy, "WRITE_SIZE", 256 * mib), (copy, "WRITE_SIZE", 256 * mib), (copy, "WRITE_SIZE", 256 * mib),
        ("k_blur_staged<...>", "WRITE_SIZE", 50 * mib), ("k_blur_staged<...>", "WRITE_SIZE", 50 * mib),
        ("k_blur_staged<...>", "WRITE_SIZE", 0.0),
        ("k_assign<...>", "WRITE_SIZE", 4 * mib),
    ])
    rec = bench.traffic_record("scene", str(fetch), str(write))
    assert rec["copy_probe"]["fetch_counter_factor"] == 0.5 and rec["copy_probe"]["write_counter_factor"] == 1.0
    blur = rec["kernels"]["blur_pass"]
    assert blur["launches"] == 2 and blur["hbm_bytes_per_launch"] == 250 << 20
    assert rec["kernels"]["assign"]["hbm_bytes_per_launch"] == (400 + 4) << 20
    assert rec["kernel_source_sha256"] == bench.kernel_source_hash()
    assert "--workload scene" in rec["commands"]["fetch"] and "--pmc FETCH_SIZE" in rec["commands"]["fetch"]
