"""Write the stored expected results of full oracle sorts.

The oracle needs tens of minutes for a full 1024 x 1024 sort, too long for
a test run, so its result is stored here once: the reorder count, the
per-level trace, the final integer energy and a SHA-256 of the permutation.
This script calls only the oracle and the seeded input generators.

Usage: python tests/golden/make_golden.py [--threads T] [name ...]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synthetic  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = {
    # 3DGS-shaped attributes, D = 59, channel-major, scene scale.
    "sort_1024_d59": dict(side=1024, data_seed=synthetic.DATA_SEED_SCENE, sort_seed=synthetic.SORT_SEED),
    # A mid-size case that the GPU test can also compare reorder by reorder.
    "sort_256_d59": dict(side=256, data_seed=11, sort_seed=synthetic.SORT_SEED),
    # The runtime experiment of App. C: a random 512 x 512 grid of U(0, 255)
    # RGB values; its VAD is stored as well.
    "sort_512_rgb": dict(side=512, data_seed=synthetic.DATA_SEED_RGB, sort_seed=synthetic.SORT_SEED, rgb=True),
    # The same grid with the Gaussian-like target filter (three box passes
    # per axis).
    "sort_512_rgb_box3": dict(side=512, data_seed=synthetic.DATA_SEED_RGB, sort_seed=synthetic.SORT_SEED, rgb=True,
                              filter="box3"),
    # A whole sort with the working grids in bfloat16 (the precision
    # workload's storage at a size the oracle finishes in about 20 minutes).
    "sort_512_d59_bf16": dict(side=512, data_seed=synthetic.DATA_SEED_PRECISION, sort_seed=synthetic.SORT_SEED,
                              storage_bf16=True),
}


def run(name: str) -> dict:
    c = CASES[name]
    side = c["side"]
    rgb = c.get("rgb", False)
    F = synthetic.random_rgb_grid(side, c["data_seed"]) if rgb else \
        synthetic.gaussian_attributes(side * side, c["data_seed"])
    t0 = time.time()
    bf16 = c.get("storage_bf16", False)
    filt = c.get("filter", "box")
    res = oracle.sort(F, side, c["sort_seed"], energy_cap=1 << 20, storage_bf16=bf16, filter=filt)
    dt = time.time() - t0
    assert res.status == 0
    energies = np.ascontiguousarray(res.reorder_energy, dtype="<u8")
    return {
        "case": name,
        "side": side,
        "d": int(F.shape[0]),
        "data_seed": c["data_seed"],
        "sort_seed": c["sort_seed"],
        "generator": ("synthetic.random_rgb_grid" if rgb else "synthetic.gaussian_attributes") +
                     " (channel-major float32)",
        "storage": "bf16" if bf16 else "f32",
        "filter": filt,
        "reorders": int(res.reorders),
        "levels": int(res.levels),
        "scale_shift": int(res.scale_shift),
        "energy": str(res.energy),
        "perm_sha256": hashlib.sha256(np.ascontiguousarray(res.perm, dtype="<i4").tobytes()).hexdigest(),
        "perm_head": [int(v) for v in res.perm[:16]],
        "reorder_energy_sha256": hashlib.sha256(energies.tobytes()).hexdigest(),
        "trace": [dict(phi=t["phi"], r=t["r"], beta=t["beta"], reorders=t["reorders"],
                       energy=str(t["energy"]), moved=t["moved"]) for t in res.trace],
        "oracle_seconds": round(dt, 1),
        "oracle_threads": oracle.set_threads(0),
        "vad_sorted": oracle.vad(F, res.perm, side),
        "vad_start": oracle.vad(F, None, side),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("names", nargs="*", default=list(CASES))
    a = ap.parse_args()
    oracle.build(force=False)
    if a.threads:
        oracle.set_threads(a.threads)
    for name in a.names:
        out = run(name)
        path = os.path.join(HERE, f"{name}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(f"{name}: {out['reorders']} reorders, {out['levels']} levels, "
              f"{out['oracle_seconds']} s -> {path}", flush=True)


if __name__ == "__main__":
    main()
