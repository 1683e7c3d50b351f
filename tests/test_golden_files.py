"""Consistency of the stored oracle results in tests/golden/ (written by
make_golden.py from oracle runs): the per-level trace adds up to the
reorder count, the levels match the schedule's count for the side, the last
level's energy is the final energy, and the recorded inputs name the seeded
generators."""
import json
import math
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NAMES = sorted(f[:-5] for f in os.listdir(GOLDEN) if f.startswith("sort_") and f.endswith(".json"))


def schedule_levels(w: int) -> int:
    phi0 = max(1.0, w / 2.0 - 1.0)
    return 1 + math.floor(math.log(phi0) / math.log(1 / 0.95))


@pytest.mark.parametrize("name", NAMES)
def test_golden_file_is_consistent(name):
    g = json.load(open(os.path.join(GOLDEN, f"{name}.json")))
    assert g["case"] == name
    assert sum(t["reorders"] for t in g["trace"]) == g["reorders"]
    assert len(g["trace"]) == g["levels"]
    assert abs(g["levels"] - schedule_levels(g["side"])) <= 1
    assert int(g["trace"][-1]["energy"]) == int(g["energy"])
    assert all(t["reorders"] >= 3 for t in g["trace"])  # improve/stall/stall at least
    assert [t["r"] for t in g["trace"]] == sorted((t["r"] for t in g["trace"]), reverse=True)
    assert len(g["perm_sha256"]) == 64 and len(g["perm_head"]) == 16
    assert g["generator"].startswith("synthetic.")
