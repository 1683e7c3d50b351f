"""Restart determinism of the oracle's sort: a sort stopped after k
reorders and resumed from its state (with its permutation as the start)
ends exactly as the uninterrupted sort, in permutation, reorder count,
energy and per-level trace, for stops at the start, inside levels, on a
level's first reorder, and repeatedly."""
import numpy as np
import pytest

import synthetic


def _full_and_levels(ref, F, side, seed, **kw):
    full = ref.sort(F, side, seed, **kw)
    assert full.status == 0 and full.state.done
    return full


def _resume(ref, F, side, seed, stops, **kw):
    """Stop at each k in `stops` (ascending) and resume, then run to the end.
    Returns the final result and the trace stitched from all segments."""
    perm, state, trace = None, None, []
    for k in list(stops) + [0]:
        r = ref.sort(F, side, seed, max_reorders=k, init_perm=perm, resume=state, **kw)
        assert r.status == 0
        first = 0 if state is None else state.levels_run
        trace = trace[:first] + r.trace[first:]
        perm, state = r.perm, r.state
    return r, trace


@pytest.mark.parametrize("side,d,seed,kw", [(24, 59, 1, {}), (33, 3, 2, {}), (20, 14, 3, {"storage_bf16": True}),
                                            (16, 8, 4, {"filter": "box3"})])
def test_stop_and_resume_equals_uninterrupted(ref, side, d, seed, kw):
    n = side * side
    F = np.ascontiguousarray(synthetic.gaussian_attributes(n, seed)[:d])
    full = _full_and_levels(ref, F, side, seed, **kw)
    # Level boundaries: the first reorder of every level.
    starts = np.cumsum([0] + [t["reorders"] for t in full.trace])[:-1]
    picks = sorted(set([1, 2, int(starts[len(starts) // 2]), int(starts[-1]), full.reorders - 1,
                        full.reorders // 3 + 1]))
    for k in picks:
        assert 0 < k < full.reorders
        r, trace = _resume(ref, F, side, seed, [k], **kw)
        assert np.array_equal(r.perm, full.perm), k
        assert r.reorders == full.reorders and r.energy == full.energy and r.levels == full.levels
        assert trace == full.trace, k
        assert r.state.done and r.state.k == full.reorders


def test_repeated_stops(ref):
    side, seed = 28, 5
    F = np.ascontiguousarray(synthetic.gaussian_attributes(side * side, seed))
    full = _full_and_levels(ref, F, side, seed)
    stops = list(range(7, full.reorders, 37))
    r, trace = _resume(ref, F, side, seed, stops)
    assert np.array_equal(r.perm, full.perm) and trace == full.trace
    assert r.reorders == full.reorders and r.energy == full.energy


def test_state_at_a_stop(ref):
    side, seed = 20, 6
    F = np.ascontiguousarray(synthetic.gaussian_attributes(side * side, seed))
    a = ref.sort(F, side, seed, max_reorders=10)
    s = a.state
    assert not s.done and s.k == 10 and a.reorders == 10
    # Resuming a finished sort changes nothing.
    full = ref.sort(F, side, seed)
    b = ref.sort(F, side, seed, init_perm=full.perm, resume=full.state)
    assert b.status == 0 and np.array_equal(b.perm, full.perm) and b.reorders == full.reorders
    # A state without the stopped permutation is rejected.
    assert ref.sort(F, side, seed, resume=s).status == ref.INVALID
