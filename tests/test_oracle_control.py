"""Pins for the oracle's progress control (Sec. 3.1): after each reorder the
distance to the target is compared with the previous one; an improvement of
less than 0.01 % counts as none, which first draws a new block position and,
if the reorder with that position does not improve either, ends the radius
level. App. C runs the same rule at a 1e-4 threshold.

The rule is pinned four ways, none of which reuses the oracle's arithmetic:

- the improvement test against exact rational arithmetic, (E_prev - E) /
  E_prev >= 1/M, at and around the threshold, where integer shortcuts
  (floor instead of ceiling, > instead of >=) go wrong;
- hand-worked energy sequences whose actions are derived here from the
  paper's sentence, including the energy a stalled reorder leaves to beat;
- a closed form: with M = 1 only a zero energy can improve on a positive
  one, so every level of a sort with positive energies runs exactly three
  reorders and draws exactly two shifts;
- whole sorts: their per-reorder energies, replayed through a controller
  written here from Sec. 3.1, give the same level lengths, level energies and
  shift-draw count as the sort, and a stopped sort's block shift is the last
  one drawn.
"""
from fractions import Fraction

import numpy as np
import pytest

import synthetic

KEEP, SHIFT, END = 0, 1, 2


def _paper_improves(E, E_prev, M):
    # Sec. 3.1: a relative improvement below 1/M (0.01 % for M = 10^4) is no
    # improvement. A rise or no change is never one.
    return E < E_prev and Fraction(E_prev - E, E_prev) >= Fraction(1, M)


def _boundary_cases():
    rng = np.random.default_rng(7)
    prevs = [1, 2, 3, 9, 10, 11, 99, 100, 101, 9_999, 10_000, 10_001, 19_999, 20_000, 20_001,
             123_456_789, 2**40 + 12_345, 2**61 - 1, 2**62 + 7, 2**63 + 5, 2**64 - 1]
    prevs += [int(v) for v in rng.integers(1, 2**62, size=20, dtype=np.int64)]
    Ms = [1, 2, 3, 7, 10, 100, 1_000, 10_000, 100_000, 2**31 + 1, 2**32 - 1]
    for E_prev in prevs:
        for M in Ms:
            need = -(-E_prev // M)  # ceil, in Python's exact integers
            for E in {E_prev - need - 1, E_prev - need, E_prev - need + 1, E_prev - 1, E_prev,
                      E_prev + 1, 0, E_prev // 2}:
                if 0 <= E < 2**64:
                    yield E, E_prev, M


def test_improvement_is_the_exact_relative_threshold(ref):
    n = 0
    for E, E_prev, M in _boundary_cases():
        assert ref.improved(E, E_prev, True, M) == _paper_improves(E, E_prev, M), (E, E_prev, M)
        n += 1
    assert n > 3000


def test_improvement_hand_worked_boundaries(ref):
    M = 10_000
    # 0.01 % of 10001 is 1.0001: a drop of 2 is enough, a drop of 1 is not
    # (a floor of E_prev / M would accept it).
    assert ref.improved(9_999, 10_001, True, M)
    assert not ref.improved(10_000, 10_001, True, M)
    # 0.01 % of 20000 is exactly 2: a drop of exactly 0.01 % is not "less
    # than 0.01 %", so it improves (a strict > would reject it).
    assert ref.improved(19_998, 20_000, True, M)
    assert not ref.improved(19_999, 20_000, True, M)
    # No change, a rise and a zero previous energy never improve.
    for E_prev in (0, 1, 10_000, 2**63):
        assert not ref.improved(E_prev, E_prev, True, M)
        if E_prev < 2**64 - 1:
            assert not ref.improved(E_prev + 1, E_prev, True, M)
    assert not ref.improved(0, 0, True, 1)
    # The first reorder of a level has nothing to compare with.
    for E in (0, 5, 2**64 - 1):
        assert ref.improved(E, 0, False, M) and ref.improved(E, 1, False, M)


def _run(ref, energies, M):
    st = ref.Control()
    acts = [ref.control(st, E, M) for E in energies]
    return acts, st


@pytest.mark.parametrize("energies,M,want", [
    # First reorder: nothing to compare with, keep. A drop of exactly 0.01 %
    # (100 of 1,000,000) improves. A drop of 50 < 0.01 % of 999,900 stalls:
    # new shift. Against the stalled 999,850 a drop of 50 stalls again right
    # after the shift: the level ends. (Comparing with the last improving
    # energy 999,900 instead would see a drop of 100 and keep going.)
    ([1_000_000, 999_900, 999_850, 999_800], 10_000, [KEEP, KEEP, SHIFT, END]),
    # A stall, then an improvement under the new shift clears the stall: the
    # next stall draws a shift again instead of ending the level.
    ([1_000_000, 1_000_000, 990_000, 990_000, 990_000], 10_000,
     [KEEP, SHIFT, KEEP, SHIFT, END]),
    # A rise stalls too; the risen energy is the one to beat afterwards:
    # 1,000,100 -> 999,999 is a drop of 101 >= 100.01, so it improves.
    ([1_000_000, 1_000_100, 999_999, 999_999, 999_999], 10_000, [KEEP, SHIFT, KEEP, SHIFT, END]),
    # A zero energy can never improve: a constant grid runs three reorders
    # per level.
    ([0, 0, 0], 10_000, [KEEP, SHIFT, END]),
    # M = 1: only a drop to zero improves on a positive energy.
    ([500, 499, 0, 7], 1, [KEEP, SHIFT, KEEP, SHIFT]),
    # Coarse threshold M = 10: 10 % steps. 900 -> 811 drops 89 < 90: stall;
    # 811 -> 729 drops 82 >= 81.1; 729 -> 720 drops 9 < 72.9: stall.
    ([1000, 900, 811, 729, 720], 10, [KEEP, KEEP, SHIFT, KEEP, SHIFT]),
])
def test_control_on_hand_worked_sequences(ref, energies, M, want):
    acts, _ = _run(ref, energies, M)
    assert acts == want


def test_control_state_after_each_action(ref):
    acts, st = _run(ref, [1_000_000], 10_000)
    assert (st.has_prev, st.just_shifted, st.E_prev) == (1, 0, 1_000_000)
    assert ref.control(st, 999_990, 10_000) == SHIFT
    assert (st.has_prev, st.just_shifted, st.E_prev) == (1, 1, 999_990)
    assert ref.control(st, 900_000, 10_000) == KEEP
    assert (st.has_prev, st.just_shifted, st.E_prev) == (1, 0, 900_000)


class _Replay:
    """The Sec. 3.1 controller, written here from the paper for checking
    whole sorts: per level, a shift is drawn at the start; a reorder that
    improves by at least 1/M keeps it; the first stall draws a new shift and
    becomes the energy to beat; a stall right after a new shift ends the
    level."""

    def __init__(self, M):
        self.M = M
        self.levels = []      # (reorders, last energy) per finished level
        self.shifts = 0
        self._new_level()

    def _new_level(self):
        self.shifts += 1
        self.count = 0
        self.prev = None
        self.after_shift = False

    def feed(self, E):
        self.count += 1
        if self.prev is None or _paper_improves(E, self.prev, self.M):
            self.prev, self.after_shift = E, False
        elif self.after_shift:
            self.levels.append((self.count, E))
            self._new_level()
        else:
            self.shifts += 1
            self.prev, self.after_shift = E, True


@pytest.mark.parametrize("M,w,seed", [(10, 32, 1), (100, 32, 2), (10_000, 32, 3), (10_000, 24, 4)])
def test_whole_sort_replays_through_the_paper_rule(ref, M, w, seed):
    F = synthetic.gaussian_attributes(w * w, 20 + seed)
    res = ref.sort(F, w, seed, inv_threshold=M, energy_cap=1_000_000)
    assert res.status == 0 and res.state.done
    E = [int(e) for e in res.reorder_energy]
    assert len(E) == res.reorders
    rp = _Replay(M)
    for e in E:
        rp.feed(e)
    # Every level ran to its end, and no reorder is left over.
    assert rp.count == 0
    assert [(t["reorders"], t["energy"]) for t in res.trace] == rp.levels
    assert res.levels == len(rp.levels) == len(ref.schedule(w)[0])
    # One shift per level start, plus one per first stall; the replay drew a
    # shift for a level after the last one, which the sort never enters.
    assert int(res.state.j) == rp.shifts - 1


def test_one_improvement_step_closed_form(ref):
    # M = 1: improving needs E_prev - E >= E_prev, i.e. E = 0. With positive
    # energies every level is improve, stall (new shift), stall (end): three
    # reorders and two shift draws per level.
    w = 32
    F = synthetic.gaussian_attributes(w * w, 31)
    res = ref.sort(F, w, 5, inv_threshold=1, energy_cap=10_000)
    L = len(ref.schedule(w)[0])
    assert np.all(res.reorder_energy > 0)
    assert res.levels == L and all(t["reorders"] == 3 for t in res.trace)
    assert res.reorders == 3 * L and int(res.state.j) == 2 * L


@pytest.mark.parametrize("stop", [1, 2, 3, 17, 40, 95])
def test_stopped_sort_holds_the_last_drawn_shift(ref, stop):
    # A shift is drawn before the level's first reorder and after a first
    # stall, never between: the block position in force after `stop`
    # reorders is the last one drawn, and the stall flags match the replay.
    w, M, seed = 32, 10_000, 9
    F = synthetic.gaussian_attributes(w * w, 40)
    full = ref.sort(F, w, seed, energy_cap=100_000)
    res = ref.sort(F, w, seed, max_reorders=stop)
    s = res.state
    assert not s.done and s.k == stop
    assert (s.dy, s.dx) == ref.shift(seed, int(s.j) - 1, w)
    rp = _Replay(M)
    for e in full.reorder_energy[:stop]:
        rp.feed(int(e))
    assert int(s.j) == rp.shifts
    assert s.level_reorders == rp.count and s.levels_run == len(rp.levels)
    if rp.count:
        assert bool(s.just_shifted) == rp.after_shift and int(s.E_prev) == rp.prev
