"""Pins for the oracle's whole sort (Sec. 3.1) and its energy queries.

- validity: the result is a permutation, reproducible, independent of the
  thread count;
- special cases: a 2x2 grid (every arrangement has the same energy), a 3x3
  grid against the brute-force optimum over all 9! arrangements, a constant
  grid (every level ends after exactly three reorders);
- schedule: the level count against its closed form;
- VAD (App. C): the shuffled-grid value against its closed form.
"""
import itertools
import math

import numpy as np
import pytest

import synthetic


def test_sort_small_is_valid_and_reproducible(ref):
    w = 32
    F = synthetic.gaussian_attributes(w * w, 1)
    a = ref.sort(F, w, 0x5EED)
    b = ref.sort(F, w, 0x5EED)
    assert a.status == 0
    assert np.array_equal(np.sort(a.perm), np.arange(w * w))
    assert np.array_equal(a.perm, b.perm) and a.reorders == b.reorders and a.energy == b.energy
    c = ref.sort(F, w, 0x5EEE)
    assert not np.array_equal(a.perm, c.perm)


def test_sort_same_at_any_thread_count(ref):
    w = 40
    F = synthetic.gaussian_attributes(w * w, 5)
    before = ref.set_threads(0)
    try:
        ref.set_threads(1)
        one = ref.sort(F, w, 3, max_reorders=60, energy_cap=60)
        ref.set_threads(4)
        four = ref.sort(F, w, 3, max_reorders=60, energy_cap=60)
    finally:
        ref.set_threads(before)
    assert np.array_equal(one.perm, four.perm)
    assert np.array_equal(one.reorder_energy, four.reorder_energy)


def test_sort_lowers_energy_and_smooths(ref):
    w = 32
    F = synthetic.gaussian_attributes(w * w, 2)
    res = ref.sort(F, w, 11)
    e_sorted = ref.grid_energy_f64(F, res.perm, w, 1)
    e_random = ref.grid_energy_f64(F, None, w, 1)
    assert e_sorted < 0.6 * e_random
    assert ref.vad(F, res.perm, w) < 0.5 * ref.vad(F, None, w)


def test_layouts_agree(ref):
    w = 24
    F = synthetic.gaussian_attributes(w * w, 3)
    a = ref.sort(F, w, 5, "cn")
    b = ref.sort(np.ascontiguousarray(F.T), w, 5, "nc")
    assert np.array_equal(a.perm, b.perm)


def test_two_by_two_every_arrangement_has_the_same_energy(ref):
    # At r >= 1 every window of a 2x2 grid is the whole grid, so the target
    # is the global mean and all 24 arrangements score alike.
    F = synthetic.random_features(4, 3, 9)
    energies = [ref.grid_energy_f64(F, np.array(p, dtype=np.int32), 2, 1)
                for p in itertools.permutations(range(4))]
    assert max(energies) - min(energies) <= 1e-12 * max(energies)
    res = ref.sort(F, 2, 1)
    assert res.status == 0 and res.levels == 1 and res.reorders >= 3
    assert sorted(res.perm) == [0, 1, 2, 3]


_PERMS9 = None


def _all_energies_3x3(F):
    """Float64 energy at r = 1 of every arrangement of a 3x3 grid, computed
    directly: target = mean over the clipped 3x3 window (a 9 x 9 averaging
    matrix), energy = mean over cells of the squared distance to it."""
    global _PERMS9
    if _PERMS9 is None:
        _PERMS9 = np.array(list(itertools.permutations(range(9))), dtype=np.int64)
    A = np.zeros((9, 9))
    for y in range(3):
        for x in range(3):
            cells = [(yy, xx) for yy in range(max(0, y - 1), min(2, y + 1) + 1)
                     for xx in range(max(0, x - 1), min(2, x + 1) + 1)]
            for yy, xx in cells:
                A[y * 3 + x, yy * 3 + xx] = 1.0 / len(cells)
    X = F.T.astype(np.float64)[_PERMS9]              # [9!, 9, d]
    Y = X - np.matmul(A, X)
    return (Y * Y).sum(axis=2).mean(axis=1), _PERMS9


def test_three_by_three_against_brute_force(ref):
    # PLAS is a heuristic: its result can only be at or above the optimum
    # over all 9! arrangements (asserted for every seed). How often it hits
    # the optimum is reported and bounded loosely (parity unpinned): with two
    # groups of four and one left-over cell per reorder it often stops in a
    # near-optimal arrangement. Over these 100 seeds it hits the optimum 11
    # times, and its median rank is 64 of 362,880.
    ranks, gaps = [], []
    for seed in range(100):
        F = synthetic.random_features(9, 3, 100 + seed)
        energies, perms = _all_energies_3x3(F)
        best = energies.min()
        res = ref.sort(F, 3, seed)
        e = ref.grid_energy_f64(F, res.perm, 3, 1)
        assert e >= best * (1 - 1e-12)
        # The f64 energy of the result appears in the brute-force table.
        idx = np.flatnonzero(np.all(perms == res.perm[None, :], axis=1))
        assert idx.size == 1 and abs(energies[idx[0]] - e) <= 1e-12 * e
        rank = int(np.sum(energies < e * (1 - 1e-12)))
        # The 8 symmetries of the square keep the energy: ranks come in 8s.
        assert rank % 8 == 0
        ranks.append(rank)
        gaps.append(e / best - 1.0)
    hits = sum(r == 0 for r in ranks)
    print("3x3 over 100 seeds: optimum hit", hits, "times; ranks", sorted(ranks),
          "; median gap", float(np.median(gaps)))
    assert hits >= 5
    assert sum(r < 0.01 * len(perms) for r in ranks) >= 90
    assert np.median(gaps) < 0.2


def test_constant_features_three_reorders_per_level(ref):
    # E = 0 throughout: the first reorder of a level counts as an
    # improvement, the second stalls (new shift), the third stalls again and
    # ends the level.
    w = 20
    F = np.full((2, w * w), 0.5, dtype=np.float32)
    res = ref.sort(F, w, 1)
    phi, _, _ = ref.schedule(w)
    assert res.levels == len(phi)
    assert all(t["reorders"] == 3 for t in res.trace)
    assert res.reorders == 3 * len(phi) and res.energy == 0


@pytest.mark.parametrize("w,expect", [(64, 67), (512, 109), (1024, 122), (1448, 129)])
def test_schedule_level_count_closed_form(ref, w, expect):
    phi, r, beta = ref.schedule(w)
    phi0 = w / 2 - 1
    assert len(phi) == 1 + math.floor(math.log(phi0) / math.log(1 / 0.95)) == expect
    assert phi[0] == phi0 and r[0] == math.floor(phi0)
    assert np.all(phi >= 1.0) and phi[-1] * 0.95 < 1.0
    assert np.all(beta == np.clip(r + 1, 16, w))


def test_schedule_tiny_grids(ref):
    for w in (2, 3):
        phi, r, beta = ref.schedule(w)
        assert list(phi) == [1.0] and list(r) == [1] and list(beta) == [w]


def test_every_level_at_least_three_reorders_or_one_improvement_chain(ref):
    w = 32
    F = synthetic.gaussian_attributes(w * w, 6)
    res = ref.sort(F, w, 2, energy_cap=100000)
    assert all(t["reorders"] >= 3 for t in res.trace)
    assert sum(t["reorders"] for t in res.trace) == res.reorders
    assert res.reorder_energy[-1] == res.energy


def test_truncation_is_a_prefix(ref):
    w = 32
    F = synthetic.gaussian_attributes(w * w, 7)
    full = ref.sort(F, w, 8, energy_cap=100000)
    part = ref.sort(F, w, 8, max_reorders=50, energy_cap=50)
    assert part.reorders == 50
    assert np.array_equal(part.reorder_energy, full.reorder_energy[:50])


def test_init_perm_default_is_the_keyed_start(ref):
    w = 16
    F = synthetic.gaussian_attributes(w * w, 8)
    start = ref.bijection_table(w * w, ref.draw(4, 0, 0)).astype(np.int32)
    a = ref.sort(F, w, 4)
    b = ref.sort(F, w, 4, init_perm=start)
    assert np.array_equal(a.perm, b.perm)
    bad = start.copy()
    bad[0] = bad[1]
    assert ref.sort(F, w, 4, init_perm=bad).status == ref.INVALID


def test_invalid_arguments(ref):
    F = synthetic.gaussian_attributes(15, 1)
    assert ref.sort(F, 4, 0).status == ref.INVALID          # n != side^2
    F = synthetic.gaussian_attributes(16, 1)
    assert ref.sort(F, 4, 0, radius_decay=1.0).status == ref.INVALID
    F[3, 2] = np.nan
    assert ref.sort(F, 4, 0).status == ref.NONFINITE


def test_grid_energy_matches_pieces(ref):
    w, r = 24, 3
    F = synthetic.gaussian_attributes(w * w, 9)
    perm = synthetic.random_permutation(w * w, 1)
    st, E, s, mean = ref.grid_energy(F, perm, w, r)
    G = ref.gather(F, perm)
    assert st == 0 and E == ref.energy_fixed(G, ref.blur(G, w, r), s)
    assert abs(mean - E * 2.0 ** -s / (w * w)) <= 1e-12 * mean
    # The fixed-point mean and the float64 energy agree to float32 rounding.
    e64 = ref.grid_energy_f64(F, perm, w, r)
    assert abs(mean - e64) <= 1e-4 * e64


def test_vad_closed_forms(ref):
    # Shuffled U(0, a) values: |X - Y| has mean a/3 and variance a^2/18.
    F = synthetic.random_rgb_grid(512, 0)
    v = ref.vad(F, None, 512)
    assert abs(v / (255.0 ** 2 / 18.0) - 1.0) < 0.01
    # Hand example: 2x2, one channel [[0, 1], [3, 5]]: pairs |0-1|, |3-5|,
    # |0-3|, |1-5| = 1, 2, 3, 4 -> mean 2.5, variance 1.25.
    F = np.array([[0, 1, 3, 5]], dtype=np.float32)
    assert ref.vad(F, None, 2) == pytest.approx(1.25, abs=1e-12)
