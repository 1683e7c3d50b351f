"""Pins for the oracle's blockwise linear assignment (Sec. 3.1, "Blockwise
Linear Assignment"; Fig. "swapping_pixels").

Each group's choice is re-derived here by exhaustive search over the 24
orderings, the 2x2 case is checked against the best of all 24 arrangements,
and the exact invariants (bijection, grid = features[perm], energy not
rising within a reorder, energy equal to a recomputation) are checked.
"""
import itertools

import numpy as np
import pytest

import synthetic


def _setup(ref, w, d, seed, layout="cn"):
    F = synthetic.random_features(w * w, d, seed, layout)
    st, s, _ = ref.scale_shift(F, layout)
    assert st == 0
    P = np.random.default_rng(seed).permutation(w * w).astype(np.int32)
    G = ref.gather(F, P, layout)
    return F, s, P, G


def _groups(ref, w, beta, dy, dx, rk):
    nb = w // beta
    pi = ref.bijection_table(beta * beta, rk)
    out = []
    for by in range(nb):
        for bx in range(nb):
            for g in range((beta * beta) // 4):
                cells = []
                for i in range(4):
                    ly, lx = divmod(int(pi[4 * g + i]), beta)
                    cells.append(((dy + by * beta + ly) % w) * w + (dx + bx * beta + lx) % w)
                out.append(cells)
    return out


@pytest.mark.parametrize("w,d,beta,r", [(16, 3, 16, 2), (20, 5, 8, 3), (17, 59, 16, 1), (9, 4, 4, 1)])
def test_each_group_takes_exhaustive_best(ref, w, d, beta, r):
    F, s, P, G = _setup(ref, w, d, seed=w + d)
    T = ref.blur(G, w, r)
    dy, dx = 3 % w, 5 % w
    rk = ref.draw(42, 1, 0)
    G0, P0 = G.copy(), P.copy()
    E, moved = ref.assign(G, T, P, w, beta, dy, dx, rk, s)
    total, moves = 0, 0
    grouped = np.zeros(w * w, dtype=bool)
    for cells in _groups(ref, w, beta, dy, dx, rk):
        q = [[ref.quantise(ref.distance(G0[a], T[b]), s) for b in cells] for a in cells]
        best = None
        for sigma in itertools.permutations(range(4)):
            cost = sum(q[i][sigma[i]] for i in range(4))
            if best is None or cost < best[0]:
                best = (cost, sigma)
        cost, sigma = best
        total += cost
        for i in range(4):
            dst = cells[sigma[i]]
            assert np.array_equal(G[dst], G0[cells[i]])
            assert P[dst] == P0[cells[i]]
            moves += sigma[i] != i
            grouped[cells[i]] = True
    for p in np.flatnonzero(~grouped):
        total += ref.quantise(ref.distance(G[p], T[p]), s)
        assert np.array_equal(G[p], G0[p]) and P[p] == P0[p]
    assert E == total
    assert moved == moves


def test_two_by_two_single_group_reaches_best_arrangement(ref):
    # beta = w = 2: the only group is the whole grid, so one reorder must
    # pick the best of all 24 arrangements against the given target.
    d = 3
    rng = np.random.default_rng(0)
    for trial in range(20):
        G = rng.uniform(-1, 1, size=(4, d)).astype(np.float32)
        T = rng.uniform(-1, 1, size=(4, d)).astype(np.float32)
        P = np.arange(4, dtype=np.int32)
        s = 40
        Gin = G.copy()
        E, _ = ref.assign(G, T, P, 2, 2, 0, 0, ref.draw(trial, 1, 0), s)
        best = min(sum(ref.quantise(ref.distance(Gin[perm[c]], T[c]), s) for c in range(4))
                   for perm in itertools.permutations(range(4)))
        assert E == best
        assert np.array_equal(G, Gin[P])


@pytest.mark.parametrize("w,d,beta", [(32, 59, 16), (33, 14, 16), (24, 3, 12), (40, 8, 40)])
def test_invariants_over_many_reorders(ref, w, d, beta):
    F, s, P, G = _setup(ref, w, d, seed=7 * w + d)
    for k in range(12):
        r = max(1, beta - 1 - k)
        T = ref.blur(G, w, r)
        before = ref.energy_fixed(G, T, s)
        dy, dx = ref.shift(9, k, w)
        E, moved = ref.assign(G, T, P, w, beta, dy, dx, ref.draw(9, 1, k), s)
        # The energy never rises within a reorder (same target), and it is
        # the energy of the new arrangement.
        assert E <= before
        assert E == ref.energy_fixed(G, T, s)
        assert moved % 1 == 0 and moved <= w * w
    # Still a bijection, and the grid is the features in that order.
    assert np.array_equal(np.sort(P), np.arange(w * w))
    assert np.array_equal(G, ref.gather(F, P))


def test_ties_keep_current_places(ref):
    # Identical features everywhere: every ordering costs the same, so the
    # identity (first in lexicographic order) wins and nothing moves.
    w, d = 16, 4
    G = np.ones((w * w, d), dtype=np.float32)
    T = ref.blur(G, w, 3)
    P = np.arange(w * w, dtype=np.int32)
    E, moved = ref.assign(G, T, P, w, 16, 5, 7, ref.draw(1, 1, 1), 30)
    assert moved == 0 and np.array_equal(P, np.arange(w * w))


def test_ungrouped_cells_outside_blocks_stay(ref):
    # w = 21, beta = 8: nb = 2, so a 5-wide strip of the rolled grid is not
    # grouped; beta^2 = 64 leaves no remainder. With beta = 9, 81 mod 4 = 1
    # leaves one cell per block.
    for beta in (8, 9):
        w, d = 21, 3
        F, s, P, G = _setup(ref, w, d, seed=beta)
        T = ref.blur(G, w, 2)
        dy, dx = 4, 11
        rk = ref.draw(3, 1, beta)
        G0, P0 = G.copy(), P.copy()
        ref.assign(G, T, P, w, beta, dy, dx, rk, s)
        grouped = np.zeros(w * w, dtype=bool)
        for cells in _groups(ref, w, beta, dy, dx, rk):
            grouped[cells] = True
        expect_ungrouped = w * w - (w // beta) ** 2 * ((beta * beta) // 4) * 4
        assert np.sum(~grouped) == expect_ungrouped
        assert np.array_equal(P[~grouped], P0[~grouped])
        assert np.array_equal(G[~grouped], G0[~grouped])
