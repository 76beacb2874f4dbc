"""Pins of O4 (per-entry section retrograde that reads (n+1)-stone child
sections, Section IV) against O2 (minimax on the concrete board, Section II)
on every slice with at most three empty cells, plus the table properties
that hold for any section (Section III: W subset of N, periodic along a dimension
whose quadrant pattern is symmetric under a turn)."""
import numpy as np
import pytest

import oracle as O


def solve_chain(counts, cache):
    """O4 over a whole section, with its child sections solved first by O4
    (recursively, down to the 36-stone slice which is computed on demand)."""
    if counts in cache:
        return cache[counts]
    stones = sum(b + w for b, w in counts)
    children = [None] * 4
    if stones < 35:
        for j in range(4):
            if sum(counts[j]) < 9:
                children[j] = solve_chain(O.child_counts(counts, j), cache)
    cache[counts] = O.section_solve(counts, children)
    return cache[counts]


def check_against_minimax(counts, table, nsample, seed):
    rng = np.random.default_rng(seed)
    idx = O.section_all_indices(counts)
    pick = rng.choice(len(idx), size=min(nsample, len(idx)), replace=False)
    boards = np.stack([O.section_board(counts, idx[k]) for k in pick])
    ref = O.minimax_tables(boards)
    assert np.array_equal(table[pick], ref)
    return O.table_values(ref)


SLICE35 = [((7, 2), (2, 7), (1, 7), (8, 1)), ((5, 4), (4, 5), (5, 4), (4, 4)),
           ((9, 0), (0, 8), (3, 6), (6, 3))]


@pytest.mark.parametrize("counts", SLICE35, ids=str)
def test_slice35_matches_minimax(counts):
    rng = np.random.default_rng(5)
    shape = O.section_shape(counts)
    idx = np.stack([rng.integers(0, m, 300) for m in shape], axis=1).astype(np.int32)
    tab = O.section_solve(counts, [None] * 4, idx)
    boards = np.stack([O.section_board(counts, t) for t in idx])
    assert np.array_equal(tab, O.minimax_tables(boards))
    vals = O.table_values(tab)
    assert {-1, 0, 1} <= set(np.unique(vals))


def test_slice34_matches_minimax():
    cache = {}
    counts = ((7, 1), (2, 7), (1, 8), (7, 1))
    tab = solve_chain(counts, cache)
    vals = check_against_minimax(counts, tab, 400, 6)
    assert {-1, 0, 1} <= set(np.unique(vals))


@pytest.mark.slow
def test_slice33_matches_minimax():
    cache = {}
    for counts in (((7, 1), (1, 7), (2, 7), (7, 1)), ((8, 0), (0, 8), (1, 8), (8, 0))):
        tab = solve_chain(counts, cache)
        check_against_minimax(counts, tab, 150, 7)


def test_tables_win_subset_notlose_and_periodic():
    cache = {}
    counts = ((7, 1), (2, 7), (1, 8), (7, 1))
    tab = solve_chain(counts, cache)
    bits = O.table_bits(tab)
    assert not (bits[:, 0] & ~bits[:, 1]).any()
    idx = O.section_all_indices(counts)
    vals = O.table_values(tab).reshape(-1, 4, 4, 4, 4)  # axes g3, g2, g1, g0
    checked = 0
    for e, t in zip(idx, vals):
        for j, (b, w) in enumerate(counts):
            code = O.class_codes(b, w)[e[j]]
            for period in (1, 2):
                if O.code_turn(code, period) == code:
                    axis = 3 - j
                    assert np.array_equal(t, np.roll(t, period, axis=axis))
                    checked += 1
    assert checked > 0


def test_missing_child_is_an_error():
    counts = ((7, 1), (2, 7), (1, 8), (7, 1))
    with pytest.raises(ValueError):
        O.section_solve(counts, [None] * 4, np.zeros((1, 4), np.int32))
