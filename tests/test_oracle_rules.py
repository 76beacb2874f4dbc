"""Pins of the oracle's rules primitives (Section I rules, f_c of Section II,
the quadrant-turn group L of Section III) against independent definitions:
a direction-vector scan for five in a row and numpy.rot90 for quadrant turns."""
import numpy as np
import pytest

import oracle as O


def scan_five(board, color):
    """Five in a row by brute force: every cell, every direction vector."""
    g = np.asarray(board).reshape(6, 6)
    for r in range(6):
        for c in range(6):
            for dr, dc in ((0, 1), (1, 0), (1, 1), (1, -1)):
                cells = [(r + i * dr, c + i * dc) for i in range(5)]
                if all(0 <= a < 6 and 0 <= b < 6 for a, b in cells):
                    if all(g[a, b] == color for a, b in cells):
                        return 1
    return 0


def rot90_turn(board, q, turns):
    """Quadrant turn via numpy.rot90 (counter-clockwise for positive k)."""
    g = np.asarray(board).reshape(6, 6).copy()
    r0, c0 = 3 * (q // 2), 3 * (q % 2)
    g[r0:r0 + 3, c0:c0 + 3] = np.rot90(g[r0:r0 + 3, c0:c0 + 3], turns)
    return g.reshape(36)


def test_thirty_two_lines():
    # 6 rows x 2 windows + 6 columns x 2 windows + 2 x 2 diagonal windows each way
    ls = O.lines()
    assert len(ls) == 32
    assert len({tuple(sorted(l)) for l in ls}) == 32


def test_five_matches_scan():
    rng = np.random.default_rng(1)
    hits = 0
    for _ in range(3000):
        density = rng.uniform(0.3, 1.0)
        b = np.where(rng.random(36) < density, rng.integers(1, 3, 36), 0).astype(np.uint8)
        for color in (1, 2):
            f = O.five(b, color)
            assert f == scan_five(b, color)
            hits += f
    assert hits > 300  # the sample exercises both outcomes


def test_each_line_alone_is_a_five():
    for line in O.lines():
        b = np.zeros(36, np.uint8)
        b[line] = 2
        assert O.five(b, 2) == 1 and O.five(b, 1) == 0
        b[line[2]] = 0
        assert O.five(b, 2) == 0


def test_turn_is_counter_clockwise():
    # a stone in the top-right corner of a quadrant moves to its top-left corner
    for q in range(4):
        r0, c0 = 3 * (q // 2), 3 * (q % 2)
        b = np.zeros(36, np.uint8)
        b[6 * r0 + c0 + 2] = 1
        t = O.turn(b, q, 1)
        assert t[6 * r0 + c0] == 1 and t.sum() == 1
        # and the top-left corner moves to the bottom-left corner
        b = np.zeros(36, np.uint8)
        b[6 * r0 + c0] = 2
        t = O.turn(b, q, 1)
        assert t[6 * (r0 + 2) + c0] == 2


def test_turn_matches_rot90():
    rng = np.random.default_rng(2)
    for _ in range(200):
        b = rng.integers(0, 3, 36).astype(np.uint8)
        for q in range(4):
            for k in range(4):
                assert np.array_equal(O.turn(b, q, k), rot90_turn(b, q, k))
            assert np.array_equal(O.turn(b, q, 3), rot90_turn(b, q, -1))


def test_apply_is_a_group_action():
    rng = np.random.default_rng(3)
    for _ in range(100):
        b = rng.integers(0, 3, 36).astype(np.uint8)
        g, h = rng.integers(0, 256, 2)
        gh = sum((((g >> (2 * j)) + (h >> (2 * j))) & 3) << (2 * j) for j in range(4))
        assert np.array_equal(O.apply(O.apply(b, h), g), O.apply(b, gh))
        # g_j turns quadrant j only
        ref = b.copy()
        for j in range(4):
            ref = rot90_turn(ref, j, (g >> (2 * j)) & 3)
        assert np.array_equal(O.apply(b, g), ref)


def test_mover_parity():
    b = np.zeros(36, np.uint8)
    assert O.mover(b) == 1
    b[0] = 1
    assert O.mover(b) == 2
    b[1] = 2
    assert O.mover(b) == 1
    b[2] = 2
    assert O.mover(b) == 0
