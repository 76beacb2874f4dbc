"""Pins of O2 (minimax over the Section II recurrence) against what the rules
fix on their own: hand-checked golden boards, the closed form of every board
with one empty cell (placement, then one of eight turns onto a full board),
the immediate-win rule, D4 invariance (Section III) and the table properties
of the 2-bit encoding (win implies not-lose)."""
import glob
import os

import numpy as np
import pytest

import oracle as O
from paper_1404_0743_amd import inputs as I
from test_oracle_rules import rot90_turn, scan_five

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(path):
    rows, value = [], None
    for line in open(path):
        line = line.rstrip("\n")
        if line.startswith("#") or not line:
            continue
        if line.startswith("value:"):
            value = int(line.split(":")[1])
            continue
        rows.append(line)
    assert len(rows) == 6 and all(len(r) == 6 for r in rows)
    b = np.array([{".": 0, "X": 1, "O": 2}[ch] for r in rows for ch in r], np.uint8)
    return b, value


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "*.txt"))),
                         ids=lambda p: os.path.basename(p))
def test_golden_boards(path):
    board, value = load_golden(path)
    assert O.value(board) == value


def test_full_board_fixture_has_no_five():
    board, _ = load_golden(os.path.join(GOLDEN, "full_board_tie.txt"))
    assert scan_five(board, 1) == 0 and scan_five(board, 2) == 0


def one_empty_value(board):
    """Closed form for one empty cell, white to move: the placement fills the
    board; a five from it wins at once, otherwise the mover must turn one of
    four quadrants either way and the full board scores f_w - f_b."""
    p = int(np.nonzero(board == 0)[0][0])
    a = board.copy()
    a[p] = 2
    if scan_five(a, 2):
        return 1
    best = -1
    for q in range(4):
        for k in (1, -1):
            u = rot90_turn(a, q, k)
            best = max(best, scan_five(u, 2) - scan_five(u, 1))
    return best


def test_one_empty_closed_form():
    boards = I.random_placement_boards(600, 18, 17, seed=11)
    seen = set()
    vals = O.minimax_tables(boards)
    for b, t in zip(boards, vals):
        tv = O.table_values(t)
        for g in (0, 1, 37, 200, 255):
            gb = O.apply(b, g)
            if scan_five(gb, 1) or scan_five(gb, 2):
                expect = scan_five(gb, 2) - scan_five(gb, 1)
            else:
                expect = one_empty_value(gb)
            assert tv[g] == expect
            seen.add(expect)
    assert seen == {-1, 0, 1}


def test_immediate_win_rule():
    # whenever a placement makes five for the mover, the value is a win
    boards = I.random_placement_boards(300, 16, 16, seed=12)
    checked = 0
    for b in boards:
        for p in np.nonzero(b == 0)[0]:
            a = b.copy()
            a[p] = 1
            if scan_five(a, 1):
                assert O.value(b) == 1
                checked += 1
                break
    assert checked > 10


def d4_maps():
    """The 8 board symmetries as (cell permutation, quadrant map, sign):
    sign +1 for rotations, -1 for reflections (a reflection reverses the
    direction of every quadrant turn)."""
    out = []
    base = np.arange(36).reshape(6, 6)
    for refl in (False, True):
        for k in range(4):
            m = np.rot90(base, k)
            if refl:
                m = m[:, ::-1]
            perm = m.reshape(36)  # new[i] = old[perm[i]]
            qmap = {}
            for q in range(4):
                r0, c0 = 3 * (q // 2), 3 * (q % 2)
                cell = 6 * (r0 + 1) + (c0 + 1)  # quadrant centre
                newpos = int(np.nonzero(perm == cell)[0][0])
                qmap[q] = 2 * ((newpos // 6) // 3) + (newpos % 6) // 3
            out.append((perm, qmap, -1 if refl else 1))
    return out


def test_d4_invariance_of_tables():
    boards = I.random_placement_boards(24, 16, 16, seed=13)
    maps = d4_maps()
    ref = O.minimax_tables(boards)
    for perm, qmap, sign in maps:
        moved = boards[:, perm]
        tab = O.minimax_tables(moved)
        for t0, t1 in zip(O.table_values(ref), O.table_values(tab)):
            for g in range(256):
                g2 = 0
                for j in range(4):
                    g2 |= ((sign * ((g >> (2 * j)) & 3)) & 3) << (2 * qmap[j])
                assert t1[g2] == t0[g]


def test_win_implies_notlose_and_shift_law():
    boards = I.random_placement_boards(40, 16, 16, seed=14)
    tabs = O.minimax_tables(boards)
    bits = O.table_bits(tabs)
    assert not (bits[:, 0] & ~bits[:, 1]).any()
    # turning quadrant j of the board by +1 shifts the table by one step along j
    for b, t in zip(boards[:8], O.table_values(tabs[:8])):
        for j in range(4):
            tj = O.table_values(O.minimax_tables(O.turn(b, j, 1)[None])[0])
            for g in range(256):
                gj = (g & ~(3 << (2 * j))) | ((((g >> (2 * j)) + 1) & 3) << (2 * j))
                assert tj[g] == t[gj]


def test_full_boards_are_terminal():
    boards = I.random_placement_boards(50, 18, 18, seed=15)
    tv = O.table_values(O.minimax_tables(boards))
    for b, t in zip(boards, tv):
        for g in range(0, 256, 17):
            gb = O.apply(b, g)
            assert t[g] == scan_five(gb, 1) - scan_five(gb, 2)
