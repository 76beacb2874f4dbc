"""Pins of the oracle's quadrant orbit tables and of the Section IV layout
reading against closed forms and against the totals the paper prints."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.counts as C
from test_oracle_rules import rot90_turn


def test_orbit_total_burnside():
    # Z4 acting on 3^9 quadrant patterns: (3^9 + 2*3^3 + 3^5) / 4 orbits
    total = sum(O.class_size(b, w) for b in range(10) for w in range(10 - b))
    assert total == (3 ** 9 + 2 * 3 ** 3 + 3 ** 5) // 4 == 4995


def test_class_sizes_burnside():
    # per (b, w): (raw + 2*fix90 + fix180) / 4 with raw the multinomial;
    # fix90 needs the 4 corners alike and the 4 edges alike; fix180 needs
    # the 4 corner/edge pairs alike, the centre free
    for b in range(10):
        for w in range(10 - b):
            raw = C.multinomial(b, w)
            fix90 = fix180 = 0
            for centre in (0, 1, 2):
                cb, cw = b - (centre == 1), w - (centre == 2)
                for corners in (0, 1, 2):
                    for edges in (0, 1, 2):
                        nb = 4 * (corners == 1) + 4 * (edges == 1)
                        nw = 4 * (corners == 2) + 4 * (edges == 2)
                        fix90 += (nb, nw) == (cb, cw)
                # 4 pairs of cells, each pair one colour
                for pb in range(5):
                    for pw in range(5 - pb):
                        if (2 * pb, 2 * pw) == (cb, cw):
                            fix180 += math.factorial(4) // (math.factorial(pb) * math.factorial(pw) * math.factorial(4 - pb - pw))
            assert O.class_size(b, w) == (raw + 2 * fix90 + fix180) // 4, (b, w)


def test_canonical_codes_are_orbit_minima():
    codes = O.class_codes(4, 4)
    assert list(codes) == sorted(codes)
    for code in codes:
        assert code == min(O.code_turn(code, k) for k in range(4))
    for code in range(0, 19683, 97):
        m, k = O.canon(code)
        assert O.code_turn(code, k) == m
        assert all(O.code_turn(code, j) != m for j in range(k))


def test_paper_totals():
    """Section IV prints: at most 8239 sections per slice; 3,654,002,393 blocks
    and 996,084,744 block lines over all slices; the largest section is 1.8 TB
    uncompressed.  Section I prints 3,009,081,623,421,558 states with
    symmetries removed and a 213 TB two-slice peak.  Section IV prints a 5.4%
    overcount from rotation abstraction and 15.2% in total."""
    max_secs = blocks = lines = 0
    largest = 0
    mem = []
    states = 0
    ent_min = ent_all = boards_all = 0
    for n in range(37):
        secs = C.slice_sections(n)
        max_secs = max(max_secs, len(secs))
        e = 0
        for s in secs:
            blocks += C.blocks(s)
            lines += C.block_lines(s)
            e += C.entries(s)
            largest = max(largest, C.entries(s))
        mem.append(64 * e)
        ent_min += e
        states += C.states_per_slice(n)
        for s in C.slice_sections(n, False):
            ent_all += C.entries(s)
            boards_all += C.boards(s)
    assert max_secs == 8239
    assert blocks == 3654002393
    assert lines == 996084744
    assert states == 3009081623421558
    assert round(64 * largest / 2 ** 40, 1) == 1.8
    assert round(max(mem[i] + mem[i + 1] for i in range(36)) / 2 ** 40) == 213
    assert round(100 * (256 * ent_all / boards_all - 1), 1) == 5.4
    assert round(100 * (256 * ent_min / states - 1), 1) == 15.2


SMALL = ((7, 1), (2, 7), (1, 8), (7, 1))


def test_offsets_are_a_bijection_with_contiguous_blocks():
    for counts in (SMALL, ((1, 1), (0, 2), (2, 1), (2, 0))):
        shape = O.section_shape(counts)
        idx = O.section_all_indices(counts)
        n = O.section_entries(counts)
        assert n == math.prod(shape) == len(idx)
        offs = np.array([O.section_offset(counts, t) for t in idx])
        assert np.array_equal(offs, np.arange(n))
        # each 8^4 block occupies one contiguous run
        blk = (idx // 8) @ np.array([1 << 24, 1 << 16, 1 << 8, 1])
        change = np.nonzero(np.diff(blk))[0]
        assert len(change) + 1 == math.prod(-(-m // 8) for m in shape)


def test_offset_hand_example():
    # shape (34,34,34,34): entry (9,17,2,33) sits in block (1,2,0,4) whose
    # extents are (8,8,8,2); earlier slabs hold 8*34^3 + 8*16*34^2 + 0 + 8*8*8*32
    counts = ((5, 4), (4, 5), (5, 4), (4, 5))
    assert O.section_shape(counts) == (34, 34, 34, 34)
    before = 8 * 34 ** 3 + 8 * 16 * 34 ** 2 + 0 + 8 * 8 * 8 * 32
    inside = ((1 * 8 + 1) * 8 + 2) * 2 + 1
    assert O.section_offset(counts, (9, 17, 2, 33)) == before + inside


def test_section_board_decodes_canonical_patterns():
    counts = ((5, 4), (4, 5), (5, 4), (4, 4))
    b = O.section_board(counts, (3, 7, 11, 150))
    for j, (nb, nw) in enumerate(counts):
        r0, c0 = 3 * (j // 2), 3 * (j % 2)
        q = b.reshape(6, 6)[r0:r0 + 3, c0:c0 + 3]
        assert (q == 1).sum() == nb and (q == 2).sum() == nw
        code = int(sum(int(d) * 3 ** l for l, d in enumerate(q.reshape(9))))
        assert code == O.class_codes(nb, nw)[(3, 7, 11, 150)[j]]
