"""Pins of the oracle's board symmetries and of its section-table transform
(Section III: the group G of approximate symmetries contains the 8 board
symmetries D4, and tables of equivalent positions are related by shifts,
dimension transpositions and reflections; Section IV: only sections whose
counts are least under D4 are computed).

The transform is pinned against sections solved directly: the table that
section_transform derives from the table of s must equal the table of the
image section solved on its own by O4 (and, on sampled entries, by the O2
minimax search on the concrete boards).  The numbering of the symmetries is
pinned to numpy's array rotation and mirroring."""
import numpy as np

import oracle as O
from oracle import counts as C
from test_oracle_sections import solve_chain


def numpy_image(board, sym):
    """Image of a 36-cell board under sym = r + 4*f: mirror left-right when f
    is set, then r counter-clockwise quarter turns (numpy's rot90)."""
    a = np.asarray(board).reshape(6, 6)
    if sym & 4:
        a = a[:, ::-1]
    return np.rot90(a, sym & 3).reshape(36)


def sym_index(perm):
    for s in range(8):
        if np.array_equal(O.sym_cells(s), perm):
            return s
    raise AssertionError("not a board symmetry")


def test_sym_cells_match_numpy_and_form_the_group():
    rng = np.random.default_rng(7)
    board = rng.integers(0, 3, 36).astype(np.uint8)
    perms = []
    for s in range(8):
        perm = O.sym_cells(s)
        assert sorted(perm) == list(range(36))
        img = np.zeros(36, np.uint8)
        img[perm] = board
        assert np.array_equal(img, numpy_image(board, s))
        perms.append(perm)
    # closed under composition, with the identity and a rotation of order 4
    for a in range(8):
        for b in range(8):
            sym_index(perms[b][perms[a]])
    assert np.array_equal(perms[0], np.arange(36))
    assert sym_index(perms[1][perms[1][perms[1][perms[1]]]]) == 0
    assert sym_index(perms[4][perms[4]]) == 0


def test_sym_quadrants_and_counts():
    # the quadrant maps are the ones the layout arithmetic uses
    maps = C.quadrant_maps()
    got = [O.sym_quadrants(s) for s in range(8)]
    assert sorted(got) == sorted(tuple(m[q] for q in range(4)) for m in maps)
    s = ((8, 1), (2, 7), (7, 2), (1, 7))
    imgs = [O.sym_counts(s, k) for k in range(8)]
    assert sorted(imgs) == sorted(C.d4_images(s))
    for k in range(8):
        q = O.sym_quadrants(k)
        for j in range(4):
            assert imgs[k][q[j]] == s[j]


# 35 stones (children computed on demand), 34 and 33 stones (children solved
# by O4 first); counts chosen with no symmetry of their own, so every image
# is a different section
SECTIONS = [((8, 1), (2, 7), (7, 2), (1, 7)),
            ((8, 1), (2, 7), (7, 1), (0, 8)),
            ((9, 0), (1, 7), (7, 1), (0, 8))]


def test_transform_equals_direct_solve():
    cache = {}
    for s in SECTIONS:
        src = solve_chain(s, cache)
        for sym in range(8):
            img = O.sym_counts(s, sym)
            direct = solve_chain(img, cache)
            assert np.array_equal(O.section_transform(s, src, sym), direct), (s, sym)


def test_transform_equals_minimax_on_sampled_entries():
    rng = np.random.default_rng(11)
    cache = {}
    s = SECTIONS[1]
    src = solve_chain(s, cache)
    for sym in (1, 4, 7):
        img = O.sym_counts(s, sym)
        idx = O.section_all_indices(img)
        pick = idx[rng.choice(len(idx), 12, replace=False)]
        got = O.section_transform(s, src, sym, idx=pick)
        boards = np.stack([O.section_board(img, i) for i in pick])
        assert np.array_equal(got, O.minimax_tables(boards))


def test_transform_composes():
    cache = {}
    s = SECTIONS[0]
    src = solve_chain(s, cache)
    perms = [O.sym_cells(k) for k in range(8)]
    for a in (1, 4, 6):
        mid = O.section_transform(s, src, a)
        sa = O.sym_counts(s, a)
        for b in (1, 5):
            ab = sym_index(perms[b][perms[a]])   # a first, then b
            assert np.array_equal(O.section_transform(sa, mid, b), O.section_transform(s, src, ab))


def test_transform_of_a_self_symmetric_section():
    # counts invariant under the reflection that exchanges quadrants 1 and 2:
    # the image section is the section itself, and its table maps onto itself
    s = ((9, 0), (1, 8), (1, 8), (7, 1))
    assert O.sym_counts(s, 5) == s
    cache = {}
    src = solve_chain(s, cache)
    assert np.array_equal(O.section_transform(s, src, 5), src)
