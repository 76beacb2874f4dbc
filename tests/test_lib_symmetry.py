"""CPU checks of the library's board symmetries (Section III: the 8 board
symmetries inside G = L x| D4 and the transform of a table when the
representative changes; Section IV: D4-minimal sections).  The library's
set transform and pattern maps run on the host from the same source as the
kernels, and are checked against their per-bit definitions and against the
oracle's transform of whole tables."""
import numpy as np

import oracle as O
from oracle import counts as C
from paper_1404_0743_amd import pentago as P
from test_oracle_sections import solve_chain

SECTIONS = [((8, 1), (2, 7), (7, 2), (1, 7)), ((8, 1), (2, 7), (7, 1), (0, 8))]


def bits_of(words):
    w = np.asarray(words, dtype=np.uint64)
    return np.unpackbits(w.view(np.uint8), bitorder="little").astype(bool)


def words_of(bits):
    return np.packbits(np.asarray(bits, dtype=np.uint8), bitorder="little").view(np.uint64)


def test_sym_apply_matches_per_bit_definition():
    rng = np.random.default_rng(21)
    for sym in range(8):
        pi = O.sym_quadrants(sym)
        sign = -1 if sym >= 4 else 1
        for _ in range(6):
            src = rng.integers(0, 2, 256).astype(bool)
            h = rng.integers(0, 4, 4)
            got = bits_of(P.pentago_debug_sym(words_of(src), sym, h))
            want = np.zeros(256, bool)
            for G in range(256):
                Gd = [(G >> (2 * j)) & 3 for j in range(4)]
                g = 0
                for i in range(4):
                    g |= ((sign * (Gd[pi[i]] - h[pi[i]])) & 3) << (2 * i)
                want[G] = src[g]
            assert np.array_equal(got, want), (sym, h)


def mirror_code(code):
    d = [(code // 3 ** l) % 3 for l in range(9)]
    return sum(d[3 * (l // 3) + 2 - l % 3] * 3 ** l for l in range(9))


def test_pattern_maps_match_oracle_canonical_forms():
    for sym in range(8):
        r, f = sym & 3, sym >> 2
        for b, w in [(0, 0), (1, 0), (2, 1), (4, 4), (3, 5), (8, 1), (5, 4), (1, 7)]:
            codes = O.class_codes(b, w)
            index = {int(c): i for i, c in enumerate(codes)}
            for i, cimg in enumerate(codes):
                x = O.code_turn(int(cimg), (4 - r) & 3)
                if f:
                    x = mirror_code(x)
                c, _ = O.canon(x)
                y = mirror_code(c) if f else c
                y = O.code_turn(y, r)
                ymin, k = O.canon(y)
                assert ymin == cimg
                assert P.pentago_debug_sym_pattern(sym, b, w, i) == (index[c], (-k) & 3)


def test_transform_emulated_on_host_matches_oracle():
    cache = {}
    for s in SECTIONS:
        src = solve_chain(s, cache)
        for sym in range(8):
            img = O.sym_counts(s, sym)
            pi = O.sym_quadrants(sym)
            inv = [pi.index(j) for j in range(4)]
            idx = O.section_all_indices(img)
            got = np.zeros((len(idx), 8), np.uint64)
            for e, jj in enumerate(idx):
                sidx = [0] * 4
                h = [0] * 4
                for j in range(4):
                    p, h[j] = P.pentago_debug_sym_pattern(sym, img[j][0], img[j][1], int(jj[j]))
                    sidx[inv[j]] = p
                t = src[O.section_offset(s, sidx)]
                got[e, :4] = P.pentago_debug_sym(t[:4], sym, h)
                got[e, 4:] = P.pentago_debug_sym(t[4:], sym, h)
            assert np.array_equal(got, O.section_transform(s, src, sym)), (s, sym)


def test_image_and_standardize_match_layout_arithmetic():
    rng = np.random.default_rng(5)
    sections = list(C.slice_sections(33, minimal_only=False))
    for k in rng.choice(len(sections), 60, replace=False):
        s = sections[k]
        for sym in range(8):
            assert P.pentago_section_image(s, sym) == O.sym_counts(s, sym)
        rep, sym = P.pentago_section_standardize(s)
        assert rep == min(C.d4_images(s))
        assert C.is_d4_minimal(rep)
        assert P.pentago_section_image(rep, sym) == s
        if C.is_d4_minimal(s):
            assert (rep, sym) == (s, 0)


def test_slice_sections_match_layout_arithmetic():
    most = 0
    for n in range(37):
        got = P.pentago_slice_sections(n)
        assert got == list(C.slice_sections(n, minimal_only=True)), n
        most = max(most, len(got))
    assert most == 8239   # at most 8239 sections per slice (Section IV)
    from paper_1404_0743_amd import slices
    assert slices.slice_positions(35, minimal_only=False) == sum(
        O.section_entries(s) and C.boards(s) for s in C.slice_sections(35, minimal_only=False))
