"""Layout arithmetic of Section IV, computed from the oracle's own quadrant
orbit tables -- TEST INFRASTRUCTURE (used only to pin the tables and the
section/block reading against the totals the paper prints).

Readings (the paper states the totals, not the procedure):
  * a section is kept iff its count tuple ((b0,w0),..,(b3,w3)) is the least,
    in lexicographic order, of its images under the 8 board symmetries, which
    permute the quadrant positions (Section IV, first paragraph);
  * a section dimension of size m holds ceil(m/8) blocks (8^4 blocks, smaller
    at the boundary, Section IV);
  * block lines run along each of the four dimensions;
  * a state count "with symmetries removed" counts orbits of valid boards
    under the 8 board symmetries (Burnside's lemma).
"""
import math
from functools import lru_cache

import numpy as np

from . import class_size

# quadrant position maps of the 8 board symmetries (TL=0, TR=1, BL=2, BR=3)
_ROT = {0: 2, 2: 3, 3: 1, 1: 0}      # a quarter turn counter-clockwise
_FLIP = {0: 1, 1: 0, 2: 3, 3: 2}     # mirror left-right


def _compose(a, b):
    return {q: a[b[q]] for q in range(4)}


def quadrant_maps():
    maps = []
    r = {q: q for q in range(4)}
    for _ in range(4):
        maps.append(r)
        maps.append(_compose(_FLIP, r))
        r = _compose(_ROT, r)
    return maps


_MAPS = quadrant_maps()


def d4_images(section):
    out = []
    for m in _MAPS:
        img = [None] * 4
        for q in range(4):
            img[m[q]] = section[q]
        out.append(tuple(img))
    return out


def is_d4_minimal(section):
    return section == min(d4_images(section))


@lru_cache(maxsize=None)
def slice_sections(stones, minimal_only=True):
    tb, tw = (stones + 1) // 2, stones // 2
    quads = [(b, w) for b in range(10) for w in range(10 - b)]
    out = []
    for q0 in quads:
        for q1 in quads:
            for q2 in quads:
                b3, w3 = tb - q0[0] - q1[0] - q2[0], tw - q0[1] - q1[1] - q2[1]
                if b3 >= 0 and w3 >= 0 and b3 + w3 <= 9:
                    s = (q0, q1, q2, (b3, w3))
                    if not minimal_only or is_d4_minimal(s):
                        out.append(s)
    return tuple(out)


@lru_cache(maxsize=None)
def _class_size(b, w):
    return class_size(b, w)


def shape(section):
    return tuple(_class_size(b, w) for b, w in section)


def entries(section):
    return math.prod(shape(section))


def blocks(section):
    return math.prod(-(-m // 8) for m in shape(section))


def block_lines(section):
    nb = [-(-m // 8) for m in shape(section)]
    return sum(math.prod(nb[:j] + nb[j + 1:]) for j in range(4))


def multinomial(b, w):
    return math.factorial(9) // (math.factorial(b) * math.factorial(w) * math.factorial(9 - b - w))


def boards(section):
    return math.prod(multinomial(b, w) for b, w in section)


# ----------------------------------------------------------------- Burnside

def _cell_perms():
    base = np.arange(36).reshape(6, 6)
    out = []
    for refl in (False, True):
        for k in range(4):
            m = np.rot90(base, k)
            if refl:
                m = m[:, ::-1]
            out.append(m.reshape(36))
    return out


def _cycle_lengths(perm):
    seen = [False] * 36
    lens = []
    for i in range(36):
        if not seen[i]:
            n, j = 0, i
            while not seen[j]:
                seen[j] = True
                j = perm[j]
                n += 1
            lens.append(n)
    return lens


def _fixed_colourings(lens, nb, nw):
    """Colourings constant on each cycle with nb black and nw white cells:
    coefficient of x^nb y^nw in prod over cycles (1 + x^l + y^l)."""
    poly = {(0, 0): 1}
    for l in lens:
        nxt = {}
        for (a, b), c in poly.items():
            for da, db in ((0, 0), (l, 0), (0, l)):
                key = (a + da, b + db)
                if key[0] <= nb and key[1] <= nw:
                    nxt[key] = nxt.get(key, 0) + c
        poly = nxt
    return poly.get((nb, nw), 0)


def states_per_slice(stones):
    """Valid boards with `stones` stones, up to the 8 board symmetries."""
    nb, nw = (stones + 1) // 2, stones // 2
    total = sum(_fixed_colourings(_cycle_lengths(p), nb, nw) for p in _cell_perms())
    assert total % 8 == 0
    return total // 8
