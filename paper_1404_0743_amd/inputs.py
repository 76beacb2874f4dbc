"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module produces inputs only and holds none of the solver's arithmetic:
no values, no rotation-abstracted tables, no canonical orderings.  Boards are
generated as the workloads describe (random placements, random legal play of
placement plus quadrant turn), and a board that already shows five in a row
is rejected with a small self-contained line scan.

Board encoding: uint8[36], cell 6*r + c (r downward, c rightward), 0 empty,
1 black, 2 white.  Quadrant j = 2*(r//3) + c//3.  A quadrant turn is
numpy.rot90 of the 3x3 sub-array (counter-clockwise for k=1).
"""
import math

import numpy as np

SEED_ENDGAME = 1404074301     # 4096 boards with 33 stones
SEED_BATCH = 1404074303       # 2^20 boards with 28..33 stones
SEED_LAYERS = 1404074304      # 64 sections per layer, slices 35..33
SEED_SERVE = 1404074305       # query stream, 26..33 stones


def _line_masks():
    """Bit masks (over 36 cells) of every straight run of five cells."""
    out = []
    for r in range(6):
        for c in range(6):
            for dr, dc in ((0, 1), (1, 0), (1, 1), (1, -1)):
                cells = [(r + i * dr, c + i * dc) for i in range(5)]
                if all(0 <= a < 6 and 0 <= b < 6 for a, b in cells):
                    m = 0
                    for a, b in cells:
                        m |= 1 << (6 * a + b)
                    out.append(m)
    return np.array(out, dtype=np.int64)


_LINES = _line_masks()


def _bits(boards, color):
    """(n, 36) boards -> (n,) int64 bit masks of `color`."""
    weights = (np.int64(1) << np.arange(36, dtype=np.int64))
    return ((boards == color).astype(np.int64) * weights).sum(axis=1)


def has_five(boards, color):
    """(n,) bool: does `color` show five in a row (vectorised line scan)."""
    b = _bits(np.atleast_2d(boards), color)
    return ((b[:, None] & _LINES[None, :]) == _LINES[None, :]).any(axis=1)


def _turn_index():
    """idx[q, d] is a permutation of 36 cells: board[idx] turns quadrant q by
    90 degrees (d=0 counter-clockwise, d=1 clockwise)."""
    base = np.arange(36).reshape(6, 6)
    idx = np.zeros((4, 2, 36), np.int64)
    for q in range(4):
        r0, c0 = 3 * (q // 2), 3 * (q % 2)
        for d, k in ((0, 1), (1, -1)):
            b = base.copy()
            b[r0:r0 + 3, c0:c0 + 3] = np.rot90(base[r0:r0 + 3, c0:c0 + 3], k)
            idx[q, d] = b.reshape(36)
    return idx


_TURN = _turn_index()


# ---------------------------------------------------------------- endgame roots

def random_placement_boards(n, nblack, nwhite, seed=SEED_ENDGAME):
    """n boards with nblack/nwhite stones on uniformly random cells, rejecting
    any board where either colour already has five in a row."""
    rng = np.random.default_rng(seed)
    out = []
    while sum(len(o) for o in out) < n:
        m = 2 * (n - sum(len(o) for o in out)) + 64
        keys = rng.random((m, 36))
        perm = np.argsort(keys, axis=1)
        b = np.zeros((m, 36), np.uint8)
        rows = np.arange(m)[:, None]
        b[rows, perm[:, :nblack]] = 1
        b[rows, perm[:, nblack:nblack + nwhite]] = 2
        ok = ~(has_five(b, 1) | has_five(b, 2))
        out.append(b[ok])
    return np.concatenate(out)[:n]


def _turn_shifts():
    """For each quadrant q and direction d (0 counter-clockwise, 1 clockwise):
    the 9 (source bit, destination bit) pairs of the turn on a 36-bit board."""
    out = np.zeros((4, 2, 9, 2), np.int64)
    for q in range(4):
        for d in range(2):
            perm = _TURN[q, d]  # new[i] = old[perm[i]]
            r0, c0 = 3 * (q // 2), 3 * (q % 2)
            k = 0
            for r in range(3):
                for c in range(3):
                    dst = 6 * (r0 + r) + c0 + c
                    out[q, d, k] = (perm[dst], dst)
                    k += 1
    return out


_SHIFTS = _turn_shifts()
_QMASK = np.array([sum(1 << int(t) for t in _SHIFTS[q, 0, :, 1]) for q in range(4)], np.int64)
_FULL = np.int64((1 << 36) - 1)


def _five_bits(bb):
    return ((bb[:, None] & _LINES[None, :]) == _LINES[None, :]).any(axis=1)


def _turn_bits(bb, q, d):
    out = bb.copy()
    for qq in range(4):
        for dd in range(2):
            sel = (q == qq) & (d == dd)
            if not sel.any():
                continue
            x = bb[sel]
            y = x & ~_QMASK[qq]
            for src, dst in _SHIFTS[qq, dd]:
                y |= ((x >> src) & 1) << dst
            out[sel] = y
    return out


_CHUNK = 1 << 15


def random_play_boards(n, stones_lo, stones_hi, seed=SEED_BATCH, workers=None):
    """n boards from random legal play: the stone count is uniform in
    [stones_lo, stones_hi]; each ply puts the mover's stone (black first) on a
    uniform empty cell, then turns a uniform quadrant in a uniform direction.
    A game that shows five in a row after any placement or turn is restarted.
    Boards come in fixed chunks of 2^15, chunk k drawn from the stream
    (seed, k), so the result does not depend on how many worker processes
    generate them (default: up to 16 for more than one chunk)."""
    nchunks = (n + _CHUNK - 1) // _CHUNK
    if nchunks <= 1:
        return _play_chunk((n, stones_lo, stones_hi, seed, 0))
    import multiprocessing as mp
    args = [(min(_CHUNK, n - k * _CHUNK), stones_lo, stones_hi, seed, k) for k in range(nchunks)]
    procs = workers or min(16, mp.cpu_count() or 1, nchunks)
    if procs <= 1:
        parts = [_play_chunk(a) for a in args]
    else:
        with mp.get_context("fork").Pool(procs) as pool:
            parts = pool.map(_play_chunk, args)
    return np.concatenate(parts)


def _play_chunk(args):
    n, stones_lo, stones_hi, seed, chunk = args
    rng = np.random.default_rng([seed, chunk])
    target = rng.integers(stones_lo, stones_hi + 1, size=n)
    out = np.zeros((n, 36), np.uint8)
    cells = np.arange(36, dtype=np.int64)
    for stones in range(stones_lo, stones_hi + 1):
        want = np.nonzero(target == stones)[0]
        got = []
        need = len(want)
        while need > 0:
            m = int(need * 1.3) + 64
            bb = np.zeros((2, m), np.int64)  # black, white bit boards
            alive = np.ones(m, bool)
            for ply in range(stones):
                col = ply % 2
                empty = _FULL & ~(bb[0] | bb[1])
                cell = rng.integers(0, 36, size=m)
                pending = ((empty >> cell) & 1) == 0
                while pending.any():
                    idx = np.nonzero(pending)[0]
                    cell[idx] = rng.integers(0, 36, size=len(idx))
                    pending[idx] = ((empty[idx] >> cell[idx]) & 1) == 0
                bb[col] |= np.int64(1) << cell
                alive &= ~_five_bits(bb[col])
                q = rng.integers(0, 4, size=m)
                d = rng.integers(0, 2, size=m)
                bb[0] = _turn_bits(bb[0], q, d)
                bb[1] = _turn_bits(bb[1], q, d)
                alive &= ~(_five_bits(bb[0]) | _five_bits(bb[1]))
            keep = np.nonzero(alive)[0][:need]
            b = np.zeros((len(keep), 36), np.uint8)
            b[((bb[0][keep, None] >> cells) & 1) == 1] = 1
            b[((bb[1][keep, None] >> cells) & 1) == 1] = 2
            got.append(b)
            need -= len(keep)
        out[want] = np.concatenate(got)
    return out


def codes_to_boards(codes):
    """(n, 4) quadrant codes (base 3, digit = 3 * (r % 3) + c % 3 of the
    quadrant's cell) -> (n, 36) uint8 cell arrays."""
    codes = np.asarray(codes, dtype=np.int64).reshape(-1, 4)
    boards = np.zeros((len(codes), 6, 6), np.uint8)
    digits = (codes[:, :, None] // (3 ** np.arange(9))[None, None, :]) % 3
    for j in range(4):
        r0, c0 = 3 * (j // 2), 3 * (j % 2)
        boards[:, r0:r0 + 3, c0:c0 + 3] = digits[:, j, :].reshape(-1, 3, 3)
    return boards.reshape(-1, 36)


def turn_quadrants(boards, seed):
    """Every quadrant of every board turned by an independent uniform number
    of quarter turns (numpy.rot90 of the 3x3 sub-array)."""
    rng = np.random.default_rng(seed)
    b = np.array(boards, dtype=np.uint8).reshape(-1, 6, 6)
    k = rng.integers(0, 4, size=(len(b), 4))
    for j in range(4):
        r0, c0 = 3 * (j // 2), 3 * (j % 2)
        for t in range(1, 4):
            sel = k[:, j] == t
            if sel.any():
                b[sel, r0:r0 + 3, c0:c0 + 3] = np.rot90(b[sel, r0:r0 + 3, c0:c0 + 3], t, axes=(1, 2))
    return b.reshape(-1, 36)


def board_symmetries(boards, seed):
    """Every board under an independent uniform one of the 8 board
    symmetries (the mirror numpy.fliplr or not, then 0..3 numpy.rot90
    quarter turns of the 6x6 array)."""
    rng = np.random.default_rng(seed)
    b = np.array(boards, dtype=np.uint8).reshape(-1, 6, 6)
    k = rng.integers(0, 8, size=len(b))
    out = b.copy()
    for sym in range(1, 8):
        sel = k == sym
        if sel.any():
            x = b[sel][:, :, ::-1] if sym & 4 else b[sel]
            out[sel] = np.rot90(x, sym & 3, axes=(1, 2))
    return out.reshape(-1, 36)


def resident_entries(section_sizes, n, seed):
    """n (section number, entry number) pairs: a uniform section, then a
    uniform entry of it.  section_sizes: the shape (4 extents) of each."""
    rng = np.random.default_rng(seed)
    sec = rng.integers(0, len(section_sizes), size=n)
    idx = np.stack([rng.integers(0, np.array([section_sizes[s][j] for s in sec]))
                    for j in range(4)], axis=1)
    return sec, idx


def poisson_arrivals(n, rate, seed=SEED_SERVE):
    """Arrival times (seconds) of an open-loop Poisson stream."""
    rng = np.random.default_rng(seed + 1)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


# ---------------------------------------------------------------- sections

def _multinomial(b, w):
    return math.factorial(9) // (math.factorial(b) * math.factorial(w) * math.factorial(9 - b - w))


def section_positions(counts):
    """Boards in a section: product over quadrants of 9!/(b! w! e!)."""
    p = 1
    for b, w in counts:
        p *= _multinomial(b, w)
    return p


def all_sections(stones):
    """Every count tuple ((b0,w0),..,(b3,w3)) with the slice's totals."""
    tb, tw = (stones + 1) // 2, stones // 2
    quads = [(b, w) for b in range(10) for w in range(10 - b)]
    out = []
    for q0 in quads:
        for q1 in quads:
            for q2 in quads:
                b3, w3 = tb - q0[0] - q1[0] - q2[0], tw - q0[1] - q1[1] - q2[1]
                if b3 >= 0 and w3 >= 0 and b3 + w3 <= 9:
                    out.append((q0, q1, q2, (b3, w3)))
    return out


def pick_layer_sections(stones, count=64, lo=1e4, hi=2e8, bins=8, seed=SEED_LAYERS):
    """`count` sections of one slice, stratified log-uniformly by size: the
    candidates with positions in [lo, hi] are split into `bins` equal log10
    bins and count/bins are drawn without replacement from each (a bin short
    of candidates gives what it has and the rest come from its neighbours)."""
    rng = np.random.default_rng(seed + stones)
    cands = [s for s in all_sections(stones) if lo <= section_positions(s) <= hi]
    logs = np.array([math.log10(section_positions(s)) for s in cands])
    edges = np.linspace(math.log10(lo), math.log10(hi), bins + 1)
    which = np.clip(np.searchsorted(edges, logs, side="right") - 1, 0, bins - 1)
    per = count // bins
    chosen = []
    spare = []
    for k in range(bins):
        ids = np.nonzero(which == k)[0]
        rng.shuffle(ids)
        chosen.extend(ids[:per].tolist())
        spare.extend(ids[per:].tolist())
    rng.shuffle(spare)
    chosen.extend(spare[:count - len(chosen)])
    return [cands[i] for i in sorted(chosen)]


def random_tables(n, seed, win_fraction=0.3, lose_fraction=0.3):
    """(n, 8) uint64 random win/not-lose tables with win a subset of not-lose.
    Each of the 256 bits is win with probability win_fraction, loss with
    probability lose_fraction, else tie."""
    rng = np.random.default_rng(seed)
    u = rng.random((n, 256))
    win = u < win_fraction
    notlose = u < 1.0 - lose_fraction
    packed = np.concatenate([np.packbits(win, axis=1, bitorder="little"),
                             np.packbits(notlose, axis=1, bitorder="little")], axis=1)
    return np.ascontiguousarray(packed).view(np.uint64).reshape(n, 8)
