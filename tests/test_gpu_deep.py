"""GPU tests of the deep endgame solver (pentago_eval_deep; Section VIII:
positions outside the database solved from scratch, one root's DAG spread
over the GPU layer by layer).

Parity: against the oracle's minimax search (O2) for roots with up to four
empty cells, and against the batched endgame solver (itself pinned to O2) for
1..10 empty cells, and against stored minimax tables (O2, written by an
oracle-only script) at 11, 12 and 13 empty cells.  Beyond that, properties
that hold at any size: a root's table follows from the tables of its
placements by the Section II recurrence (checked bit by bit at 12 empty
cells, every placement solved separately), and tables are carried into each
other by the board symmetries (14 empty cells, the map written out with
numpy).  The parity-halved form (32 B records) against minimax and against
the full-table solver up to 18 empty cells.  Full boards, boards showing
fives, and argument errors."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1404_0743_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1404_0743_amd import pentago
    pentago.lib()
    return pentago


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def deep(P, board):
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    P.pentago_eval_deep(P.boards_to_codes(np.asarray(board).reshape(1, 36))[0], out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


def batch(P, boards):
    codes = P.boards_to_codes(np.asarray(boards).reshape(-1, 36))
    dev = torch.from_numpy(codes.view(np.int16).copy()).cuda()
    out = torch.empty((len(codes), 8), dtype=torch.int64, device="cuda")
    P.pentago_eval_batch(dev, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


def test_small_roots_match_minimax(P):
    boards = I.random_play_boards(24, 32, 35, seed=71)
    boards = np.concatenate([boards, I.random_placement_boards(8, 18, 18, seed=72)])
    want = O.minimax_tables(boards)
    for k, b in enumerate(boards):
        log("deep vs minimax", k)
        assert np.array_equal(deep(P, b), want[k]), k


def test_roots_match_batched_solver_up_to_10_empty(P):
    boards = I.random_play_boards(60, 26, 35, seed=73)
    want = batch(P, boards)
    for k, b in enumerate(boards):
        log("deep vs batch", k, "empties", int((b == 0).sum()))
        assert np.array_equal(deep(P, b), want[k]), k


def values(t):
    """8 uint64 -> int8[256] values (win + notlose - 1)."""
    return O.table_values(np.asarray(t, dtype=np.uint64).reshape(1, 8))[0]


def test_root_follows_from_its_placements_at_12_empty(P):
    """v(g.s) = terminal value if g.s shows a five, else the max over empty
    cells p of +1 when placing at p makes the mover's five, else the max over
    the 8 single-quadrant turns r of -v_t(g + r), t = s with the stone on p
    (Section II; turns commute with placements, Section III)."""
    root = I.random_play_boards(1, 24, 24, seed=74)[0]
    mover = O.mover(root)
    other = 3 - mover
    got = values(deep(P, root))
    cells = np.nonzero(root == 0)[0]
    assert len(cells) == 12
    child = {}
    for p in cells:
        t = root.copy()
        t[p] = mover
        log("placement", int(p))
        child[int(p)] = (t, values(deep(P, t)))
    want = np.zeros(256, np.int8)
    for g in range(256):
        gs = O.apply(root, g)
        fx, fy = O.five(gs, mover), O.five(gs, other)
        if fx or fy:
            want[g] = int(fx) - int(fy)
            continue
        best = -1
        for p, (t, vt) in child.items():
            if O.five(O.apply(t, g), mover):
                best = 1
                break
            for j in range(4):
                for d in (1, 3):
                    gr = (g & ~(3 << (2 * j))) | ((((g >> (2 * j)) + d) & 3) << (2 * j))
                    best = max(best, -int(vt[gr]))
        want[g] = best
    assert np.array_equal(got, want)


def d4_maps():
    """The 8 board symmetries written out with numpy (independent of the
    library and of the oracle): (cell permutation, quadrant map, sign), new
    board = old[perm]; a reflection (sign -1) reverses every quadrant turn."""
    out = []
    base = np.arange(36).reshape(6, 6)
    for refl in (False, True):
        for k in range(4):
            m = np.rot90(base, k)
            if refl:
                m = m[:, ::-1]
            perm = m.reshape(36)
            qmap = {}
            for q in range(4):
                cell = 6 * (3 * (q // 2) + 1) + (3 * (q % 2) + 1)  # quadrant centre
                newpos = int(np.nonzero(perm == cell)[0][0])
                qmap[q] = 2 * ((newpos // 6) // 3) + (newpos % 6) // 3
            out.append((perm, qmap, -1 if refl else 1))
    return out


def test_symmetric_roots_at_14_empty(P):
    """Values are invariant under the board symmetries (Section III): the
    table of the image board at g' equals the root's at g, where g' moves
    each quadrant's turns to its image quadrant, negated for a reflection."""
    root = I.random_play_boards(1, 22, 22, seed=75)[0]
    base = values(deep(P, root))
    maps = d4_maps()
    for k in (1, 2, 4, 6):
        perm, qmap, sign = maps[k]
        log("symmetry", k)
        got = values(deep(P, root[perm]))
        want = np.zeros(256, np.int8)
        for g in range(256):
            g2 = 0
            for j in range(4):
                g2 |= ((sign * ((g >> (2 * j)) & 3)) & 3) << (2 * qmap[j])
            want[g2] = base[g]
        assert np.array_equal(got, want), k


def golden_deep():
    """Boards with 11-13 empty cells and their minimax tables (oracle only:
    tests/golden/make_deep_tables.py)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "deep_minimax.tab")
    boards, tables = [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            cells, *words = line.split()
            boards.append(np.array([int(c) for c in cells], np.uint8))
            tables.append(np.array([int(w, 16) for w in words], np.uint64))
    return np.array(boards), np.array(tables)


def test_deep_roots_match_minimax_golden(P):
    """Section VIII deep positions solved from scratch: 11, 12 and 13 empty
    cells, every bit of the full table and of both parity halves against the
    oracle's minimax tables."""
    m = parity_masks()
    boards, want = golden_deep()
    assert len(boards) == 9
    assert sorted(set(int((b == 0).sum()) for b in boards)) == [11, 12, 13]
    for k, b in enumerate(boards):
        log("deep vs golden minimax", k, "empties", int((b == 0).sum()))
        assert np.array_equal(deep(P, b), want[k]), k
        for par in (0, 1):
            assert np.array_equal(deep_parity(P, b, par), want[k] & m[par]), (k, par)


def test_full_boards_and_fives(P):
    full = I.random_placement_boards(4, 18, 18, seed=76)
    # boards with two empty cells that already show a five (of either side)
    rng = np.random.default_rng(77)
    fives = []
    while len(fives) < 6:
        b = np.zeros(36, np.uint8)
        perm = rng.permutation(36)
        b[perm[:17]] = 1
        b[perm[17:34]] = 2
        if I.has_five(b, 1)[0] or I.has_five(b, 2)[0]:
            fives.append(b)
    boards = np.concatenate([full, np.array(fives)])
    want = O.minimax_tables(boards)
    for k, b in enumerate(boards):
        assert np.array_equal(deep(P, b), want[k]), k


def parity_masks():
    """Per parity of g0 + g1 + g2 + g3, the 8 uint64 words of a W/N table
    whose set bits are the rotations g of that parity (bit g0 + 4 g1 +
    16 (g2 & 1) of 32-bit word (g2 >> 1) + 2 g3 of each 256-bit set; two
    32-bit words per uint64, low word first; W then N)."""
    words = [[0] * 8, [0] * 8]
    for g in range(256):
        g0, g1, g2, g3 = g & 3, (g >> 2) & 3, (g >> 4) & 3, g >> 6
        words[(g0 + g1 + g2 + g3) & 1][(g2 >> 1) + 2 * g3] |= 1 << (g0 + 4 * g1 + 16 * (g2 & 1))
    out = np.zeros((2, 8), np.uint64)
    for par in range(2):
        for j in range(4):
            v = np.uint64(words[par][2 * j] | (words[par][2 * j + 1] << 32))
            out[par, j] = v          # W
            out[par, 4 + j] = v      # N
    return out


def deep_parity(P, board, par):
    out = torch.full((8,), -1, dtype=torch.int64, device="cuda")   # every bit set: cleared bits show
    P.pentago_eval_deep_parity(P.boards_to_codes(np.asarray(board).reshape(1, 36))[0], par, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


def test_parity_masks_split_l():
    m = parity_masks()
    assert int(np.bitwise_and(m[0], m[1]).sum()) == 0
    assert all(int(x) == (1 << 64) - 1 for x in np.bitwise_or(m[0], m[1]))
    assert sum(bin(int(x)).count("1") for x in m[0]) == 256   # 128 rotations x (W, N)


def test_parity_halves_match_minimax(P):
    """Section VIII parity halving: each half equals the minimax table (O2)
    on the rotations of its parity and is zero on the others."""
    m = parity_masks()
    boards = I.random_play_boards(8, 32, 35, seed=78)
    want = O.minimax_tables(boards)
    for k, b in enumerate(boards):
        for par in (0, 1):
            log("deep parity vs minimax", k, par)
            assert np.array_equal(deep_parity(P, b, par), want[k] & m[par]), (k, par)


def test_parity_halves_match_full_solver(P):
    """Both halves against the full-table solver, 6 to 18 empty cells; the
    two halves together give the full table."""
    m = parity_masks()
    roots = [I.random_play_boards(1, 36 - e, 36 - e, seed=80 + e)[0] for e in (6, 9, 12, 15, 16, 18)]
    for b in roots:
        e = int((b == 0).sum())
        full = deep(P, b)
        halves = []
        for par in (0, 1):
            log("deep parity vs full, empties", e, "parity", par)
            h = deep_parity(P, b, par)
            assert np.array_equal(h, full & m[par]), (e, par)
            halves.append(h)
        assert np.array_equal(halves[0] | halves[1], full), e


def test_errors(P):
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    with pytest.raises(P.PentagoError) as e:
        P.pentago_eval_deep((19683, 0, 0, 0), out)
    assert e.value.code == P.EINVAL
    for par in (-1, 2):
        with pytest.raises(P.PentagoError) as e:
            P.pentago_eval_deep_parity((0, 0, 0, 0), par, out)
        assert e.value.code == P.EINVAL
    b = np.zeros(36, np.uint8)
    b[[0, 1]] = 1                          # two black stones, no white: invalid counts
    with pytest.raises(P.PentagoError) as e:
        P.pentago_eval_deep(P.boards_to_codes(b.reshape(1, 36))[0], out)
    assert e.value.code == P.EINVAL
    b = np.zeros(36, np.uint8)
    b[:8] = 1
    b[8:15] = 2                            # 15 stones: 21 empty cells
    with pytest.raises(P.PentagoError) as e:
        P.pentago_eval_deep(P.boards_to_codes(b.reshape(1, 36))[0], out)
    assert e.value.code == P.ERANGE
