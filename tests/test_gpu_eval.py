"""GPU parity of the endgame solver (pentago_eval_batch, the Section VIII
serial solver run per board on the device) against O2 (minimax over the
Section II rules), bit for bit.  Covers 0..10 empty cells (the LDS and the
global layer paths, the roots packed several to a wave and the short chunks
at the end of a bin), boards that already show fives, invalid boards, the
persistent and the grouped launch forms and their equality."""
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


def gpu_eval(P, boards, grouped=False):
    codes = P.boards_to_codes(boards)
    dev = torch.from_numpy(codes.view(np.int16).copy()).cuda()
    out = torch.empty((len(boards), 8), dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    P.pentago_eval_batch(dev, out, status, grouped=grouped)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64), int(status.item())


def test_endgame_roots_33_stones(P):
    """The 4096 seeded boards with 17 black and 16 white stones, all checked."""
    log("33-stone roots")
    boards = I.random_placement_boards(4096, 17, 16)
    got, bad = gpu_eval(P, boards)
    assert bad == 0
    want = O.minimax_tables(boards)
    assert np.array_equal(got, want)


def test_mixed_empties_and_forms(P):
    log("mixed empties")
    boards = I.random_play_boards(3000, 28, 35, seed=21)
    full = I.random_placement_boards(40, 18, 18, seed=22)
    # boards that already show five in a row (17 black, 16 white, no rejection)
    rng = np.random.default_rng(23)
    five = []
    while len(five) < 20:
        b = np.zeros(36, np.uint8)
        perm = rng.permutation(36)
        b[perm[:17]], b[perm[17:33]] = 1, 2
        if O.five(b, 1) or O.five(b, 2):
            five.append(b)
    allb = np.concatenate([boards, full, np.array(five)])
    got, bad = gpu_eval(P, allb)
    assert bad == 0
    got2, _ = gpu_eval(P, allb, grouped=True)
    assert np.array_equal(got, got2)
    rng = np.random.default_rng(3)
    pick = np.concatenate([rng.choice(len(boards), 300, replace=False), np.arange(len(boards), len(allb))])
    want = O.minimax_tables(allb[pick])
    assert np.array_equal(got[pick], want)


@pytest.mark.parametrize("e", range(7))
def test_packed_wave_chunks_and_tails(P, e):
    """Roots with up to 6 empty cells are solved several to a wave (eight up
    to 3 empty cells, four with 4, two with 5); a bin whose size is not a
    multiple of the chunk ends in a short chunk that repeats its last root.
    Batches of 1 to 9 and 17 roots with e empty cells leave every tail
    length; each batch is checked against O2."""
    stones = 36 - e
    if e >= 3:
        boards = I.random_play_boards(17, stones, stones, seed=60 + e)
    else:
        boards = I.random_placement_boards(17, (stones + 1) // 2, stones // 2, seed=60 + e)
    log("packed chunks, empty cells", e)
    want = O.minimax_tables(boards)
    for n in (1, 2, 3, 4, 5, 6, 7, 8, 9, 17):
        got, bad = gpu_eval(P, boards[:n])
        assert bad == 0
        assert np.array_equal(got, want[:n]), n


def test_deep_roots_global_layers(P):
    log("deep roots")
    boards = np.concatenate([I.random_play_boards(3, 27, 27, seed=31),
                             I.random_play_boards(2, 26, 26, seed=32)])
    got, bad = gpu_eval(P, boards)
    assert bad == 0
    got2, _ = gpu_eval(P, boards, grouped=True)
    assert np.array_equal(got, got2)
    want = O.minimax_tables(boards)
    assert np.array_equal(got, want)


def test_invalid_boards_are_counted(P):
    log("invalid boards")
    good = I.random_placement_boards(5, 17, 16, seed=41)
    bad = good.copy()
    bad[:, :] = 0
    bad[:, :3] = 2  # white ahead of black
    many = np.zeros((1, 36), np.uint8)  # 36 empty cells: more than 10
    allb = np.concatenate([good, bad, many])
    got, nbad = gpu_eval(P, allb)
    assert nbad == 6
    assert not got[5:].any()
    assert np.array_equal(got[:5], O.minimax_tables(good))


def test_autotuned_class_threads_same_results(P):
    """The endgame autotuner picks workgroup sizes for the per-root classes;
    every pick leaves results bit-identical (8-10 empty cells included)."""
    log("endgame autotune")
    boards = np.concatenate([I.random_play_boards(500, 26, 33, seed=51)])
    want, _ = gpu_eval(P, boards)
    codes = torch.from_numpy(P.boards_to_codes(boards).view(np.int16).copy()).cuda()
    out = torch.empty((len(boards), 8), dtype=torch.int64, device="cuda")
    threads, ms = P.pentago_autotune_eval(codes, out)
    torch.cuda.synchronize()
    assert all(t in (256, 512) for t in threads) and ms > 0
    assert np.array_equal(out.cpu().numpy().view(np.uint64), want)
    got, _ = gpu_eval(P, boards)
    assert np.array_equal(got, want)
