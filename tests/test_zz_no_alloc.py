"""The allocation-free endgame call (pentago_eval_batch_noalloc, for callers
that cannot allocate device memory) against pentago_eval_batch on the same
boards, bit for bit, through the C ABI: two calls in a row, the second with a
smaller batch, so the fixed scratch array is reused with stale contents.
The batches mix 3 to 10 empty cells (the LDS classes and the global layer
slots of 9 and 10), boards showing fives and invalid boards."""
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
    pentago.pentago_init()
    return pentago


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def boards_mix(seed, n_play, n_deep):
    rng = np.random.default_rng(seed)
    play = I.random_play_boards(n_play, 28, 33, seed=seed)
    deep = I.random_play_boards(n_deep, 26, 27, seed=seed + 1)
    five = []
    while len(five) < 8:
        b = np.zeros(36, np.uint8)
        perm = rng.permutation(36)
        b[perm[:17]], b[perm[17:33]] = 1, 2
        if O.five(b, 1) or O.five(b, 2):
            five.append(b)
    bad = np.zeros((3, 36), np.uint8)
    bad[:, :3] = 2  # white ahead of black
    allb = np.concatenate([play, deep, np.array(five), bad])
    return allb[rng.permutation(len(allb))]


def run(P, boards, noalloc):
    codes = torch.from_numpy(P.boards_to_codes(boards).view(np.int16).copy()).cuda()
    out = torch.full((len(boards), 8), -1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    if noalloc:
        P.pentago_eval_batch_noalloc(codes, out, status)
    else:
        P.pentago_eval_batch(codes, out, status)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64), int(status.item())


def test_noalloc_matches_eval_batch_twice(P):
    for call, (seed, n_play, n_deep) in enumerate([(71, 6000, 150), (73, 900, 40)]):
        boards = boards_mix(seed, n_play, n_deep)
        log("call", call, "boards", len(boards), "seed", seed)
        want, want_bad = run(P, boards, noalloc=False)
        got, got_bad = run(P, boards, noalloc=True)
        assert want_bad == 3 and got_bad == 3
        bad = np.nonzero((got != want).any(axis=1))[0]
        assert len(bad) == 0, "call %d: first mismatching boards %s" % (call, bad[:10])
    # the second call's results for the small batch against the oracle too
    pick = [i for i in range(len(boards)) if (boards[i] == 0).sum() <= 6][:64]
    assert np.array_equal(got[pick], O.minimax_tables(boards[pick]))


def test_noalloc_limits(P):
    codes = torch.zeros(((1 << 20) + 1, 4), dtype=torch.int16, device="cuda")
    out = torch.empty((1, 8), dtype=torch.int64, device="cuda")
    with pytest.raises(P.PentagoError) as e:
        P.pentago_eval_batch_noalloc(codes, out)
    assert e.value.code == P.ERANGE
    empty = torch.zeros((0, 4), dtype=torch.int16, device="cuda")
    P.pentago_eval_batch_noalloc(empty, out)
