"""Determinism double-runs: every GPU path run twice on the same inputs gives
the same bytes (the section sweep in its tuned shape, a batched layer, the
endgame batch, the deep solver, the symmetry transform), also with other
work on the device between the runs."""
import sys

import numpy as np
import pytest
import torch

from paper_1404_0743_amd import inputs as I

pytestmark = pytest.mark.gpu


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


def twice(fn, out):
    fn()
    torch.cuda.synchronize()
    first = out.clone()
    out.fill_(-1)
    junk = torch.randn(1 << 22, device="cuda").sum()   # unrelated work in between
    fn()
    torch.cuda.synchronize()
    del junk
    return first


def test_sweep_twice(P):
    s = ((6, 3), (3, 6), (5, 4), (4, 4))
    c = P.pentago_child_section(s, 3)
    ct = torch.empty((P.pentago_section_shape(c)[1], 8), dtype=torch.int64, device="cuda")
    P.pentago_solve_section(c, [None] * 4, ct)
    out = torch.empty((P.pentago_section_shape(s)[1], 8), dtype=torch.int64, device="cuda")
    P.pentago_autotune_section(s, [None, None, None, ct], out)
    first = twice(lambda: P.pentago_solve_section(s, [None, None, None, ct], out), out)
    assert torch.equal(first, out)
    img = torch.empty_like(out)
    first = twice(lambda: P.pentago_section_transform(s, out, 6, img), img)
    assert torch.equal(first, img)


def test_batched_layer_twice(P):
    secs = I.pick_layer_sections(35, count=16, lo=1e3, hi=3e6, seed=9235)
    jobs = [(s, [None] * 4, torch.empty((P.pentago_section_shape(s)[1], 8), dtype=torch.int64, device="cuda"))
            for s in secs]
    P.pentago_solve_sections(jobs)
    torch.cuda.synchronize()
    first = [o.clone() for _, _, o in jobs]
    for _, _, o in jobs:
        o.fill_(-1)
    P.pentago_solve_sections(jobs)
    torch.cuda.synchronize()
    for s, a, (_, _, b) in zip(secs, first, jobs):
        assert torch.equal(a, b), s


def test_endgame_and_deep_twice(P):
    boards = I.random_play_boards(1 << 14, 28, 33, seed=9333)
    codes = torch.from_numpy(P.boards_to_codes(boards).view(np.int16).copy()).cuda()
    out = torch.empty((len(boards), 8), dtype=torch.int64, device="cuda")
    first = twice(lambda: P.pentago_eval_batch(codes, out, None), out)
    assert torch.equal(first, out)
    b = I.random_play_boards(1, 22, 22, seed=9334)[0]
    code = P.boards_to_codes(b.reshape(1, 36))[0]
    d = torch.empty(8, dtype=torch.int64, device="cuda")
    first = twice(lambda: P.pentago_eval_deep(code, d), d)
    assert torch.equal(first, d)
