"""GPU parity of the batched forms: pentago_solve_sections (one batched
launch over many sections of one slice) and the sweep plan launched directly
and from a captured hipGraph must give the bytes of the per-section sweep,
which itself is checked against the oracle (O4) on sampled entries here."""
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


def solve(P, counts, children):
    out = torch.empty((O.section_entries(counts), 8), dtype=torch.int64, device="cuda")
    P.pentago_solve_section(counts, children, out)
    return out


def chain(P, counts, cache):
    if counts in cache:
        return cache[counts]
    ch = [None] * 4
    if sum(b + w for b, w in counts) < 35:
        for j in range(4):
            if sum(counts[j]) < 9:
                ch[j] = chain(P, O.child_counts(counts, j), cache)[0]
    cache[counts] = (solve(P, counts, ch), ch)
    return cache[counts]


def layer(P, stones, count, seed, lo=1e3, hi=3e6):
    secs = I.pick_layer_sections(stones, count=count, lo=lo, hi=hi, seed=seed)
    cache = {}
    plain, jobs = [], []
    for s in secs:
        ref, ch = chain(P, s, cache)
        plain.append(ref)
        jobs.append((s, ch, torch.full_like(ref, -1)))
    torch.cuda.synchronize()
    return secs, plain, jobs


@pytest.mark.parametrize("stones", [35, 34, 33])
def test_solve_sections_matches_plain(P, stones):
    log("batched layer", stones)
    secs, plain, jobs = layer(P, stones, 24, seed=500 + stones)
    P.pentago_solve_sections(jobs)
    torch.cuda.synchronize()
    for s, ref, (_, _, out) in zip(secs, plain, jobs):
        assert torch.equal(ref, out), s
    # the plain sweep itself against the oracle, sampled, on two sections
    rng = np.random.default_rng(stones)
    for s, ref in list(zip(secs, plain))[:2]:
        if stones < 35:
            continue
        shape = O.section_shape(s)
        idx = np.stack([rng.integers(0, m, 200) for m in shape], axis=1).astype(np.int32)
        offs = np.array([O.section_offset(s, t) for t in idx])
        got = ref.cpu().numpy().view(np.uint64)[offs]
        assert np.array_equal(got, O.section_solve(s, [None] * 4, idx))


def test_plan_graph_replays(P):
    log("plan graph")
    secs, plain, jobs = layer(P, 34, 16, seed=777)
    plan = P.SweepPlan(jobs)
    info = plan.info()
    assert info["tiles"] > 0 and info["grid"] > 0
    for rep in range(3):
        for _, _, out in jobs:
            out.fill_(-1)  # eager work between replays
        torch.cuda.synchronize()
        plan.launch(graph=True)
        torch.cuda.synchronize()
        for s, ref, (_, _, out) in zip(secs, plain, jobs):
            assert torch.equal(ref, out), (rep, s)
    for _, _, out in jobs:
        out.fill_(-1)
    plan.launch(graph=False)
    torch.cuda.synchronize()
    for s, ref, (_, _, out) in zip(secs, plain, jobs):
        assert torch.equal(ref, out), s
    plan.close()


def test_autotuned_tiles_give_same_bytes(P):
    log("autotune")
    counts = ((5, 4), (4, 5), (5, 4), (4, 4))
    ch = solve(P, O.child_counts(counts, 3), [None] * 4)
    ref = solve(P, counts, [None, None, None, ch])
    out = torch.full_like(ref, -1)
    shape, ms = P.pentago_autotune_section(counts, [None, None, None, ch], out)
    assert 1 <= shape["lines"] <= 8 and shape["threads"] in (256, 512) and shape["order"] in (0, 1)
    assert ms > 0
    assert torch.equal(ref, out)
    out2 = solve(P, counts, [None, None, None, ch])
    torch.cuda.synchronize()
    assert torch.equal(ref, out2)


@pytest.mark.parametrize("stones", [35, 34, 33])
def test_autotuned_batch_shape_gives_same_bytes(P, stones):
    """The batched sweep's tile-shape autotuner (threads per tile, LDS cap)
    leaves the jobs' results in their outputs, and later batches of that
    stone count (which take the tuned shape) give the same bytes as the
    per-section sweep."""
    log("batch autotune", stones)
    secs, plain, jobs = layer(P, stones, 16, seed=700 + stones)
    cap, threads, ms = P.pentago_autotune_sections(jobs)
    assert cap in (24576, 32768, 40960, 53248) and threads in (256, 512) and ms > 0
    torch.cuda.synchronize()
    for s, ref, (_, _, out) in zip(secs, plain, jobs):
        assert torch.equal(ref, out), s
    for _, _, out in jobs:
        out.fill_(-1)
    P.pentago_solve_sections(jobs)
    torch.cuda.synchronize()
    for s, ref, (_, _, out) in zip(secs, plain, jobs):
        assert torch.equal(ref, out), s


# sections whose staged quadrant (the one with most empty cells) is 2, 1, 0
# and 3, with full-board children (35 stones) or children from the chain
SHAPE_SECTIONS = [((7, 2), (2, 7), (1, 7), (8, 1)),
                  ((9, 0), (0, 8), (3, 6), (6, 3)),
                  ((8, 0), (2, 7), (2, 7), (6, 3)),
                  ((5, 4), (4, 5), (5, 4), (4, 4)),
                  ((7, 1), (2, 7), (1, 8), (7, 1)),
                  ((7, 1), (1, 7), (2, 7), (7, 1))]


@pytest.mark.parametrize("counts", SHAPE_SECTIONS, ids=str)
def test_every_tile_shape_gives_same_bytes(P, counts):
    log("tile shapes", counts)
    cache = {}
    ref, ch = chain(P, counts, cache)
    torch.cuda.synchronize()
    tried = 0
    out = torch.empty_like(ref)
    for order in (0, 1):
        for threads in (256, 512):
            for lines in range(1, 9):
                out.fill_(-1)
                try:
                    P.pentago_solve_section_shape(counts, ch, out, lines, threads, order)
                except P.PentagoError as e:
                    assert e.code == P.ERANGE  # tile over 64 KiB of LDS
                    continue
                torch.cuda.synchronize()
                assert torch.equal(ref, out), (lines, threads, order)
                tried += 1
    assert tried >= 8
    for bad in ((9, 256, 0), (4, 128, 0), (4, 256, 2)):
        with pytest.raises(P.PentagoError):
            P.pentago_solve_section_shape(counts, ch, out, *bad)
