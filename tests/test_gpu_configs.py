"""Oracle parity at the scale of the benchmark's own workloads, on their own
seeded inputs (the analogue of the paper's Section VII checks: forward search
on samples of the computed slices), bit for bit (tolerance 0):

  single section 36->35  (5,4),(4,5),(5,4),(4,4): all 6,288,640 entries of
                          the sweep in its tuned launch shape against O4, and
                          all 1,336,336 entries of its 36-stone child;
  batched endgame         2^20 random-play roots with 28..33 stones (seed
                          1404074303) in one persistent launch: a seeded
                          subset of 4096 against O2 (minimax), the rest against
                          the per-group launches;
  uneven layers 35/34/33  64 sections per layer (seed 1404074304 + layer):
                          the batched launch, the plan launched directly and
                          replayed from its hipGraph give the same bytes, and
                          sampled entries of every section equal O2 on the
                          concrete boards (and O4 for layer 35);
  serving                 the first 8192 queries of the serving stream (seed
                          1404074305) replayed with Poisson arrivals: every
                          answer equals the batched solver's, and a sample
                          stratified by empty cells equals O2.
"""
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


def gather(t, offs):
    """Rows offs of a device table, as (n, 8) uint64 on the host."""
    idx = torch.from_numpy(np.ascontiguousarray(offs, dtype=np.int64)).cuda()
    return t.index_select(0, idx).cpu().numpy().view(np.uint64).reshape(-1, 8)


SECTION = ((5, 4), (4, 5), (5, 4), (4, 4))
CHILD = ((5, 4), (4, 5), (5, 4), (4, 5))
PARTS = 4


@pytest.fixture(scope="module")
def section_tables(P):
    """The 36->35 section as the benchmark times it: child materialised, tile
    shape from the autotuner, then the plain call in that shape."""
    _, ce, _ = P.pentago_section_shape(CHILD)
    _, e, _ = P.pentago_section_shape(SECTION)
    child = torch.empty((ce, 8), dtype=torch.int64, device="cuda")
    P.pentago_solve_section(CHILD, [None] * 4, child)
    out = torch.empty((e, 8), dtype=torch.int64, device="cuda")
    P.pentago_autotune_section(SECTION, [None, None, None, child], out)
    out.fill_(-1)
    P.pentago_solve_section(SECTION, [None, None, None, child], out)
    torch.cuda.synchronize()
    return (child.cpu().numpy().view(np.uint64).reshape(-1, 8),
            out.cpu().numpy().view(np.uint64).reshape(-1, 8))


@pytest.mark.parametrize("part", range(PARTS))
def test_section_36to35_every_entry(P, section_tables, part):
    _, got = section_tables
    n = len(got)
    assert n == 6288640
    lo, hi = part * n // PARTS, (part + 1) * n // PARTS
    log("section 36->35, entries [%d, %d)" % (lo, hi))
    idx = O.section_all_indices(SECTION)[lo:hi]
    want = O.section_solve(SECTION, [None] * 4, idx)
    bad = np.nonzero((got[lo:hi] != want).any(axis=1))[0]
    assert len(bad) == 0, "first mismatching offsets %s" % (lo + bad[:10])


def test_child_section_36_every_entry(P, section_tables):
    child, _ = section_tables
    log("36-stone child, all entries")
    want = O.section_solve(CHILD, [None] * 4)
    bad = np.nonzero((child != want).any(axis=1))[0]
    assert len(bad) == 0, "first mismatching offsets %s" % bad[:10]


def test_batched_endgame_2p20(P):
    log("generating the 2^20 endgame roots")
    boards = I.random_play_boards(1 << 20, 28, 33)
    codes = torch.from_numpy(P.boards_to_codes(boards).view(np.int16).copy()).cuda()
    out = torch.empty((len(boards), 8), dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    P.pentago_eval_batch(codes, out, status)
    grouped = torch.empty_like(out)
    P.pentago_eval_batch(codes, grouped, status, grouped=True)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert torch.equal(out, grouped)
    rng = np.random.default_rng(I.SEED_BATCH)
    pick = np.sort(rng.choice(len(boards), 4096, replace=False))
    log("O2 on 4096 of the 2^20 roots")
    want = O.minimax_tables(boards[pick])
    got = gather(out, pick)
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert len(bad) == 0, "first mismatching roots %s" % pick[bad[:10]]


LAYER_SAMPLE = 24


@pytest.mark.parametrize("stones", [35, 34, 33])
def test_uneven_layer(P, stones):
    log("layer", stones)
    cache = {}

    def chain(counts):
        if counts in cache:
            return cache[counts]
        ch = [None] * 4
        if sum(b + w for b, w in counts) < 35:
            for j in range(4):
                if sum(counts[j]) < 9:
                    ch[j] = chain(O.child_counts(counts, j))
        t = torch.empty((O.section_entries(counts), 8), dtype=torch.int64, device="cuda")
        P.pentago_solve_section(counts, ch, t)
        cache[counts] = t
        return t

    secs = I.pick_layer_sections(stones)
    assert len(secs) == 64
    jobs = []
    for s in secs:
        ch = [None] * 4
        if stones < 35:
            for j in range(4):
                if sum(s[j]) < 9:
                    ch[j] = chain(O.child_counts(s, j))
        jobs.append((s, ch, torch.full((O.section_entries(s), 8), -1, dtype=torch.int64, device="cuda")))
    P.pentago_solve_sections(jobs)
    torch.cuda.synchronize()
    batched = [o.clone() for _, _, o in jobs]
    plan = P.SweepPlan(jobs)
    for _, _, o in jobs:
        o.fill_(-1)
    plan.launch()
    torch.cuda.synchronize()
    assert all(torch.equal(a, o) for a, (_, _, o) in zip(batched, jobs))
    for rep in range(3):
        for _, _, o in jobs:
            o.fill_(-1)
        torch.cuda.synchronize()
        plan.launch(graph=True)
        torch.cuda.synchronize()
        assert all(torch.equal(a, o) for a, (_, _, o) in zip(batched, jobs)), "graph replay %d" % rep
    plan.close()
    # sampled entries of every section against the rules (O2 on the boards)
    rng = np.random.default_rng(I.SEED_LAYERS + stones)
    boards, got, o4 = [], [], []
    for s, t in zip(secs, batched):
        n = O.section_entries(s)
        offs = np.sort(rng.choice(n, min(n, LAYER_SAMPLE), replace=False))
        idx = O.section_all_indices(s)[offs]
        boards.extend(O.section_board(s, i) for i in idx)
        g = gather(t, offs)
        got.append(g)
        if stones == 35:
            o4.append(np.array_equal(g, O.section_solve(s, [None] * 4, idx)))
    got = np.concatenate(got)
    log("O2 on %d entries of layer %d" % (len(boards), stones))
    want = O.minimax_tables(np.array(boards))
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert len(bad) == 0, "first mismatching sampled entries %s" % bad[:10]
    assert all(o4)


def test_serving_stream_sample(P):
    n = 8192
    log("serving stream: %d queries" % n)
    boards = I.random_play_boards(1 << 15, 26, 33, seed=I.SEED_SERVE)[:n]
    codes = P.boards_to_codes(boards)
    # resident: the 36->35 section and its child, as in the benchmark
    _, ce, _ = P.pentago_section_shape(CHILD)
    _, e, _ = P.pentago_section_shape(SECTION)
    child = torch.empty((ce, 8), dtype=torch.int64, device="cuda")
    P.pentago_solve_section(CHILD, [None] * 4, child)
    sec = torch.empty((e, 8), dtype=torch.int64, device="cuda")
    P.pentago_solve_section(SECTION, [None, None, None, child], sec)
    torch.cuda.synchronize()
    srv = P.Server(memory_budget=1 << 30, max_inflight=4096, max_batch=1024, streams=3)
    srv.add_section(SECTION, sec)
    srv.add_section(CHILD, child)
    arrivals = I.poisson_arrivals(n, rate=1e5, seed=I.SEED_SERVE)
    served = srv.replay(codes, arrivals)
    st = srv.stats()
    srv.close()
    assert st["queries"] == n
    dev = torch.from_numpy(codes.view(np.int16).copy()).cuda()
    ref = torch.empty((n, 8), dtype=torch.int64, device="cuda")
    P.pentago_eval_batch(dev, ref)
    torch.cuda.synchronize()
    assert np.array_equal(served, ref.cpu().numpy().view(np.uint64))
    empt = (boards == 0).sum(axis=1)
    rng = np.random.default_rng(I.SEED_SERVE)
    pick = []
    for k in range(3, 11):
        cand = np.nonzero(empt == k)[0]
        pick.extend(rng.choice(cand, min(len(cand), 20), replace=False))
    pick = np.sort(np.array(pick))
    log("O2 on %d served answers (3..10 empty cells)" % len(pick))
    want = O.minimax_tables(boards[pick])
    bad = np.nonzero((served[pick] != want).any(axis=1))[0]
    assert len(bad) == 0, "first mismatching queries %s" % pick[bad[:10]]
