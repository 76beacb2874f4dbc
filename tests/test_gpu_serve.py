"""GPU tests of the query server (pentago_serve_*): every answer, looked up
in a resident section or searched on the device, equals the oracle's minimax
table of the query board; each answer is the same alone and in a mixed
stream; a tiny memory budget still answers everything; the in-flight bound
gives EAGAIN."""
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


RESIDENT = ((7, 2), (2, 7), (1, 7), (8, 1))   # 35 stones, solved on the GPU


@pytest.fixture(scope="module")
def resident(P):
    child = O.child_counts(RESIDENT, 2)
    ct = torch.empty((O.section_entries(child), 8), dtype=torch.int64, device="cuda")
    P.pentago_solve_section(child, [None] * 4, ct)
    t = torch.empty((O.section_entries(RESIDENT), 8), dtype=torch.int64, device="cuda")
    P.pentago_solve_section(RESIDENT, [None, None, ct, None], t)
    torch.cuda.synchronize()
    return t


def queries(n_lookup, n_search, seed):
    """Lookups: boards of the resident section, each quadrant turned at random
    (so the server must canonicalise); searches: random-play boards."""
    rng = np.random.default_rng(seed)
    shape = O.section_shape(RESIDENT)
    look = []
    for _ in range(n_lookup):
        b = O.section_board(RESIDENT, [rng.integers(0, m) for m in shape])
        look.append(O.apply(b, int(rng.integers(0, 256))))
    search = I.random_play_boards(n_search, 29, 34, seed=seed) if n_search else np.zeros((0, 36), np.uint8)
    boards = np.concatenate([np.array(look).reshape(-1, 36), search])
    perm = rng.permutation(len(boards))
    return boards[perm]


def run_all(P, srv, codes):
    """Submit everything (waiting on the oldest ticket whenever the server
    answers EAGAIN), then collect the results in order."""
    tickets, out, done = [], {}, 0
    for c in codes:
        while True:
            t = srv.submit(c)
            if t is not None:
                tickets.append(t)
                break
            r = srv.poll(tickets[done])
            if r is not None:
                out[done] = r
                done += 1
    for i in range(done, len(tickets)):
        while True:
            r = srv.poll(tickets[i])
            if r is not None:
                out[i] = r
                break
    return np.array([out[i] for i in range(len(tickets))])


def test_answers_match_oracle_alone_and_mixed(P, resident):
    log("serve mixed")
    boards = queries(120, 200, seed=3)
    codes = P.boards_to_codes(boards)
    srv = P.Server(memory_budget=1 << 30, max_inflight=4096, max_batch=64, streams=3)
    srv.add_section(RESIDENT, resident)
    mixed = run_all(P, srv, codes)
    st = srv.stats()
    assert st["queries"] == len(boards) and st["lookups"] == 120 and st["searches"] == 200
    assert st["p50_us"] > 0 and st["p99_us"] >= st["p50_us"]
    alone = np.array([run_all(P, srv, codes[i:i + 1])[0] for i in range(0, len(codes), 7)])
    assert np.array_equal(alone, mixed[::7])
    srv.close()
    want = O.minimax_tables(boards)
    assert np.array_equal(mixed, want)


def test_tiny_budget_and_backpressure(P, resident):
    log("serve budget")
    boards = queries(10, 60, seed=4)
    codes = P.boards_to_codes(boards)
    srv = P.Server(memory_budget=1, max_inflight=16, max_batch=8, streams=2)
    srv.add_section(RESIDENT, resident)
    tickets, got = [], {}
    for c in codes[:16]:
        tickets.append(srv.submit(c))
    assert all(t is not None for t in tickets)
    assert srv.submit(codes[16]) is None          # 16 in flight: EAGAIN
    for t in tickets:
        while srv.poll(t) is None:
            pass
    res = run_all(P, srv, codes)
    srv.close()
    assert np.array_equal(res, O.minimax_tables(boards))


def test_replay_open_loop(P, resident):
    log("serve replay")
    boards = queries(50, 150, seed=5)
    codes = P.boards_to_codes(boards)
    srv = P.Server(memory_budget=1 << 30, max_inflight=4096, max_batch=64, streams=2)
    srv.add_section(RESIDENT, resident)
    arrivals = I.poisson_arrivals(len(codes), rate=20000.0, seed=6)
    res = srv.replay(codes, arrivals)
    st = srv.stats()
    srv.close()
    assert st["queries"] == len(codes)
    assert np.array_equal(res, O.minimax_tables(boards))


def test_lookups_through_board_symmetries(P, resident):
    """Boards of every image of the resident section under the 8 board
    symmetries (quadrants also turned at random) are answered by lookup in
    the one resident table, and equal the oracle's minimax tables."""
    log("serve symmetric lookups")
    rng = np.random.default_rng(9)
    shape = O.section_shape(RESIDENT)
    boards, syms = [], []
    for k in range(160):
        sym = k % 8
        b = O.section_board(RESIDENT, [rng.integers(0, m) for m in shape])
        b = O.apply(b, int(rng.integers(0, 256)))
        img = np.zeros(36, np.uint8)
        img[O.sym_cells(sym)] = b
        boards.append(img)
        syms.append(sym)
    boards = np.array(boards)
    assert len({O.sym_counts(RESIDENT, s) for s in range(8)}) == 8
    codes = P.boards_to_codes(boards)
    srv = P.Server(memory_budget=1 << 30, max_inflight=4096, max_batch=64, streams=2)
    srv.add_section(RESIDENT, resident)
    got = run_all(P, srv, codes)
    st = srv.stats()
    srv.close()
    assert st["lookups"] == len(boards) and st["searches"] == 0
    assert np.array_equal(got, O.minimax_tables(boards))


def test_deep_queries(P, resident):
    """Boards with 11 to 14 empty cells are searched by the deep solver, one
    at a time, next to ordinary searches and lookups; each answer equals the
    deep solver called directly (itself checked against minimax, the batched
    solver and the recurrence)."""
    log("serve deep queries")
    deep = I.random_play_boards(6, 22, 25, seed=91)
    mixed = np.concatenate([deep, queries(20, 20, seed=92)])
    codes = P.boards_to_codes(mixed)
    srv = P.Server(memory_budget=1 << 30, max_inflight=4096, max_batch=64, streams=3)
    srv.add_section(RESIDENT, resident)
    got = run_all(P, srv, codes)
    st = srv.stats()
    srv.close()
    assert st["queries"] == len(mixed) and st["lookups"] == 20
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    for k, c in enumerate(codes[:len(deep)]):
        P.pentago_eval_deep(c, out)
        torch.cuda.synchronize()
        assert np.array_equal(got[k], out.cpu().numpy().view(np.uint64)), k
    assert np.array_equal(got[len(deep):], O.minimax_tables(mixed[len(deep):]))


def test_lookups_do_not_wait_behind_a_deep_search(P, resident):
    """A 1 GiB budget with a 20-empty query running on the deep solver (about
    17 GB of scratch, admitted because nothing else runs): lookups hold no
    scratch, so the budget must not hold them back; they are all answered
    while the deep search is still running, and their answers equal the
    oracle's."""
    log("serve lookups beside a deep search")
    deep = I.random_play_boards(1, 16, 16, seed=93)
    look = queries(64, 0, seed=94)
    srv = P.Server(memory_budget=1 << 30, max_inflight=4096, max_batch=64, streams=2)
    srv.add_section(RESIDENT, resident)
    td = srv.submit(P.boards_to_codes(deep)[0])
    assert td is not None
    # the deep query is admitted first (it is alone), then the lookups arrive
    tl = [srv.submit(c) for c in P.boards_to_codes(look)]
    assert all(t is not None for t in tl)
    got = []
    for t in tl:
        while True:
            r = srv.poll(t)
            if r is not None:
                got.append(r)
                break
    deep_still_running = srv.poll(td) is None
    while srv.poll(td) is None:
        pass
    st = srv.stats()
    srv.close()
    assert st["lookups"] == 64 and st["searches"] == 1
    assert deep_still_running, "the lookups waited for the deep search"
    assert np.array_equal(np.array(got), O.minimax_tables(look))
