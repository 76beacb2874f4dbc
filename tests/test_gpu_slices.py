"""GPU parity of whole-slice sweeps over D4 representatives
(pentago_solve_sections_d4 through paper_1404_0743_amd.slices; Section IV: a
slice's D4-minimal sections, each computed from the representatives of the
slice above): every section of slice 35 (330 sections, 1.2e8 entries,
7.7 GB; the 36-stone children on demand) and of slice 34 (750 sections,
9.9e8 entries, 63 GB, from slice 35).

Sampled entries of every section against the oracle's minimax search on the
concrete boards (one and two empty cells); whole sections against the
single-section sweeps (with the children themselves, rebuilt by the
symmetry transform, and over representatives); the slice-35 plan replayed
from a hipGraph."""
import sys

import numpy as np
import pytest

import oracle as O
from test_gpu_sweep import from_dev

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


@pytest.fixture(scope="module")
def slices(P):
    from paper_1404_0743_amd import slices as S
    log("slice 35")
    t35 = S.solve_slice(35)
    torch.cuda.synchronize()
    log("slice 34")
    t34 = S.solve_slice(34, t35)
    torch.cuda.synchronize()
    yield S, t35, t34
    del t35, t34
    torch.cuda.empty_cache()


def sampled_against_minimax(P, tables, per_section, seed):
    rng = np.random.default_rng(seed)
    boards, rows = [], []
    for counts, t in tables.items():
        shape = O.section_shape(counts)
        idxs = [[int(rng.integers(0, m)) for m in shape] for _ in range(per_section)]
        offs = torch.tensor([O.section_offset(counts, i) for i in idxs], dtype=torch.int64, device="cuda")
        boards += [O.section_board(counts, i) for i in idxs]
        rows.append(from_dev(t.index_select(0, offs)))
    return np.array_equal(np.concatenate(rows), O.minimax_tables(np.array(boards)))


def test_slice_sizes(P, slices):
    S, t35, t34 = slices
    assert len(t35) == 330 and len(t34) == 750
    for tables in (t35, t34):
        assert all(t.shape[0] == O.section_entries(s) for s, t in tables.items())
    assert all(P.pentago_section_standardize(s) == (s, 0) for s in list(t35) + list(t34))


def test_slice35_sampled_against_minimax(P, slices):
    S, t35, _ = slices
    log("slice 35 sampled")
    assert sampled_against_minimax(P, t35, 3, seed=35)


def test_slice34_sampled_against_minimax(P, slices):
    S, _, t34 = slices
    log("slice 34 sampled")
    assert sampled_against_minimax(P, t34, 2, seed=34)


def whole_sections(tables, k):
    """The k largest sections and k more spread over the rest."""
    order = sorted(tables, key=lambda s: -tables[s].shape[0])
    return order[:k] + order[k::max(1, len(order) // k)][:k]


def test_slice35_whole_sections_against_single_sweeps(P, slices):
    S, t35, _ = slices
    for s in whole_sections(t35, 4):
        log("slice 35 section", s)
        out = torch.empty_like(t35[s])
        P.pentago_solve_section(s, [None] * 4, out)
        torch.cuda.synchronize()
        assert torch.equal(out, t35[s])


def test_slice34_whole_sections_against_single_sweeps(P, slices):
    S, t35, t34 = slices
    for s in whole_sections(t34, 4):
        log("slice 34 section", s)
        direct, reps = [None] * 4, [None] * 4
        for j in range(4):
            if sum(s[j]) < 9:
                c = P.pentago_child_section(s, j)
                rep, sym = P.pentago_section_standardize(c)
                reps[j] = t35[rep]
                direct[j] = torch.empty_like(t35[rep])
                P.pentago_section_transform(rep, t35[rep], sym, direct[j])
        plain = torch.empty_like(t34[s])
        P.pentago_solve_section(s, direct, plain)
        d4 = torch.empty_like(t34[s])
        P.pentago_solve_section_d4(s, reps, d4)
        torch.cuda.synchronize()
        assert torch.equal(plain, t34[s])
        assert torch.equal(d4, t34[s])


def test_slice35_plan_graph_replays(P, slices):
    S, t35, _ = slices
    jobs, tables = S.slice_jobs(35, None)
    plan = P.SweepPlan(jobs, reps=True)
    for rep in range(3):
        for t in tables.values():
            t.zero_()
        plan.launch(graph=True)
        torch.cuda.synchronize()
        assert all(torch.equal(tables[s], t35[s]) for s in tables), rep
    plan.close()


def test_server_answers_whole_slices_from_representatives(P, slices):
    """Every representative of slices 35 and 34 registered in a server:
    any position with 34 or 35 stones is then a lookup (its section is an
    image of a representative), and the answers equal the minimax search."""
    from paper_1404_0743_amd import inputs as I
    from test_gpu_serve import run_all
    S, t35, t34 = slices
    srv = P.Server(memory_budget=1 << 30, max_inflight=4096, max_batch=256, streams=3)
    for tables in (t35, t34):
        for counts, t in tables.items():
            srv.add_section(counts, t)
    boards = np.concatenate([I.random_play_boards(150, 35, 35, seed=351),
                             I.random_play_boards(150, 34, 34, seed=341)])
    log("whole-slice lookups", len(boards))
    got = run_all(P, srv, P.boards_to_codes(boards))
    st = srv.stats()
    srv.close()
    assert st["lookups"] == len(boards) and st["searches"] == 0
    assert np.array_equal(got, O.minimax_tables(boards))


def test_slice33_streamed_sampled_against_minimax(P, slices):
    """Slice 33 (1,343 D4-minimal sections, 5.3e9 entries, 337.8 GB: more
    than the GPU holds next to slice 34) solved whole from the slice-34
    representatives in batches through one arena in HBM; after each batch,
    every section is checked for win within not-lose and sampled, and the
    samples are compared with the oracle's minimax search on the boards
    (three empty cells)."""
    S, _, t34 = slices
    rng = np.random.default_rng(33)
    boards, rows, seen = [], [], []
    bad_subset = []

    def sink(tables):
        for counts, t in tables.items():
            seen.append(counts)
            if bool((t[:, :4] & ~t[:, 4:]).any()):
                bad_subset.append(counts)
            shape = O.section_shape(counts)
            idxs = [[int(rng.integers(0, m)) for m in shape] for _ in range(2)]
            offs = torch.tensor([O.section_offset(counts, i) for i in idxs], dtype=torch.int64, device="cuda")
            boards.extend(O.section_board(counts, i) for i in idxs)
            rows.append(from_dev(t.index_select(0, offs)))
        log("slice 33: %d sections so far" % len(seen))

    nb = S.solve_slice_streamed(33, t34, sink)
    torch.cuda.synchronize()
    assert nb > 1
    assert len(seen) == 1343 and len(set(seen)) == 1343
    assert set(seen) == set(P.pentago_slice_sections(33))
    assert not bad_subset
    log("slice 33: minimax on %d sampled entries" % len(boards))
    assert np.array_equal(np.concatenate(rows), O.minimax_tables(np.array(boards)))
