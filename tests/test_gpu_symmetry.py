"""GPU parity of the board-symmetry transform of section tables
(pentago_section_transform; Section III: tables under the board symmetries
of G = L x| D4) against the oracle's transform, bit for bit, and against
the sweep of each image section solved on its own.

Cases: all 8 symmetries on small sections (oracle source tables, ragged
blocks, several blocks per dimension), a 1.6e6-entry section, and the full
1.26e9-position section (5,4),(4,5),(5,4),(4,4) (every entry against the
direct sweep of the image, sampled entries against the oracle).  Then the
sweep over representatives (pentago_solve_section_d4, Section IV: only
D4-minimal sections are computed): whole chains of 35-, 34- and 33-stone
sections in which every level holds only representatives, against the
oracle's chain over the sections themselves, and a 4.07e6-entry section
against the plain sweep."""
import sys

import numpy as np
import pytest

import oracle as O
from test_gpu_sweep import from_dev, gpu_chain, gpu_solve, oracle_chain, to_dev

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


def transform(P, counts, table, sym):
    out = torch.empty_like(table)
    P.pentago_section_transform(counts, table, sym, out)
    torch.cuda.synchronize()
    return out


SMALL = [((8, 1), (2, 7), (7, 2), (1, 7)),    # 35 stones, shape (3, 9, 9, 18)
         ((8, 1), (2, 7), (7, 1), (0, 8)),    # 34 stones
         ((9, 0), (1, 7), (7, 1), (0, 8)),    # 33 stones
         ((9, 0), (1, 8), (1, 8), (7, 1))]    # invariant under symmetry 5


@pytest.mark.parametrize("counts", SMALL, ids=str)
def test_small_sections_match_oracle(P, counts):
    cache = {}
    src = oracle_chain(counts, cache)
    dsrc = to_dev(src)
    for sym in range(8):
        log("transform", counts, "sym", sym)
        got = from_dev(transform(P, counts, dsrc, sym))
        want = O.section_transform(counts, src, sym)
        bad = np.nonzero((got != want).any(axis=1))[0]
        assert len(bad) == 0, (sym, bad[:10])


def test_medium_section_matches_direct_sweep_and_oracle(P):
    counts = ((5, 4), (4, 5), (3, 6), (6, 2))    # 35 stones
    cache = {}
    src = gpu_chain(P, counts, cache)
    host = from_dev(src)
    rng = np.random.default_rng(3)
    for sym in range(8):
        img = P.pentago_section_image(counts, sym)
        log("medium", counts, "sym", sym, "image", img)
        got = transform(P, counts, src, sym)
        assert torch.equal(got, gpu_chain(P, img, cache))
        if sym in (3, 6):
            idx = O.section_all_indices(img)
            pick = np.sort(rng.choice(len(idx), 48, replace=False))
            want = O.section_transform(counts, host, sym, idx=idx[pick])
            assert np.array_equal(from_dev(got)[pick], want)


def test_full_size_section(P):
    counts = ((5, 4), (4, 5), (5, 4), (4, 4))
    cache = {}
    src = gpu_chain(P, counts, cache)
    host = None
    rng = np.random.default_rng(4)
    for sym in range(8):
        img = P.pentago_section_image(counts, sym)
        log("full size sym", sym, "image", img)
        got = transform(P, counts, src, sym)
        direct = gpu_chain(P, img, cache)
        assert torch.equal(got, direct)
        if sym == 5:
            host = from_dev(src)
            idx = O.section_all_indices(img)
            pick = np.sort(rng.choice(len(idx), 40, replace=False))
            want = O.section_transform(counts, host, sym, idx=idx[pick])
            assert np.array_equal(from_dev(got)[pick], want)
        if img != counts:
            del cache[img]
        del got, direct
        torch.cuda.empty_cache()


def test_transform_errors(P):
    counts = SMALL[0]
    t = torch.zeros((O.section_entries(counts), 8), dtype=torch.int64, device="cuda")
    with pytest.raises(P.PentagoError) as e:
        P.pentago_section_transform(counts, t, 1, t)
    assert e.value.code == P.EINVAL
    with pytest.raises(P.PentagoError) as e:
        P.pentago_section_transform(counts, t, 8, torch.empty_like(t))
    assert e.value.code == P.EINVAL
    with pytest.raises(P.PentagoError) as e:
        P.pentago_section_transform(((9, 9), (0, 0), (0, 0), (0, 0)), t, 0, torch.empty_like(t))
    assert e.value.code == P.EINVAL


# ------------------------------------------------- sweeps over representatives

def d4_chain(P, counts, cache):
    """Table of a representative section, computed with every section below
    it held only as its representative (pentago_solve_section_d4 at every
    level; 36-stone representatives by the terminal path)."""
    if counts in cache:
        return cache[counts]
    if sum(b + w for b, w in counts) == 36:
        t = gpu_solve(P, counts, [None] * 4)
    else:
        reps = [None] * 4
        for j in range(4):
            if sum(counts[j]) < 9:
                rep, _ = P.pentago_section_standardize(O.child_counts(counts, j))
                reps[j] = d4_chain(P, rep, cache)
        t = torch.empty((O.section_entries(counts), 8), dtype=torch.int64, device="cuda")
        P.pentago_solve_section_d4(counts, reps, t)
        torch.cuda.synchronize()
    cache[counts] = t
    return t


# representatives with children that are not (35, 34 and 33 stones)
D4_SECTIONS = [((1, 7), (1, 8), (9, 0), (7, 2)),
               ((1, 8), (7, 0), (7, 2), (2, 7)),
               ((1, 7), (1, 8), (8, 1), (7, 1)),
               ((1, 7), (1, 8), (8, 0), (7, 1)),
               ((0, 9), (8, 0), (8, 0), (1, 7))]


@pytest.mark.parametrize("counts", D4_SECTIONS, ids=str)
def test_d4_chain_matches_oracle(P, counts):
    log("d4 chain", counts)
    assert P.pentago_section_standardize(counts) == (counts, 0)
    assert any(sum(counts[j]) < 9 and P.pentago_section_standardize(O.child_counts(counts, j))[1] != 0
               for j in range(4))
    got = from_dev(d4_chain(P, counts, {}))
    want = oracle_chain(counts, {})
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert len(bad) == 0, bad[:10]


def test_d4_sweep_full_size(P):
    # 35 stones, 4,069,120 entries; its 36-stone child is an image of its
    # representative ((4,5),(4,5),(4,5),(6,3)), not that section itself
    counts = ((4, 4), (4, 5), (6, 3), (4, 5))
    child = O.child_counts(counts, 0)
    rep, sym = P.pentago_section_standardize(child)
    log("d4 full size", counts, "child", child, "rep", rep, "sym", sym)
    assert sym != 0
    n = O.section_entries(counts)
    rep_t = gpu_solve(P, rep, [None] * 4)
    got = torch.empty((n, 8), dtype=torch.int64, device="cuda")
    P.pentago_solve_section_d4(counts, [rep_t, None, None, None], got)
    direct = gpu_solve(P, counts, [gpu_solve(P, child, [None] * 4), None, None, None])
    assert torch.equal(got, direct)
    ondemand = gpu_solve(P, counts, [None] * 4)
    assert torch.equal(got, ondemand)


def test_d4_sweep_with_tuned_shape(P):
    """Once the tile autotuner has tuned the plain sweep of the headline
    section, later sweeps of its geometry take the tuned shape; the sweep
    over the child's representative, whose kernel variant takes more lines
    per tile than that shape at 512 threads, still equals the plain sweep
    bit for bit."""
    counts = ((5, 4), (4, 5), (5, 4), (4, 4))
    child = O.child_counts(counts, 3)
    rep, sym = P.pentago_section_standardize(child)
    assert sym != 0
    n = O.section_entries(counts)
    ct = gpu_solve(P, child, [None] * 4)
    rep_t = gpu_solve(P, rep, [None] * 4)
    plain = torch.empty((n, 8), dtype=torch.int64, device="cuda")
    shape, _ = P.pentago_autotune_section(counts, [None, None, None, ct], plain)
    log("tuned shape", shape)
    got = torch.full_like(plain, -1)
    P.pentago_solve_section_d4(counts, [None, None, None, rep_t], got)
    torch.cuda.synchronize()
    assert torch.equal(got, plain)
