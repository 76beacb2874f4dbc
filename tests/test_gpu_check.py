"""GPU checks of solved tables (pentago_table_counts, pentago_validate_table,
debug-validate mode): the counts of won, tied and lost (entry, rotation) pairs
that Section VII uses to check computed slices, against the same counts taken
in numpy on the oracle's own tables (O4) and on the GPU tables; their
invariance under the board symmetries; and the rejection of a table with an
entry whose win set is not inside its not-lose set."""
import sys

import numpy as np
import pytest

import oracle as O

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


def np_counts(table):
    """wins, ties, losses over (entry, rotation) pairs and invalid entries,
    from the 512 bits of each entry (u64 words 0-3 win, 4-7 not-lose)."""
    t = np.ascontiguousarray(table).view(np.uint64).reshape(-1, 8)
    w, n = t[:, :4], t[:, 4:]
    return [int(np.bitwise_count(w).sum()), int(np.bitwise_count(n & ~w).sum()),
            256 * len(t) - int(np.bitwise_count(n).sum()), int(((w & ~n) != 0).any(axis=1).sum())]


def gpu_counts(P, t):
    out = torch.zeros(4, dtype=torch.int64, device="cuda")
    P.pentago_table_counts(t, out)
    torch.cuda.synchronize()
    return [int(x) for x in out.cpu()]


def gpu_solve(P, counts, children):
    out = torch.empty((O.section_entries(counts), 8), dtype=torch.int64, device="cuda")
    P.pentago_solve_section(counts, children, out)
    torch.cuda.synchronize()
    return out


SMALL = [((8, 1), (1, 7), (4, 5), (5, 4)), ((9, 0), (0, 9), (4, 4), (5, 4)),
         ((8, 1), (1, 8), (5, 3), (4, 5))]


@pytest.mark.parametrize("counts", SMALL)
def test_counts_match_oracle_tables(P, counts):
    """Counts of the GPU table equal the counts of O4's table, taken in numpy
    (35-stone sections, 36-stone children on demand on both sides)."""
    log("section", counts)
    ref = O.section_solve(counts, [None] * 4)
    t = gpu_solve(P, counts, [None] * 4)
    want = np_counts(ref)
    got = gpu_counts(P, t)
    assert got == want
    assert sum(got[:3]) == 256 * O.section_entries(counts)
    assert got[3] == 0


def test_counts_of_the_headline_child_section(P):
    """The full-board child of the headline section: GPU counts equal numpy's
    over the whole GPU table, and W/T/L are all present."""
    counts = ((5, 4), (4, 5), (5, 4), (4, 5))
    t = gpu_solve(P, counts, [None] * 4)
    got = gpu_counts(P, t)
    assert got == np_counts(t.cpu().numpy())
    assert got[3] == 0 and min(got[:3]) > 0


def test_counts_invariant_under_board_symmetries(P):
    """A section's image under a board symmetry holds the same positions, so
    its table has the same counts (Section III: values are invariant under
    the board symmetries; the image table permutes entries and rotations)."""
    counts = ((6, 3), (3, 6), (5, 4), (4, 4))
    child = P.pentago_child_section(counts, 3)
    ct = gpu_solve(P, child, [None] * 4)
    t = gpu_solve(P, counts, [None, None, None, ct])
    base = gpu_counts(P, t)
    assert base[3] == 0
    for sym in range(1, 8):
        img = torch.empty_like(t)
        P.pentago_section_transform(counts, t, sym, img)
        torch.cuda.synchronize()
        assert gpu_counts(P, img) == base, sym


def test_empty_table(P):
    t = torch.empty((0, 8), dtype=torch.int64, device="cuda")
    assert gpu_counts(P, t) == [0, 0, 0, 0]
    P.pentago_validate_table(t)


def test_validate_rejects_win_outside_not_lose(P):
    counts = ((5, 4), (4, 5), (5, 4), (4, 5))
    t = gpu_solve(P, counts, [None] * 4)
    P.pentago_validate_table(t)
    bad = t.clone()
    bad[7, 0] = -1   # every win bit of u64 word 0 of entry 7
    bad[7, 4] = 0    # and no not-lose bit there
    with pytest.raises(P.PentagoError) as ei:
        P.pentago_validate_table(bad)
    assert ei.value.code == P.EINVAL
    assert gpu_counts(P, bad)[3] == 1


def test_validate_mode_checks_children(P):
    """With debug-validate mode on, a sweep given a child table with an
    invalid entry fails with EINVAL and launches nothing; a valid child
    passes and gives the same table as with the mode off."""
    counts = ((5, 4), (4, 5), (5, 4), (4, 4))
    child = P.pentago_child_section(counts, 3)
    ct = gpu_solve(P, child, [None] * 4)
    ref = gpu_solve(P, counts, [None, None, None, ct])
    bad = ct.clone()
    bad[123, 0] = -1   # every win bit of word pair 0
    bad[123, 4] = 0    # and no not-lose bit there
    out = torch.zeros_like(ref)
    P.pentago_set_validate(True)
    try:
        with pytest.raises(P.PentagoError) as ei:
            P.pentago_solve_section(counts, [None, None, None, bad], out)
        assert ei.value.code == P.EINVAL
        torch.cuda.synchronize()
        assert int(out.abs().sum()) == 0
        with pytest.raises(P.PentagoError):
            P.pentago_solve_sections([(counts, [None, None, None, bad], out)])
        P.pentago_solve_section(counts, [None, None, None, ct], out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    finally:
        P.pentago_set_validate(False)
    P.pentago_solve_section(counts, [None, None, None, bad], out)   # mode off: no check
    torch.cuda.synchronize()
