"""Whole-slice sweeps over D4 representatives (Section IV: a slice is every
board with one number of stones; only the sections whose counts are least
under the board symmetries are computed, and every other section is an image
of one of them).

Each slice is one batched call (pentago_solve_sections_d4): every
D4-minimal section of the slice, its children read from the representatives
of the slice above through their symmetries.  Tables are device tensors
(entries x 8 int64 = 64 B per entry) owned by the caller's dictionaries.
"""
import torch

from . import pentago as P


def slice_jobs(stones, reps_above):
    """(jobs, tables) for the D4-minimal sections of a slice: tables maps
    counts -> a new device table, jobs are (counts, children, out) with each
    child the representative's table from reps_above (counts -> table of the
    slice with stones + 1 stones); for 35 stones the 36-stone children are
    evaluated on demand and reps_above may be None."""
    jobs, tables = [], {}
    for s in P.pentago_slice_sections(stones):
        _, entries, _ = P.pentago_section_shape(s)
        out = torch.empty((entries, 8), dtype=torch.int64, device="cuda")
        children = [None] * 4
        if stones < 35:
            for j in range(4):
                if sum(s[j]) < 9:
                    rep, _ = P.pentago_section_standardize(P.pentago_child_section(s, j))
                    children[j] = reps_above[rep]
        jobs.append((s, children, out))
        tables[s] = out
    return jobs, tables


def solve_slice(stones, reps_above=None, stream=None):
    """Tables of every D4-minimal section of the slice (dict counts -> table),
    enqueued on `stream` as one persistent launch."""
    if not 0 <= stones <= 35:
        raise ValueError("slices of 0..35 stones (36-stone boards are evaluated on demand)")
    jobs, tables = slice_jobs(stones, reps_above)
    P.pentago_solve_sections_d4(jobs, stream)
    return tables


def slice_positions(stones, minimal_only=True):
    """Boards in the slice's D4-minimal sections, or (minimal_only=False) in
    all its sections: each minimal section stands for its distinct images."""
    total = 0
    for s in P.pentago_slice_sections(stones):
        pos = P.pentago_section_shape(s)[2]
        total += pos * (1 if minimal_only else len({P.pentago_section_image(s, d) for d in range(8)}))
    return total
