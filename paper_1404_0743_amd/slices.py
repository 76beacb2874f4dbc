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
    enqueued on `stream` as one batched launch."""
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


def prep_bound(counts):
    """An upper bound of the prepared-child scratch (bytes) a batched sweep of
    the section may allocate: 64 B per entry of every child table (the sweep
    prepares the children of the quadrants it does not stage)."""
    shape, _, _ = P.pentago_section_shape(counts)
    total = 0
    for j in range(4):
        if sum(counts[j]) < 9:
            cshape, _, _ = P.pentago_section_shape(P.pentago_child_section(counts, j))
            n = 1
            for i in range(4):
                n *= cshape[j] if i == j else shape[i]
            total += 64 * n
    return total


def stream_batches(stones, out_budget, prep_budget):
    """The D4-minimal sections of a slice split into batches (largest first,
    first fit) whose tables fit out_budget bytes and whose prepared-child
    scratch bound fits prep_budget bytes."""
    secs = sorted(P.pentago_slice_sections(stones), key=lambda s: -P.pentago_section_shape(s)[1])
    batches = []  # [sections, out bytes, prep bytes]
    for s in secs:
        out_b, prep_b = 64 * P.pentago_section_shape(s)[1], prep_bound(s)
        if out_b > out_budget or prep_b > prep_budget:
            raise ValueError("section %s does not fit the budgets" % (s,))
        for b in batches:
            if b[1] + out_b <= out_budget and b[2] + prep_b <= prep_budget:
                b[0].append(s)
                b[1] += out_b
                b[2] += prep_b
                break
        else:
            batches.append([[s], out_b, prep_b])
    return [b[0] for b in batches]


def solve_slice_streamed(stones, reps_above, sink, out_budget=64 << 30, prep_budget=96 << 30,
                         stream=None, events=None):
    """Every D4-minimal section of a slice whose tables do not fit in HBM
    together (slice 33: 337.8 GB), solved in batches through one arena of
    out_budget bytes: each batch is one batched launch
    (pentago_solve_sections_d4) whose tables are views of the arena; after
    it, sink(tables) is called (tables: counts -> device view, valid until
    sink returns; work sink enqueues on the stream is ordered before the next
    batch) and the arena is reused.  events: a list that receives a pair of
    timing events recorded around each batched launch.  Returns the number of
    batches."""
    batches = stream_batches(stones, out_budget, prep_budget)
    rows = max(sum(P.pentago_section_shape(s)[1] for s in b) for b in batches)
    arena = torch.empty((rows, 8), dtype=torch.int64, device="cuda")
    for secs in batches:
        jobs, tables, off = [], {}, 0
        for s in secs:
            entries = P.pentago_section_shape(s)[1]
            out = arena[off:off + entries]
            off += entries
            children = [None] * 4
            if stones < 35:
                for j in range(4):
                    if sum(s[j]) < 9:
                        rep, _ = P.pentago_section_standardize(P.pentago_child_section(s, j))
                        children[j] = reps_above[rep]
            jobs.append((s, children, out))
            tables[s] = out
        if events is not None:
            st = stream if stream is not None else torch.cuda.current_stream()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
            P.pentago_solve_sections_d4(jobs, stream)
            b.record(st)
            events.append((a, b))
        else:
            P.pentago_solve_sections_d4(jobs, stream)
        sink(tables)
    del arena
    return len(batches)
