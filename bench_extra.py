"""The workloads beside the headline sweep, timed on the GPU for bench.py.

  endgame_4096   4096 boards with 17 black and 16 white stones (3 empty
                 cells), solved to the full board: pentago_eval_batch.
  endgame_2p20   2^20 boards with 28..33 stones from random legal play:
                 one persistent launch (pentago_eval_batch) against one launch
                 per empties group (pentago_eval_batch_grouped).
  layers         64 sections per slice for slices 35, 34, 33 (sizes 1e4..2e8
                 positions, stratified by size), child chains solved first
                 (untimed): one batched launch per layer replayed from a
                 hipGraph against 64 per-section launches.
  serving        an open-loop Poisson stream of 2^17 queries with 26..33
                 stones (first 4096 dropped as warm-up) against the server
                 holding every section solved above resident; p50/p99 latency
                 and queries/s, against one query per launch.
  serving_resident
                 2^16 queries drawn from the resident sections (random
                 quadrant turns, then a random one of the 8 board
                 symmetries), answered by lookup: alone, and mixed one to one
                 with random-play queries under Poisson arrivals.
  slices         whole slices 35 and 34 (330 and 750 D4-minimal sections, 7.7
                 and 63 GB) over representatives: one batched launch, a
                 hipGraph replay, and one launch per section; then 2^15
                 positions of 34-35 stones answered by a server holding only
                 those representatives; then slice 33 (1,343 sections,
                 337.8 GB) from the slice-34 representatives, streamed
                 through a 64 GB arena in batches.
  deep           one position each of 22, 20 and 18 stones solved from scratch
                 (pentago_eval_deep: the DAG of 14, 16, 18 empty cells across
                 the GPU, layers in HBM).
  serving_deep   32 positions with 18..22 stones submitted at once to the
                 server, which runs them on the deep solver, three at a time.
  symmetry       the table transform under each of the 7 non-trivial board
                 symmetries of the 36->35 section (6,288,640 entries), and
                 sweeps whose child is held only as its D4 representative
                 (pentago_solve_section_d4) against the plain sweep.
Inputs are resident on the GPU when timing starts; times are HIP events on
the launch stream.
"""
import math
import sys
import time

import numpy as np

from paper_1404_0743_amd import inputs as I

# DAG nodes per root by number of empty cells e: sum over t of C(e,t) C(t, t//2)
NODES = [sum(math.comb(e, t) * math.comb(t, t // 2) for t in range(e + 1)) for e in range(11)]


def _parity_mask(p):
    """uint64[8] mask of the rotations g with g0 + g1 + g2 + g3 = p mod 2, for
    the win and the not-lose words (bit g in word g >> 6)."""
    words = [0, 0, 0, 0]
    for g in range(256):
        if ((g & 3) + ((g >> 2) & 3) + ((g >> 4) & 3) + (g >> 6)) % 2 == p:
            words[g >> 6] |= 1 << (g & 63)
    return np.array(words * 2, dtype=np.uint64)


PARITY0 = _parity_mask(0)


def bench_profile(name):
    import bench
    return bench.profile_counts(name)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _time(torch, stream, fn, reps):
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts)), float(np.min(ts))


def endgame(P, torch, stream, boards, grouped_too):
    codes = torch.from_numpy(P.boards_to_codes(boards).view(np.int16).copy()).cuda()
    out = torch.empty((len(boards), 8), dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    empt = (boards == 0).sum(axis=1)
    nodes = int(sum(NODES[e] for e in empt))
    res = {"roots": len(boards), "dag_nodes": nodes}
    if grouped_too:
        # the persistent form's workgroup sizes, tuned on these roots (set-up)
        threads, _ = P.pentago_autotune_eval(codes, out, stream)
        res["persistent_class_threads"] = list(threads)
    med, mn = _time(torch, stream, lambda: P.pentago_eval_batch(codes, out, status, stream), 5)
    res.update(persistent_ms=med, persistent_roots_per_s=len(boards) / (med * 1e-3),
               persistent_node_evals_per_s=nodes * 256 / (med * 1e-3))
    if grouped_too:
        ref = out.clone()
        med2, _ = _time(torch, stream, lambda: P.pentago_eval_batch(codes, out, status, stream, grouped=True), 5)
        res.update(grouped_ms=med2, grouped_roots_per_s=len(boards) / (med2 * 1e-3),
                   persistent_over_grouped=med2 / med, same_bytes=bool(torch.equal(ref, out)))
    res["invalid_boards"] = int(status.item())
    if grouped_too:
        # VALU issue of the persistent form: the class kernels' instructions
        # (committed counters, while their sources are unchanged) over its time
        import bench
        per = [bench.profile_counts("eval_persistent_kernel_class%d_2p20_roots_valu" % c) for c in range(3)]
        if all(p is not None for p in per):
            instr = sum(p["valu_instr"] for p in per)
            res["roofline_valu"] = {"bound": "alu", "achieved": instr / (med * 1e-3) / 1e9,
                                    "peak": bench.VALU_PEAK / 1e9, "unit": "G wave64 VALU instructions/s",
                                    "frac": instr / (med * 1e-3) / bench.VALU_PEAK,
                                    "per_class_frac": [p["valu_issue_frac"] for p in per]}
    return res


def layers(P, torch, stream, resident=None):
    """resident: a list that receives (counts, table) of every layer section
    and child section solved here (for the serving workload)."""
    out = {}
    cache = {}

    def solve_chain(counts):
        if counts in cache:
            return cache[counts]
        ch = [None] * 4
        if sum(b + w for b, w in counts) < 35:
            for j in range(4):
                if sum(counts[j]) < 9:
                    ch[j] = solve_chain(P.pentago_child_section(counts, j))
        _, entries, _ = P.pentago_section_shape(counts)
        t = torch.empty((entries, 8), dtype=torch.int64, device="cuda")
        P.pentago_solve_section(counts, ch, t, stream)
        cache[counts] = t
        return t

    for stones in (35, 34, 33):
        secs = I.pick_layer_sections(stones)
        jobs = []
        positions = 0
        for s in secs:
            ch = [None] * 4
            if stones < 35:
                for j in range(4):
                    if sum(s[j]) < 9:
                        ch[j] = solve_chain(P.pentago_child_section(s, j))
            _, entries, pos = P.pentago_section_shape(s)
            positions += pos
            jobs.append((s, ch, torch.empty((entries, 8), dtype=torch.int64, device="cuda")))
        torch.cuda.synchronize()

        def plain():
            for s, ch, o in jobs:
                P.pentago_solve_section(s, ch, o, stream)

        med_plain, _ = _time(torch, stream, plain, 5)
        ref = [o.clone() for _, _, o in jobs]
        # the batched sweep's tile shape (threads, LDS cap), tuned on this layer (set-up)
        cap, nt, _ = P.pentago_autotune_sections(jobs, stream=stream)
        plan = P.SweepPlan(jobs)
        med_graph, _ = _time(torch, stream, lambda: plan.launch(stream, graph=True), 5)
        same = all(torch.equal(r, o) for r, (_, _, o) in zip(ref, jobs))
        info = plan.info()
        plan.close()
        if resident is not None:
            resident.extend((s, o) for s, _, o in jobs)
        sizes = [I.section_positions(s) for s in secs]
        out["slice%d" % stones] = {
            "sections": len(secs), "positions": positions,
            "min_positions": min(sizes), "max_positions": max(sizes),
            "plain_ms": med_plain, "plain_positions_per_s": positions / (med_plain * 1e-3),
            "batched_graph_ms": med_graph, "batched_positions_per_s": positions / (med_graph * 1e-3),
            "batched_over_plain": med_plain / med_graph, "same_bytes": same,
            "tiles": info["tiles"], "grid": info["grid"], "tile_lds_cap": cap, "tile_threads": nt,
            "counts": table_counts(P, torch, [o for _, _, o in jobs], stream)}
        log("layer %d: plain %.3f ms, batched %.3f ms" % (stones, med_plain, med_graph))
    out["resident_child_bytes"] = sum(t.numel() * 8 for t in cache.values())
    if resident is not None:
        resident.extend(cache.items())
    return out


def sustained_capacity(srv, codes, seed):
    """The highest Poisson arrival rate the server keeps up with: bisection
    between 0 and the all-at-once throughput, each probe a replay of 2^14
    queries, "keeps up" meaning at least 97 % of the offered rate served."""
    n = min(len(codes), 1 << 14)
    t0 = time.perf_counter()
    srv.replay(codes[:n], np.zeros(n))
    hi = n / (time.perf_counter() - t0)
    lo = 0.0
    for it in range(7):
        r = hi if it == 0 else 0.5 * (lo + hi)
        arr = I.poisson_arrivals(n, r, seed=seed + it)
        srv.reset_stats()
        srv.replay(codes[:n], arr)
        served = srv.stats()["queries_per_s"]
        if served >= 0.97 * r:
            lo = r
            if it == 0:
                break
        else:
            hi = r
    return max(lo, 1.0)


def serving(P, torch, stream, resident, queries):
    """Open-loop Poisson stream of position queries (26..33 stones) against a
    server holding the given resident sections.  The rate is 0.7 of the
    sustained capacity measured first on the same queries.  The plain form
    answers a sample of the stream one query per launch."""
    codes = P.boards_to_codes(queries)
    srv = P.Server(memory_budget=4 << 30, max_inflight=1 << 20, max_batch=4096, streams=8)
    for counts, table in resident:
        srv.add_section(counts, table)
    warm = 4096
    cap = sustained_capacity(srv, codes, I.SEED_SERVE + 10)
    rate = 0.7 * cap
    arrivals = I.poisson_arrivals(len(codes), rate)
    srv.reset_stats()
    srv.replay(codes[:warm], arrivals[:warm])
    srv.reset_stats()
    res = srv.replay(codes[warm:], arrivals[warm:] - arrivals[warm])
    st = srv.stats()
    srv.close()
    # plain form: one query per launch, on a sample of the stream
    sample = codes[warm:warm + 2048]
    dev = torch.from_numpy(sample.view(np.int16).copy()).cuda()
    out = torch.empty((len(sample), 8), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(len(sample)):
        P.pentago_eval_batch(dev[i:i + 1], out[i:i + 1], None, stream)
        torch.cuda.synchronize()
    plain_qps = len(sample) / (time.perf_counter() - t0)
    # per-launch answers equal the served ones (searches; lookups are not in the sample's kind mix check)
    served = res[:len(sample)]
    empt = (queries[warm:warm + len(sample)] == 0).sum(axis=1)
    same = bool(np.array_equal(out.cpu().numpy().view(np.uint64)[empt <= 10], served[empt <= 10]))
    return {"queries": int(st["queries"]), "lookups": int(st["lookups"]), "searches": int(st["searches"]),
            "batches": int(st["batches"]), "sustained_capacity_per_s": cap, "offered_rate_per_s": rate,
            "p50_us": st["p50_us"], "p99_us": st["p99_us"], "queries_per_s": st["queries_per_s"],
            "plain_one_query_per_launch_per_s": plain_qps, "served_over_plain": st["queries_per_s"] / plain_qps,
            "plain_answers_equal_served": same, "warmup_dropped": warm}


def serving_resident(P, torch, stream, resident, queries):
    """Queries drawn from the resident sections (uniform section, uniform
    entry, every quadrant turned at random, the board under a random board
    symmetry) answered by table lookup: alone
    at full speed, and mixed one to one with the random-play stream under
    Poisson arrivals at 0.7 of the mix's sustained capacity."""
    shapes = [P.pentago_section_shape(c)[0] for c, _ in resident]
    n = 1 << 16
    sec, idx = I.resident_entries(shapes, n, seed=I.SEED_SERVE + 2)
    codes = np.array([P.pentago_section_board(resident[s][0], i) for s, i in zip(sec, idx)], np.uint16)
    # every quadrant turned at random, then every board under a random board
    # symmetry: the images of the resident sections are answered from them
    looked = P.boards_to_codes(I.board_symmetries(I.turn_quadrants(I.codes_to_boards(codes), seed=I.SEED_SERVE + 3),
                                                  seed=I.SEED_SERVE + 5))
    srv = P.Server(memory_budget=4 << 30, max_inflight=1 << 20, max_batch=4096, streams=8)
    for counts, table in resident:
        srv.add_section(counts, table)
    out = {}
    # lookups alone, everything arriving at once
    srv.replay(looked[:4096], np.zeros(4096))
    srv.reset_stats()
    t0 = time.perf_counter()
    got = srv.replay(looked, np.zeros(n))
    dt = time.perf_counter() - t0
    st = srv.stats()
    # the same boards solved by the endgame search (resident sections have
    # at most 3 empty cells): the lookups must give the same bytes
    dev = torch.from_numpy(looked.view(np.int16).copy()).cuda()
    ref = torch.empty((n, 8), dtype=torch.int64, device="cuda")
    P.pentago_eval_batch(dev, ref, None, stream)
    torch.cuda.synchronize()
    same = bool(np.array_equal(ref.cpu().numpy().view(np.uint64), got))
    out["lookup_only"] = {"queries": int(st["queries"]), "lookups": int(st["lookups"]),
                          "queries_per_s": n / dt, "p50_us": st["p50_us"], "p99_us": st["p99_us"],
                          "answers_equal_search": same}
    # one to one with random-play queries
    rp = P.boards_to_codes(queries[:n])
    mix = np.empty((2 * n, 4), np.uint16)
    mix[0::2] = looked
    mix[1::2] = rp
    cap = sustained_capacity(srv, mix, I.SEED_SERVE + 20)
    arrivals = I.poisson_arrivals(len(mix), 0.7 * cap, seed=I.SEED_SERVE + 4)
    srv.reset_stats()
    srv.replay(mix, arrivals)
    st = srv.stats()
    srv.close()
    out["mixed"] = {"queries": int(st["queries"]), "lookups": int(st["lookups"]), "searches": int(st["searches"]),
                    "sustained_capacity_per_s": cap, "offered_rate_per_s": 0.7 * cap,
                    "p50_us": st["p50_us"], "p99_us": st["p99_us"], "queries_per_s": st["queries_per_s"],
                    "lookup_p50_us": st["lookup_p50_us"], "lookup_p99_us": st["lookup_p99_us"],
                    "search_p50_us": st["search_p50_us"], "search_p99_us": st["search_p99_us"]}
    return out


def symmetry(P, torch, stream, resident):
    """Transform of the resident 36->35 section under each board symmetry
    (algorithmic bytes: 64 B read + 64 B written per entry), and sweeps over
    representatives against plain sweeps of the same sections."""
    src_counts, src = resident[0]
    n = src.shape[0]
    out = torch.empty_like(src)
    res = {"section": str(src_counts), "entries": n, "transform": {}}
    for sym in range(1, 8):
        med, mn = _time(torch, stream, lambda: P.pentago_section_transform(src_counts, src, sym, out, stream), 10)
        gbs = 128 * n / (med * 1e-3) / 1e9
        res["transform"][str(sym)] = {"ms": med, "min_ms": mn, "GB_s": gbs, "frac_hbm": gbs / 8000.0}
    fr = [v["frac_hbm"] for v in res["transform"].values()]
    res["transform_frac_hbm_mean"] = float(np.mean(fr))
    del out
    res["sweep_d4"] = []
    for counts in (((5, 4), (4, 5), (5, 4), (4, 4)), ((4, 4), (4, 5), (6, 3), (4, 5))):
        j = [k for k in range(4) if sum(counts[k]) < 9][0]
        child = P.pentago_child_section(counts, j)
        rep, sym = P.pentago_section_standardize(child)
        _, ce, _ = P.pentago_section_shape(child)
        _, e, pos = P.pentago_section_shape(counts)
        ct = torch.empty((ce, 8), dtype=torch.int64, device="cuda")
        rt = torch.empty((ce, 8), dtype=torch.int64, device="cuda")
        P.pentago_solve_section(child, [None] * 4, ct, stream)
        P.pentago_solve_section(rep, [None] * 4, rt, stream)
        kids, reps = [None] * 4, [None] * 4
        kids[j], reps[j] = ct, rt
        a = torch.empty((e, 8), dtype=torch.int64, device="cuda")
        b = torch.empty((e, 8), dtype=torch.int64, device="cuda")
        P.pentago_autotune_section(counts, kids, a, stream)
        t_plain, _ = _time(torch, stream, lambda: P.pentago_solve_section(counts, kids, a, stream), 10)
        t_d4, _ = _time(torch, stream, lambda: P.pentago_solve_section_d4(counts, reps, b, stream), 10)
        res["sweep_d4"].append({"section": str(counts), "child": str(child), "child_rep": str(rep),
                                "child_sym": sym, "positions": pos, "plain_ms": t_plain, "d4_ms": t_d4,
                                "d4_positions_per_s": pos / (t_d4 * 1e-3), "bit_exact": bool(torch.equal(a, b))})
        del a, b, ct, rt
    torch.cuda.empty_cache()
    return res


NAMES = ("endgame_4096", "endgame_2p20", "layers", "serving", "serving_resident", "symmetry", "slices",
         "deep", "serving_deep")


def table_counts(P, torch, tables, stream, acc=None):
    """The per-slice checksum of Section VII: wins, ties and losses over
    every (entry, rotation) pair of the tables (each entry holds 256
    rotations of one board), and the entries whose win set is not inside
    their not-lose set (none in a solved table).  acc: a device tensor of 4
    int64 to add to (stream-ordered), else the totals are returned."""
    own = acc is None
    if own:
        acc = torch.zeros(4, dtype=torch.int64, device="cuda")
    out = torch.empty(4, dtype=torch.int64, device="cuda")
    for t in tables:
        P.pentago_table_counts(t, out, stream)
        acc += out
    if not own:
        return None
    torch.cuda.synchronize()
    w, ti, lo, bad = (int(x) for x in acc.cpu())
    return {"win": w, "tie": ti, "loss": lo, "invalid_entries": bad}


def slices(P, torch, stream):
    """Whole slices 35 and 34 over D4 representatives: every D4-minimal
    section of the slice, children read from the representatives of the
    slice above (slice 35: the 36-stone boards on demand).  One batched
    launch, the same replayed from a hipGraph, and one launch per section;
    all three must leave the same tables."""
    from paper_1404_0743_amd import slices as S
    res = {}
    above = None
    for stones in (35, 34):
        jobs, tables = S.slice_jobs(stones, above)
        entries = sum(t.shape[0] for t in tables.values())
        reads = 0
        for counts, children, _ in jobs:
            reads += sum(c.shape[0] for c in children if c is not None)
        alg = 64 * entries + 64 * reads
        cap, nt, _ = P.pentago_autotune_sections(jobs, reps=True, stream=stream)   # set-up
        t_batched, _ = _time(torch, stream, lambda: P.pentago_solve_sections_d4(jobs, stream), 5)
        keep = {k: v.clone() for k, v in sorted(tables.items(), key=lambda kv: -kv[1].shape[0])[:8]}
        w = torch.randint(-(1 << 62), 1 << 62, (8,), dtype=torch.int64, device="cuda")
        check = lambda: [int((t * w).sum()) for t in tables.values()]
        sums = check()
        plan = P.SweepPlan(jobs, reps=True)
        t_graph, _ = _time(torch, stream, lambda: plan.launch(stream, graph=True), 5)
        same = check() == sums and all(torch.equal(tables[k], v) for k, v in keep.items())
        plan.close()

        def per_section():
            for counts, children, out in jobs:
                P.pentago_solve_section_d4(counts, children, out, stream)
        t_plain, _ = _time(torch, stream, per_section, 3)
        same = same and check() == sums and all(torch.equal(tables[k], v) for k, v in keep.items())
        pos = S.slice_positions(stones)
        cover = S.slice_positions(stones, minimal_only=False)
        res["slice%d" % stones] = {
            "sections": len(jobs), "entries": entries, "bytes_written": 64 * entries,
            "positions": pos, "positions_all_images": cover,
            "batched_ms": t_batched, "graph_ms": t_graph, "per_section_ms": t_plain,
            "graph_positions_per_s": pos / (t_graph * 1e-3),
            "graph_positions_all_images_per_s": cover / (t_graph * 1e-3),
            "graph_algorithmic_GB_s": alg / (t_graph * 1e-3) / 1e9,
            "graph_over_per_section": t_plain / t_graph, "same_bytes": bool(same), "tile_lds_cap": cap, "tile_threads": nt,
            "counts": table_counts(P, torch, tables.values(), stream)}
        del keep
        if stones == 34:
            # a server holding only the representatives of both slices answers
            # every 34- and 35-stone position by lookup through a symmetry
            boards = I.random_play_boards(1 << 15, 34, 35, seed=I.SEED_SERVE + 70)
            codes = P.boards_to_codes(boards)
            srv = P.Server(memory_budget=1 << 30, max_inflight=1 << 16, max_batch=4096, streams=4)
            for tabs in (above, tables):
                for counts, t in tabs.items():
                    srv.add_section(counts, t)
            srv.replay(codes[:1024], np.zeros(1024))
            srv.reset_stats()
            t0 = time.perf_counter()
            got = srv.replay(codes, np.zeros(len(codes)))
            dt = time.perf_counter() - t0
            st = srv.stats()
            srv.close()
            dev = torch.from_numpy(codes[:4096].view(np.int16).copy()).cuda()
            ref = torch.empty((4096, 8), dtype=torch.int64, device="cuda")
            P.pentago_eval_batch(dev, ref, None, stream)
            torch.cuda.synchronize()
            res["lookups_from_slices"] = {
                "resident_sections": len(above) + len(tables), "queries": int(st["queries"]),
                "lookups": int(st["lookups"]), "queries_per_s": len(codes) / dt,
                "p50_us": st["p50_us"], "p99_us": st["p99_us"],
                "answers_equal_search": bool(np.array_equal(ref.cpu().numpy().view(np.uint64), got[:4096]))}
        above = tables
    # slice 33 (1,343 sections, 337.8 GB of tables: more than the GPU holds
    # next to slice 34) from the slice-34 representatives, streamed through
    # one 64 GB arena in batches; the time counts the batched launches only
    # (HIP events around each), not the per-batch counts of the sink
    evs = []
    acc33 = torch.zeros(4, dtype=torch.int64, device="cuda")

    def sink(tables):
        table_counts(P, torch, tables.values(), stream, acc33)

    t0 = time.perf_counter()
    nb = S.solve_slice_streamed(33, above, sink, stream=stream, events=evs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = sum(a.elapsed_time(b) for a, b in evs)
    secs = P.pentago_slice_sections(33)
    entries = sum(P.pentago_section_shape(s)[1] for s in secs)
    reads = 0
    for s in secs:
        for j in range(4):
            if sum(s[j]) < 9:
                rep, _ = P.pentago_section_standardize(P.pentago_child_section(s, j))
                reads += P.pentago_section_shape(rep)[1]
    pos = S.slice_positions(33)
    res["slice33_streamed"] = {
        "sections": len(secs), "entries": entries, "bytes_written": 64 * entries, "batches": nb,
        "arena_bytes": 64 << 30, "gpu_ms": gpu_ms, "wall_s": wall,
        "positions": pos, "positions_per_s": pos / (gpu_ms * 1e-3),
        "algorithmic_GB_s": 64 * (entries + reads) / (gpu_ms * 1e-3) / 1e9,
        "counts": dict(zip(("win", "tie", "loss", "invalid_entries"), (int(x) for x in acc33.cpu())))}
    log("slice 33 streamed: %d batches, %.1f ms GPU, %.1f s wall" % (nb, gpu_ms, wall))
    del above
    torch.cuda.empty_cache()
    return res


def deep(P, torch, stream):
    """One position of 22, 20 and 18 stones (14, 16, 18 empty cells) from
    random legal play, each solved from scratch by pentago_eval_deep.
    Algorithmic bytes: 64 B read per (node, child) edge + 64 B written per
    node below the root; half of that for the parity-halved form (32 B
    records, the rotations of the board's own parity only)."""
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    res = {}
    for stones in (22, 20, 18):
        b = I.random_play_boards(1, stones, stones, seed=I.SEED_SERVE + 50 + stones)[0]
        codes = P.boards_to_codes(b.reshape(1, 36))[0]
        e = 36 - stones
        nodes = [math.comb(e, t) * math.comb(t, (t + 1) // 2) for t in range(e + 1)]
        alg = 64 * sum(n * (e - t) for t, n in enumerate(nodes)) + 64 * sum(nodes[1:])
        med, mn = _time(torch, stream, lambda: P.pentago_eval_deep(codes, out, stream), 5)
        # the same root through the batched solver's layout limit: not
        # comparable beyond 10 empty cells, so the check is the recurrence and
        # symmetry tests; here the result must be stable across launches
        first = out.clone()
        P.pentago_eval_deep(codes, out, stream)
        torch.cuda.synchronize()
        # the parity-halved form (32 B records) for the board's own parity
        # (g = 0): half the algorithmic bytes; its bits equal the full table's
        half = torch.zeros(8, dtype=torch.int64, device="cuda")
        hmed, hmn = _time(torch, stream, lambda: P.pentago_eval_deep_parity(codes, 0, half, stream), 5)
        torch.cuda.synchronize()
        hw = half.cpu().numpy().view(np.uint64)
        fw = out.cpu().numpy().view(np.uint64)
        # floor bytes: every node's record written once and read once
        floor = 2 * 64 * sum(nodes)
        prof = bench_profile("deep_node_kernel_valu")
        res["empty%d" % e] = {"stones": stones, "dag_nodes": sum(nodes), "ms": med, "min_ms": mn,
                              "valu_issue_frac_profiled": None if prof is None else
                              {"full": prof["deep_node_kernel<false>"]["valu_issue_frac"],
                               "parity_half": prof["deep_node_kernel<true>"]["valu_issue_frac"]},
                              "nodes_per_s": sum(nodes) / (med * 1e-3),
                              # 64 B per (node, child) edge read + 64 B per node
                              # written: L2 serves part of the edge reads, so
                              # this is not an HBM fraction
                              "algorithmic_GB_s": alg / (med * 1e-3) / 1e9,
                              "algorithmic_frac": alg / (med * 1e-3) / 8e12,
                              "floor_GB_s": floor / (med * 1e-3) / 1e9,
                              "floor_frac_hbm": floor / (med * 1e-3) / 8e12,
                              "repeatable": bool(torch.equal(first, out)),
                              "parity_half_ms": hmed, "parity_half_min_ms": hmn,
                              "parity_half_algorithmic_GB_s": alg / 2 / (hmed * 1e-3) / 1e9,
                              "parity_half_floor_frac_hbm": floor / 2 / (hmed * 1e-3) / 8e12,
                              "parity_half_equals_full_masked": bool(np.array_equal(hw, fw & PARITY0)),
                              "parity_half_bits": int(sum(bin(int(x)).count("1") for x in hw))}
    return res


def serving_deep(P, torch, stream):
    """Deep queries through the server: 32 positions with 18..22 stones (14
    to 18 empty cells) from random legal play, all submitted at once; the
    server runs them on the deep solver, one per search stream (3).  Latency p50/p99
    from submission; a sample of answers against the deep solver called
    directly."""
    boards = I.random_play_boards(32, 18, 22, seed=I.SEED_SERVE + 60)
    codes = P.boards_to_codes(boards)
    srv = P.Server(memory_budget=8 << 30, max_inflight=1024, max_batch=64, streams=4)
    srv.replay(codes[:2], np.zeros(2))
    srv.reset_stats()
    t0 = time.perf_counter()
    got = srv.replay(codes, np.zeros(len(codes)))
    dt = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    same = True
    for k in range(0, len(codes), 8):
        P.pentago_eval_deep(codes[k], out, stream)
        torch.cuda.synchronize()
        same = same and bool(np.array_equal(out.cpu().numpy().view(np.uint64), got[k]))
    empties = 36 - (boards != 0).sum(axis=1)
    return {"queries": int(st["queries"]), "searches": int(st["searches"]),
            "empty_cells": [int(empties.min()), int(empties.max())], "queries_per_s": len(codes) / dt,
            "p50_us": st["p50_us"], "p99_us": st["p99_us"], "answers_equal_deep_solver": same}


def run_all(P, torch, stream, boards_2p20=None, serve_queries=None, resident=None, only=None):
    res = {}
    for name, fn in (("endgame_4096", lambda: endgame(P, torch, stream, I.random_placement_boards(4096, 17, 16), False)),
                     ("endgame_2p20", lambda: endgame(P, torch, stream, boards_2p20, True)),
                     ("layers", lambda: layers(P, torch, stream, resident)),
                     ("serving", lambda: serving(P, torch, stream, resident, serve_queries)),
                     ("serving_resident", lambda: serving_resident(P, torch, stream, resident, serve_queries)),
                     ("symmetry", lambda: symmetry(P, torch, stream, resident)),
                     ("slices", lambda: slices(P, torch, stream)),
                     ("deep", lambda: deep(P, torch, stream)),
                     ("serving_deep", lambda: serving_deep(P, torch, stream))):
        if only is not None and name not in only:
            continue
        if name == "endgame_2p20" and boards_2p20 is None:
            continue
        if name in ("serving", "serving_resident") and serve_queries is None:
            continue
        t0 = time.perf_counter()
        try:
            res[name] = fn()
        except Exception as e:  # report, keep the headline line alive
            res[name] = {"error": repr(e)}
        log("%s done in %.1f s" % (name, time.perf_counter() - t0))
    return res
