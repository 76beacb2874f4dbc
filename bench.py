"""Benchmark of the n+1 -> n retrograde sweep on one MI355X.

Workload (one step): the sweep of the section whose quadrants hold
(black, white) = (5,4),(4,5),(5,4),(4,4), white to move: 6,288,640 entries,
1,260,236,880 positions, reading its 36-stone child section
(5,4),(4,5),(5,4),(4,5) (1,336,336 entries) which is materialised on the
GPU before the timed region.  Inputs are resident in HBM when timing starts.

Prints one JSON line: throughput in positions/s, the roofline of the sweep
kernel (algorithmic bytes over HIP-event time on the launch stream) and the
CPU oracle timed on a bounded sample of the same section.  The timed
launches' output is compared bit for bit with the oracle's tables of that
sample (``parity``); a mismatch exits with status 1.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra] [--extra a,b]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "positions/sec of n+1->n retrograde sweep (bit-exact) + p50/p99 query latency"
SECTION = ((5, 4), (4, 5), (5, 4), (4, 4))
CHILD = ((5, 4), (4, 5), (5, 4), (4, 5))
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    """What the host offers: logical CPUs, the CPUs this process may run on,
    the thread count the box grants (OMP_NUM_THREADS) and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = affinity
    if omp and omp.isdigit() and int(omp) > 0:
        threads = min(threads, int(omp))
    return {"nproc": os.cpu_count(), "affinity": affinity, "omp_num_threads": omp, "model": model,
            "threads": max(1, threads)}


def cpu_baseline(entries, positions, seconds_target=15.0):
    """The oracle (O4, per-entry plain retrograde) on a bounded random sample
    of the section's entries, on every host thread this process is granted,
    and on one thread; scaled to positions/s.  Returns the baseline record,
    the sampled blocked offsets and the oracle's tables for them (the
    parity check of the timed output reuses them)."""
    import oracle as O
    cpu = host_cpu()
    threads = cpu["threads"]
    rng = np.random.default_rng(12345)
    all_idx = O.section_all_indices(SECTION)
    pos_per_entry = positions / entries
    # one thread, ~3 s
    n1 = 512
    while True:
        offs1 = rng.choice(entries, n1, replace=False)
        t0 = time.perf_counter()
        O.section_solve(SECTION, [None] * 4, all_idx[offs1], nthreads=1)
        dt1 = time.perf_counter() - t0
        if dt1 > 1.5 or n1 >= 1 << 16:
            break
        n1 = int(n1 * min(8.0, max(2.0, 3.0 / max(dt1, 1e-3))))
    # all granted threads: calibrate, then size the sample to ~seconds_target
    n = 4096
    while True:
        offs = np.sort(rng.choice(entries, n, replace=False))
        t0 = time.perf_counter()
        want = O.section_solve(SECTION, [None] * 4, all_idx[offs], nthreads=threads)
        dt = time.perf_counter() - t0
        if dt > seconds_target / 4 or n >= 1 << 21:
            break
        n = int(n * min(8.0, max(2.0, seconds_target / max(dt, 1e-3))))
    rec = {"value": n * pos_per_entry / dt, "unit": "positions/s", "cores": threads,
           "kind": "oracle",
           "sample": "%d random entries of the section (%.0f positions), plain per-entry "
                     "retrograde on concrete boards, %d threads, %.1f s" % (n, n * pos_per_entry, threads, dt),
           "single_thread": {"value": n1 * pos_per_entry / dt1, "unit": "positions/s",
                             "sample": "%d random entries, 1 thread, %.1f s" % (n1, dt1)},
           "host": cpu}
    return rec, offs, want


def parity_sample(entries, n=4096):
    """Oracle tables of n random entries of the section (blocked offsets)."""
    import oracle as O
    rng = np.random.default_rng(54321)
    all_idx = O.section_all_indices(SECTION)
    offs = np.sort(rng.choice(entries, n, replace=False))
    return offs, O.section_solve(SECTION, [None] * 4, all_idx[offs], nthreads=host_cpu()["threads"])


VALU_PEAK = 256 * 4 * 2.4e9 / 4   # wave64 VALU instructions/s: 256 CUs x 4 SIMD16 at 2.4 GHz


def profile_counts(name):
    """A committed rocprofv3 counter summary (profiles/<name>.json), or None
    when any source it was taken on has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    h = hashlib.sha1()
    for src in d.get("sources", []):
        full = os.path.join(ROOT, src)
        if not os.path.exists(full):
            return None
        with open(full, "rb") as f:
            h.update(f.read())
    return d if h.hexdigest() == d.get("sources_sha1") else None


def measured_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, scaled by the copy-kernel calibration it records;
    None when the kernel sources have changed since the counters were taken."""
    d = profile_counts("sweep_kernel_section_36to35_traffic")
    return None if d is None else d.get("bytes_per_launch")


def roofline_valu(avg_ms):
    """The sweep's VALU issue rate against the chip's: wave64 VALU
    instructions per launch (committed counters, while the kernel sources
    are unchanged) over the live mean launch time."""
    d = profile_counts("sweep_kernel_section_36to35_valu")
    if d is None:
        return None
    achieved = d["valu_instr"] / (avg_ms * 1e-3)
    return {"bound": "alu", "achieved": achieved / 1e9, "peak": VALU_PEAK / 1e9,
            "unit": "G wave64 VALU instructions/s", "frac": achieved / VALU_PEAK,
            "instructions_per_launch": d["valu_instr"],
            "source": "profiles/sweep_kernel_section_36to35_valu.json"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (endgame batches, uneven layers)")
    ap.add_argument("--extra", default=None,
                    help="comma-separated subset of the other workloads to run (default: all)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 512 MiB fill and a 512 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: sharding the sweep over several GPUs "
              "is not implemented", file=sys.stderr)
        sys.exit(2)

    only = None
    if args.extra:
        import bench_extra
        only = set(args.extra.split(","))
        unknown = only - set(bench_extra.NAMES)
        if unknown:
            print("unknown workloads: %s (known: %s)" % (sorted(unknown), ", ".join(bench_extra.NAMES)),
                  file=sys.stderr)
            sys.exit(2)
    boards_2p20 = serve_queries = None
    if not args.no_extra and (only is None or only & {"endgame_2p20", "serving", "serving_resident"}):
        # generated before the GPU is touched (the generator forks workers)
        from paper_1404_0743_amd import inputs as I
        t0 = time.perf_counter()
        boards_2p20 = I.random_play_boards(1 << 20, 28, 33)
        serve_queries = I.random_play_boards(1 << 17, 26, 33, seed=I.SEED_SERVE)
        log("generated 2^20 endgame roots and 2^17 queries in %.1f s" % (time.perf_counter() - t0))

    import torch
    from paper_1404_0743_amd import pentago as P

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    shape, entries, positions = P.pentago_section_shape(SECTION)
    cshape, centries, _ = P.pentago_section_shape(CHILD)
    child = torch.empty((centries, 8), dtype=torch.int64, device="cuda")
    out = torch.empty((entries, 8), dtype=torch.int64, device="cuda")
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    P.pentago_solve_section(CHILD, [None] * 4, child, stream)  # first call: table upload
    # the full-board child section: tile shape tuned, then launches back to
    # back like the headline (one launch between two events would also count
    # the host's job set-up, which back-to-back launches hide)
    P.pentago_autotune_section(CHILD, [None] * 4, child, stream)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(args.steps):
        P.pentago_solve_section(CHILD, [None] * 4, child, stream)
    t1.record(stream)
    torch.cuda.synchronize()
    terminal_ms = t0.elapsed_time(t1) / args.steps
    children = [None, None, None, child]
    # tile shape picked by the library's autotuner (setup, not timed)
    tile, tune_ms = P.pentago_autotune_section(SECTION, children, out, stream)

    for _ in range(args.warmup):
        P.pentago_solve_section(SECTION, children, out, stream)
    torch.cuda.synchronize()

    # timed region: K launches back to back, HIP events on the launch stream
    # at its two ends (per-launch events would put bubbles between launches)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        P.pentago_solve_section(SECTION, children, out, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    avg_ms = ev0.elapsed_time(ev1) / args.steps
    # after the timed region: per-launch durations, for their spread
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for k in range(args.steps):
        starts[k].record(stream)
        P.pentago_solve_section(SECTION, children, out, stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    kernel_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    if args.copy_calibration:
        src = torch.ones(1 << 26, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ms_per_step = 1000.0 * wall / args.steps

    # algorithmic bytes of one sweep: every parent superinfo written once,
    # every child superinfo read once
    alg_bytes = 64 * entries + 64 * centries
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic()

    res = {
        "metric": METRIC,
        "value": positions / (ms_per_step * 1e-3),
        "unit": "positions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "single-section sweep 36->35: section (5,4),(4,5),(5,4),(4,4) "
                               "white to move, %d entries, %d positions, child section "
                               "(5,4),(4,5),(5,4),(4,5) %d entries resident" % (entries, positions, centries),
                   "entries": entries, "positions": positions, "shape": list(shape),
                   "tile_lines": tile["lines"], "tile_threads": tile["threads"], "tile_order": tile["order"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "roofline_valu": roofline_valu(avg_ms),
        "kernel_ms": {"sweep_avg": avg_ms, "sweep_min": float(np.min(kernel_ms)),
                      "sweep_median_single": float(np.median(kernel_ms)),
                      "terminal_child_section": terminal_ms},
    }
    # the timed launches' output, kept on the host for the parity check
    # against the oracle below (a 402 MB copy, after the timed region)
    out_host = out.cpu().numpy().view(np.uint64)
    if not args.no_extra:
        import bench_extra
        out_keep, child_keep = out, child
        resident = [(SECTION, out_keep), (CHILD, child_keep)]
        res["extra"] = bench_extra.run_all(P, torch, stream, boards_2p20, serve_queries, resident, only)
    if not args.no_cpu:
        log("timing the CPU oracle on a sample ...")
        res["cpu_baseline"], offs, want = cpu_baseline(entries, positions)
    else:
        offs, want = parity_sample(entries)
    # the timed launches' output against the oracle, bit for bit, on the
    # sampled entries (their blocked offsets)
    got = out_host[offs]
    bad = int((got != want).any(axis=1).sum())
    res["parity"] = {"entries_checked": int(len(offs)), "bit_exact": bad == 0, "mismatches": bad,
                     "oracle": "O4, plain per-entry retrograde on concrete boards, 36-stone children "
                               "evaluated directly"}
    print(json.dumps(res), flush=True)
    if bad:
        log("PARITY FAILURE: %d of %d sampled entries differ from the oracle" % (bad, len(offs)))
        sys.exit(1)


if __name__ == "__main__":
    main()
