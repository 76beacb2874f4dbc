// batch.hip -- many sections of one slice in one launch (the whole layer's
// block lines as one grid of tiles: within a slice the block lines are
// independent and may be computed in any order, Section IV-A), plus the sweep
// plan that keeps the layer's job table resident and replays it from a
// hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "internal.h"

using namespace pg;

struct pentago_sweep_plan {
    int device = 0;
    int njobs = 0, nunits = 0;
    long long total_tiles = 0, total_chunks = 0;
    int lds_bytes = 0;
    int threads = 512;  // per tile workgroup
    // jobs [0, nbig) have tiles above the LDS cap even with one line;
    // they take a second launch, beside the first on a side stream
    int nbig = 0;
    long long tiles_big = 0;
    int lds_big = 0;
    char *dev = nullptr;  // one device block: jobs, tile starts, units, chunk starts, prep
    SweepJob *d_jobs = nullptr;
    long long *d_tile_start = nullptr;
    int *d_unit = nullptr;
    long long *d_chunk_start = nullptr;
    bool async_alloc = false;
    bool sym = false;  // children held as their representatives
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    DevTables T;
};

namespace pg {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Tile shape of a batch unless pentago_autotune_sections has picked one
// for the layer's stone count: an LDS bound per tile of 52 KiB (three
// workgroups per CU, the headline tile shape, 7 lines of 160 patterns,
// included) and 512 threads per tile.
struct BatchShape {
    int cap, threads;
};
constexpr BatchShape kBatchDefault = {53248, 512};
// Caps and workgroup sizes the autotuner tries (at most three 512-thread
// workgroups run per CU, so larger caps only cost occupancy; 256 threads
// suit layers of short lines, whose small tiles leave most of 512 threads
// idle).
constexpr int kBatchCaps[] = {24576, 32768, 40960, 53248};
constexpr int kBatchThreadChoices[] = {256, 512};

static std::mutex g_shape_mutex;
static BatchShape g_shape[37];   // per stone count; cap 0: kBatchDefault

static BatchShape batch_shape(int stones)
{
    std::lock_guard<std::mutex> lock(g_shape_mutex);
    const BatchShape b = stones >= 0 && stones <= 36 ? g_shape[stones] : BatchShape{0, 0};
    return b.cap > 0 ? b : kBatchDefault;
}

// Build a plan: job table in decreasing order of work, prep units for the
// dimensions that are not staged, and the device block holding all of it.
// With `stream` the device block is allocated stream-ordered on it.
static int plan_build(const pentago_section_job *jobs, size_t n, hipStream_t stream, bool async,
                      bool reps, pentago_sweep_plan **out, BatchShape shape = {0, 0})
{
    if (!jobs || n == 0) return fail(PENTAGO_EINVAL, "no jobs");
    if (n > 65536) return fail(PENTAGO_ERANGE, "more than 65536 jobs");
    const int stones = section_stones(jobs[0].section);
    if (shape.cap <= 0) shape = batch_shape(stones);
    const int lds_cap = shape.cap;
    std::vector<SweepJob> J(n);
    for (size_t i = 0; i < n; i++) {
        if (section_stones(jobs[i].section) != stones)
            return fail(PENTAGO_EINVAL, "jobs of one call must share the stone count");
        int rc = make_job(jobs[i].section, jobs[i].child, jobs[i].out, &J[i], -1, 0);
        if (rc) return rc;
        // in a batch, stage the quadrant with the longest lines (the most
        // patterns; ties: the larger child class): short lines pay the
        // per-line table set-up over few parents, and the children of the
        // other quadrants go through the one batched prep launch anyway
        int dl = -1;
        for (int j = 0; j < 4; j++)
            if (((J[i].emask >> j) & 1) &&
                (dl < 0 || J[i].m[j] > J[i].m[dl] || (J[i].m[j] == J[i].m[dl] && J[i].cm[j] > J[i].cm[dl])))
                dl = j;
        if (dl >= 0 && dl != J[i].d) {
            rc = make_job(jobs[i].section, jobs[i].child, jobs[i].out, &J[i], dl, 0);
            if (rc) return rc;
        }
        // a launch's occupancy follows its largest tile's LDS: keep every
        // tile within the cap by taking fewer lines per tile
        if (J[i].lds_bytes > lds_cap && J[i].G > 1) {
            int G = J[i].G;
            const int cmd = (J[i].emask >> J[i].d) & 1 ? J[i].cm[J[i].d] : 0;
            while (G > 1 && sweep_lds_bytes(G, J[i].m[J[i].d], cmd) > lds_cap) G--;
            rc = make_job(jobs[i].section, jobs[i].child, jobs[i].out, &J[i], J[i].d, G);
            if (rc) return rc;
        }
        if (reps) set_child_syms(jobs[i].section, jobs[i].child, &J[i]);
        rc = validate_children(J[i], stream);
        if (rc) return rc;
    }
    // jobs whose tiles need more than the cap even with one line (long
    // lines of large classes) go first and to their own launch, so that their
    // LDS does not set the occupancy of every other tile; within each group,
    // largest sections first: their tiles start early and small ones fill the
    // tail
    std::vector<size_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    auto work = [&](size_t i) { return (double)J[i].m[0] * J[i].m[1] * J[i].m[2] * J[i].m[3]; };
    auto big = [&](size_t i) { return J[i].lds_bytes > lds_cap; };
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        if (big(a) != big(b)) return big(a);
        return work(a) > work(b);
    });
    std::vector<SweepJob> S(n);
    int nbig = 0;
    for (size_t i = 0; i < n; i++) {
        S[i] = J[order[i]];
        nbig += big(order[i]) ? 1 : 0;
    }

    // tile numbers start at 0 in each group
    std::vector<long long> tile_start(n);
    long long tiles = 0, tiles_big = 0;
    int lds = 0, lds_big = 0;
    for (size_t i = 0; i < n; i++) {
        if ((int)i == nbig) {
            tiles_big = tiles;
            tiles = 0;
        }
        tile_start[i] = tiles;
        tiles += S[i].ntiles;
        if ((int)i < nbig) lds_big = std::max(lds_big, S[i].lds_bytes);
        else lds = std::max(lds, S[i].lds_bytes);
    }
    if (nbig == (int)n) {
        tiles_big = tiles;
        tiles = 0;
    }
    if (tiles > 0x7fffffffLL || tiles_big > 0x7fffffffLL)
        return fail(PENTAGO_ERANGE, "more than 2^31 - 1 tiles in one launch");
    std::vector<int> unit;
    std::vector<long long> chunk_start;
    std::vector<size_t> prep_off;
    size_t prep_total = 0;
    long long chunks = 0;
    for (size_t i = 0; i < n; i++)
        for (int j = 0; j < 4; j++) {
            if (j == S[i].d || !((S[i].emask >> j) & 1)) continue;
            unit.push_back((int)(i << 2) | j);
            chunk_start.push_back(chunks);
            const size_t bytes = prep_bytes(S[i], j);
            chunks += (long long)((bytes / 64 + 255) / 256);
            prep_off.push_back(prep_total);
            prep_total += align256(bytes);
        }

    pentago_sweep_plan *P = new pentago_sweep_plan;
    (void)hipGetDevice(&P->device);
    int rc = device_tables(&P->T);
    if (rc) { delete P; return rc; }
    P->njobs = (int)n;
    P->nunits = (int)unit.size();
    P->total_tiles = tiles;
    P->total_chunks = chunks;
    P->lds_bytes = lds;
    P->threads = shape.threads;
    P->nbig = nbig;
    P->tiles_big = tiles_big;
    P->lds_big = lds_big;
    P->async_alloc = async;
    P->sym = reps;

    const size_t o_jobs = 0;
    const size_t o_tiles = align256(o_jobs + n * sizeof(SweepJob));
    const size_t o_unit = align256(o_tiles + n * sizeof(long long));
    const size_t o_chunk = align256(o_unit + unit.size() * sizeof(int) + 4);
    const size_t o_prep = align256(o_chunk + chunk_start.size() * sizeof(long long) + 8);
    const size_t total = o_prep + prep_total;
    hipError_t e = async ? hipMallocAsync((void **)&P->dev, total, stream) : hipMalloc((void **)&P->dev, total);
    if (e != hipSuccess) { delete P; return hip_fail(e, "plan allocation"); }
    P->d_jobs = (SweepJob *)(P->dev + o_jobs);
    P->d_tile_start = (long long *)(P->dev + o_tiles);
    P->d_unit = (int *)(P->dev + o_unit);
    P->d_chunk_start = (long long *)(P->dev + o_chunk);
    size_t u = 0;
    for (size_t i = 0; i < n; i++)
        for (int j = 0; j < 4; j++) {
            if (j == S[i].d || !((S[i].emask >> j) & 1)) continue;
            uint4 *p = (uint4 *)(P->dev + o_prep + prep_off[u++]);
            S[i].prep[j] = p;
            S[i].prep_out[j] = p;
        }
    // one host image of the table block, copied in one transfer
    std::vector<char> img(o_prep, 0);
    memcpy(img.data() + o_jobs, S.data(), n * sizeof(SweepJob));
    memcpy(img.data() + o_tiles, tile_start.data(), n * sizeof(long long));
    if (!unit.empty()) {
        memcpy(img.data() + o_unit, unit.data(), unit.size() * sizeof(int));
        memcpy(img.data() + o_chunk, chunk_start.data(), chunk_start.size() * sizeof(long long));
    }
    e = async ? hipMemcpyAsync(P->dev, img.data(), img.size(), hipMemcpyHostToDevice, stream)
              : hipMemcpy(P->dev, img.data(), img.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && async) e = hipStreamSynchronize(stream);  // img is freed on return
    if (e != hipSuccess) { (void)hipFree(P->dev); delete P; return hip_fail(e, "plan upload"); }
    *out = P;
    return 0;
}

// The side stream of the current device (default priority), for the
// launch of the large-LDS tiles beside the others.
static hipStream_t side_stream()
{
    static std::mutex mu;
    static hipStream_t st[64];
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!st[dev] && hipStreamCreateWithFlags(&st[dev], hipStreamNonBlocking) != hipSuccess) st[dev] = nullptr;
    return st[dev];
}

static int plan_enqueue(pentago_sweep_plan *P, hipStream_t st)
{
    hipError_t e = launch_prep_batch(P->d_jobs, P->d_unit, P->d_chunk_start, P->nunits,
                                     P->total_chunks, P->T, st);
    const bool both = P->tiles_big > 0 && P->total_tiles > 0;
    hipStream_t side = both ? side_stream() : nullptr;
    if (both && !side) return fail(PENTAGO_EDEVICE, "side stream");
    hipEvent_t fork = nullptr, join = nullptr;
    if (e == hipSuccess && both) {
        e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
    }
    // the large-LDS tiles on the caller's stream, the others beside them
    if (e == hipSuccess && P->tiles_big > 0)
        e = launch_sweep_batch(P->d_jobs, P->d_tile_start, P->nbig, P->tiles_big, P->lds_big, P->threads, P->sym,
                               P->T, st);
    if (e == hipSuccess && P->total_tiles > 0)
        e = launch_sweep_batch(P->d_jobs + P->nbig, P->d_tile_start + P->nbig, P->njobs - P->nbig,
                               P->total_tiles, P->lds_bytes, P->threads, P->sym, P->T, both ? side : st);
    if (e == hipSuccess && both) {
        e = hipEventRecord(join, side);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, join, 0);
    }
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (e != hipSuccess) return hip_fail(e, "batched sweep launch");
    return 0;
}

}  // namespace pg

extern "C" {

int pentago_plan_create(const pentago_section_job *jobs, size_t n, pentago_sweep_plan **plan)
{
    if (!plan) return fail(PENTAGO_EINVAL, "plan is NULL");
    return plan_build(jobs, n, nullptr, false, false, plan);
}

int pentago_plan_create_d4(const pentago_section_job *jobs, size_t n, pentago_sweep_plan **plan)
{
    if (!plan) return fail(PENTAGO_EINVAL, "plan is NULL");
    return plan_build(jobs, n, nullptr, false, true, plan);
}

int pentago_plan_launch(pentago_sweep_plan *plan, void *hip_stream)
{
    if (!plan) return fail(PENTAGO_EINVAL, "plan is NULL");
    return plan_enqueue(plan, (hipStream_t)hip_stream);
}

int pentago_plan_launch_graph(pentago_sweep_plan *plan, void *hip_stream)
{
    if (!plan) return fail(PENTAGO_EINVAL, "plan is NULL");
    hipError_t e;
    if (!plan->exec) {
        e = hipStreamCreateWithFlags(&plan->capture, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        e = hipStreamBeginCapture(plan->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        int rc = plan_enqueue(plan, plan->capture);
        e = hipStreamEndCapture(plan->capture, &plan->graph);
        if (rc) return rc;
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    }
    e = hipGraphLaunch(plan->exec, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return 0;
}

int pentago_plan_info(const pentago_sweep_plan *plan, long long *tiles, int *grid, int *lds_bytes)
{
    if (!plan) return fail(PENTAGO_EINVAL, "plan is NULL");
    if (tiles) *tiles = plan->total_tiles + plan->tiles_big;
    if (grid) *grid = (int)std::min<long long>(plan->total_tiles + plan->tiles_big, 0x7fffffff);
    if (lds_bytes) *lds_bytes = std::max(plan->lds_bytes, plan->lds_big);
    return 0;
}

int pentago_plan_destroy(pentago_sweep_plan *plan)
{
    if (!plan) return 0;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->capture) (void)hipStreamDestroy(plan->capture);
    if (plan->dev) (void)hipFree(plan->dev);  // waits for work that uses it
    delete plan;
    return 0;
}

static int solve_sections(const pentago_section_job *jobs, size_t n, void *hip_stream, bool reps)
{
    const hipStream_t st = (hipStream_t)hip_stream;
    pentago_sweep_plan *P = nullptr;
    int rc = plan_build(jobs, n, st, true, reps, &P);
    if (rc) return rc;
    rc = plan_enqueue(P, st);
    (void)hipFreeAsync(P->dev, st);
    delete P;
    return rc;
}

int pentago_solve_sections(const pentago_section_job *jobs, size_t n, void *hip_stream)
{
    return solve_sections(jobs, n, hip_stream, false);
}

int pentago_solve_sections_d4(const pentago_section_job *jobs, size_t n, void *hip_stream)
{
    return solve_sections(jobs, n, hip_stream, true);
}

int pentago_autotune_sections(const pentago_section_job *jobs, size_t n, int reps, void *hip_stream,
                              int *cap_bytes, int *threads, float *best_ms)
{
    if (!jobs || n == 0) return fail(PENTAGO_EINVAL, "no jobs");
    const hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return fail(PENTAGO_EDEVICE, "hipEventCreate");
    BatchShape best_shape = kBatchDefault;
    int rc = 0;
    float best = 1e30f;
    for (int nt : kBatchThreadChoices) {
        for (int cap : kBatchCaps) {
            const BatchShape shape = {cap, nt};
            pentago_sweep_plan *P = nullptr;
            rc = plan_build(jobs, n, st, true, reps != 0, &P, shape);
            if (rc) break;
            rc = plan_enqueue(P, st);  // warm-up
            float t = 1e30f;
            for (int r = 0; r < 3 && rc == 0; r++) {
                (void)hipEventRecord(a, st);
                rc = plan_enqueue(P, st);
                (void)hipEventRecord(b, st);
                if (rc == 0 && hipEventSynchronize(b) != hipSuccess) rc = fail(PENTAGO_EDEVICE, "hipEventSynchronize");
                float ms = 0;
                if (rc == 0) (void)hipEventElapsedTime(&ms, a, b);
                t = std::min(t, ms);
            }
            (void)hipFreeAsync(P->dev, st);
            (void)hipStreamSynchronize(st);
            delete P;
            if (rc) break;
            if (t < best) {
                best = t;
                best_shape = shape;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    const int stones = section_stones(jobs[0].section);
    {
        std::lock_guard<std::mutex> lock(g_shape_mutex);
        if (stones >= 0 && stones <= 36) g_shape[stones] = best_shape;
    }
    if (cap_bytes) *cap_bytes = best_shape.cap;
    if (threads) *threads = best_shape.threads;
    if (best_ms) *best_ms = best;
    return 0;
}

}  // extern "C"
