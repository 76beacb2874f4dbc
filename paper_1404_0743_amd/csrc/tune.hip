// tune.hip -- the tile autotuner of the sweep: times the tile shapes a
// section admits (lines per tile) and remembers the fastest per section
// geometry, so later sweeps of the same geometry use it.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace pg {

using TileKey = std::tuple<int, int, int, int, int, int, int>;
static std::mutex g_tune_mutex;
static std::map<TileKey, TileShape> g_tile_cache;

static TileKey tile_key(const SweepJob &J)
{
    return TileKey(J.m[0], J.m[1], J.m[2], J.m[3], J.d, J.emask, J.cm[J.d]);
}

TileShape tuned_tile_shape(const SweepJob &J)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tile_cache.find(tile_key(J));
    return it == g_tile_cache.end() ? TileShape{0, 0, 0} : it->second;
}

void remember_tile_shape(const SweepJob &J, TileShape t)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tile_cache[tile_key(J)] = t;
}

// Launch prep passes and the sweep of one job (prep buffers stream-ordered).
int run_job(SweepJob &J, const DevTables &T, hipStream_t st)
{
    void *prep[4] = {nullptr, nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (int j = 0; j < 4 && e == hipSuccess; j++) {
        if (j == J.d || !((J.emask >> j) & 1)) continue;
        e = hipMallocAsync(&prep[j], prep_bytes(J, j), st);
        if (e != hipSuccess) break;
        J.prep[j] = J.prep_out[j] = (uint4 *)prep[j];
        e = launch_prep(J, j, T, st);
    }
    // full boards (no empty cell) take the terminal kernel
    if (e == hipSuccess) e = J.emask ? launch_sweep(J, T, st) : launch_terminal(J, T, st);
    for (int j = 0; j < 4; j++)
        if (prep[j]) (void)hipFreeAsync(prep[j], st);
    if (e != hipSuccess) return hip_fail(e, "sweep launch");
    return 0;
}

}  // namespace pg

using namespace pg;

extern "C" int pentago_autotune_section(pentago_section s, const pentago_superinfo *const child[4],
                                        pentago_superinfo *out, void *hip_stream, pentago_tile_shape *shape,
                                        float *best_ms)
{
    DevTables T;
    int rc = device_tables(&T);
    if (rc) return rc;
    SweepJob J0;
    rc = make_job(s, child, out, &J0, -1, 0);
    if (rc) return rc;
    const hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return fail(PENTAGO_EDEVICE, "hipEventCreate");
    TileShape best_shape{0, 0, 0};
    float best = 1e30f;
    const int cmd = (J0.emask >> J0.d) & 1 ? J0.cm[J0.d] : 0;
    for (int order = 0; order < 2 && rc == 0; order++) {
        for (int nt = 256; nt <= 512 && rc == 0; nt *= 2) {
            for (int G = 1; G <= 8 && rc == 0; G++) {
                if (sweep_lds_bytes(G, J0.m[J0.d], cmd) > 65536) break;
                SweepJob J;
                rc = make_job(s, child, out, &J, -1, G, nt, order);
                if (rc) break;
                rc = run_job(J, T, st);  // warm-up
                float t = 1e30f;
                for (int rep = 0; rep < 3 && rc == 0; rep++) {
                    (void)hipEventRecord(a, st);
                    rc = run_job(J, T, st);
                    (void)hipEventRecord(b, st);
                    if (hipEventSynchronize(b) != hipSuccess) rc = fail(PENTAGO_EDEVICE, "hipEventSynchronize");
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, a, b);
                    t = std::min(t, ms);
                }
                if (rc == 0 && t < best) {
                    best = t;
                    best_shape = TileShape{G, nt, order};
                }
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    remember_tile_shape(J0, best_shape);
    // leave out holding the result of the chosen shape
    SweepJob J;
    rc = make_job(s, child, out, &J, -1, best_shape.lines, best_shape.threads, best_shape.order);
    if (rc == 0) rc = run_job(J, T, st);
    if (shape) *shape = pentago_tile_shape{best_shape.lines, best_shape.threads, best_shape.order};
    if (best_ms) *best_ms = best;
    return rc;
}

extern "C" int pentago_solve_section_shape(pentago_section s, const pentago_superinfo *const child[4],
                                           pentago_superinfo *out, void *hip_stream,
                                           const pentago_tile_shape *shape)
{
    if (!shape) return fail(PENTAGO_EINVAL, "shape is NULL");
    if (shape->lines < 1 || shape->lines > 8 || (shape->threads != 256 && shape->threads != 512) ||
        shape->order < 0 || shape->order > 1)
        return fail(PENTAGO_ERANGE, "tile shape: 1..8 lines, 256 or 512 threads, order 0 or 1");
    DevTables T;
    int rc = device_tables(&T);
    if (rc) return rc;
    SweepJob J;
    rc = make_job(s, child, out, &J, -1, shape->lines, shape->threads, shape->order);
    if (rc) return rc;
    if (J.lds_bytes > 65536) return fail(PENTAGO_ERANGE, "tile shape needs more than 64 KiB of LDS");
    return run_job(J, T, (hipStream_t)hip_stream);
}
