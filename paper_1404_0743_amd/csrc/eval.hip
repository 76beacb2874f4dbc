// eval.hip -- C ABI of the endgame solver: arbitrary boards solved to the
// full board over all 256 quadrant rotations (Section VIII serial solver),
// binned by number of empty cells on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <set>

#include "internal.h"

namespace pg {

static std::mutex g_pool_mutex;
static std::set<int> g_pool_ready;

// Keep stream-ordered allocations pooled instead of returning them to the
// driver after every call.
void keep_pool(int dev)
{
    std::lock_guard<std::mutex> lock(g_pool_mutex);
    if (g_pool_ready.count(dev)) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t big = ~0ull;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &big);
    }
    g_pool_ready.insert(dev);
}

int eval_grid(int *grid)
{
    static int cached[64] = {0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 64 && cached[dev]) {
        *grid = cached[dev];
        return 0;
    }
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    // two 256-thread workgroups per CU fit the LDS of the deepest in-LDS DAG
    *grid = std::max(1, 2 * cus);
    if (dev < 64) cached[dev] = *grid;
    keep_pool(dev);
    return 0;
}

struct EvalAlloc {
    void *base = nullptr;
    EvalScratch S;
};

static int eval_alloc(size_t n, int grid, hipStream_t st, EvalAlloc *A)
{
    const size_t ints = 64;
    const size_t glayer = (size_t)grid * 2 * kDagGlobalLayer * 64;
    const size_t bytes = glayer + ints * 4 + 32 + n * 4 + n + 256;
    hipError_t e = hipMallocAsync(&A->base, bytes, st);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(eval scratch)");
    char *p = (char *)A->base;
    A->S.global_layers = (uint4 *)p;
    p += glayer;
    A->S.count = (int *)p;
    A->S.start = A->S.count + 16;
    A->S.cursor = A->S.count + 32;
    p += ints * 4;
    A->S.counter = (unsigned long long *)p;  // one work-queue counter per persistent class
    p += 32;
    A->S.order = (int *)p;
    p += n * 4;
    A->S.empties = (uint8_t *)p;
    A->S.global_slots = grid;
    return 0;
}

// Scratch bytes of one endgame batch of n roots (deep: some root has 9 or
// 10 empty cells and needs the global layer buffers).
size_t eval_scratch_bytes(size_t n, int grid, bool deep)
{
    return (deep ? (size_t)grid * 2 * kDagGlobalLayer * 64 : 0) + 64 * 4 + 32 + n * 5 + 256;
}

// Enqueue one endgame batch on st with stream-ordered scratch.
int eval_enqueue(const uint64_t *boards, size_t n, uint4 *out, int *status, bool deep, int grid,
                 hipStream_t st)
{
    DevTables T;
    int rc = device_tables(&T);
    if (rc) return rc;
    EvalAlloc A;
    rc = eval_alloc(n, deep ? grid : 0, st, &A);
    if (rc) return rc;
    A.S.global_slots = grid;
    hipError_t e = launch_eval_bin(boards, n, A.S, status, out, T, st);
    if (e == hipSuccess) e = launch_eval_persistent(boards, n, out, A.S, grid, T, st);
    (void)hipFreeAsync(A.base, st);
    if (e != hipSuccess) return hip_fail(e, "eval launch");
    return 0;
}

// Enqueue one batch whose roots all belong to endgame class cls (see
// launch_eval_direct): one queue counter and, for roots with 9 or 10 empty
// cells, the global layer slots; no binning.
int eval_enqueue_class(const uint64_t *boards, size_t n, uint4 *out, int cls, bool deep, int grid,
                       hipStream_t st)
{
    DevTables T;
    int rc = device_tables(&T);
    if (rc) return rc;
    void *base = nullptr;
    const size_t glayer = deep ? (size_t)grid * 2 * kDagGlobalLayer * 64 : 0;
    hipError_t e = hipMallocAsync(&base, glayer + 256, st);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(eval scratch)");
    uint4 *gl = deep ? (uint4 *)base : nullptr;
    unsigned long long *counter = (unsigned long long *)((char *)base + glayer);
    e = launch_eval_direct(boards, (int)n, out, cls, counter, gl, grid, T, st);
    (void)hipFreeAsync(base, st);
    if (e != hipSuccess) return hip_fail(e, "eval launch");
    return 0;
}

}  // namespace pg

using namespace pg;

extern "C" {

int pentago_eval_batch(const pentago_board *boards, size_t n, pentago_superinfo *out,
                       int32_t *status, void *hip_stream)
{
    if (n && (!boards || !out)) return fail(PENTAGO_EINVAL, "NULL boards or out");
    if (n > (size_t)1 << 30) return fail(PENTAGO_ERANGE, "more than 2^30 boards");
    if (n == 0) return 0;
    DevTables T;
    int rc = device_tables(&T);
    if (rc) return rc;
    int grid;
    rc = eval_grid(&grid);
    if (rc) return rc;
    const hipStream_t st = (hipStream_t)hip_stream;
    EvalAlloc A;
    rc = eval_alloc(n, grid, st, &A);
    if (rc) return rc;
    hipError_t e = launch_eval_bin((const uint64_t *)boards, n, A.S, status, (uint4 *)out, T, st);
    if (e == hipSuccess)
        e = launch_eval_persistent((const uint64_t *)boards, n, (uint4 *)out, A.S, grid, T, st);
    (void)hipFreeAsync(A.base, st);
    if (e != hipSuccess) return hip_fail(e, "eval launch");
    return 0;
}

int pentago_autotune_eval(const pentago_board *boards, size_t n, pentago_superinfo *out, void *hip_stream,
                          int threads[2], float *best_ms)
{
    if (n && (!boards || !out)) return fail(PENTAGO_EINVAL, "NULL boards or out");
    if (n > (size_t)1 << 30) return fail(PENTAGO_ERANGE, "more than 2^30 boards");
    if (n == 0) return 0;
    const hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return fail(PENTAGO_EDEVICE, "hipEventCreate");
    int best0 = 0, best1 = 0, rc = 0;
    float best = 1e30f;
    for (int c0 = 256; c0 <= 512 && rc == 0; c0 *= 2)
        for (int c1 = 256; c1 <= 512 && rc == 0; c1 *= 2) {
            set_eval_class_threads(c0, c1);
            rc = pentago_eval_batch(boards, n, out, nullptr, hip_stream);  // warm-up
            float t = 1e30f;
            for (int rep = 0; rep < 3 && rc == 0; rep++) {
                (void)hipEventRecord(a, st);
                rc = pentago_eval_batch(boards, n, out, nullptr, hip_stream);
                (void)hipEventRecord(b, st);
                if (hipEventSynchronize(b) != hipSuccess) rc = fail(PENTAGO_EDEVICE, "hipEventSynchronize");
                float ms = 0;
                (void)hipEventElapsedTime(&ms, a, b);
                t = std::min(t, ms);
            }
            if (rc == 0 && t < best) {
                best = t;
                best0 = c0;
                best1 = c1;
            }
        }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    set_eval_class_threads(best0, best1);
    rc = pentago_eval_batch(boards, n, out, nullptr, hip_stream);
    if (threads) {
        threads[0] = best0;
        threads[1] = best1;
    }
    if (best_ms) *best_ms = best;
    return rc;
}

int pentago_eval_batch_grouped(const pentago_board *boards, size_t n, pentago_superinfo *out,
                               int32_t *status, void *hip_stream)
{
    if (n && (!boards || !out)) return fail(PENTAGO_EINVAL, "NULL boards or out");
    if (n > (size_t)1 << 30) return fail(PENTAGO_ERANGE, "more than 2^30 boards");
    if (n == 0) return 0;
    DevTables T;
    int rc = device_tables(&T);
    if (rc) return rc;
    int grid;
    rc = eval_grid(&grid);
    if (rc) return rc;
    const hipStream_t st = (hipStream_t)hip_stream;
    EvalAlloc A;
    rc = eval_alloc(n, grid, st, &A);
    if (rc) return rc;
    hipError_t e = launch_eval_bin((const uint64_t *)boards, n, A.S, status, (uint4 *)out, T, st);
    int start[16];
    if (e == hipSuccess) e = hipMemcpyAsync(start, A.S.start, sizeof(start), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    for (int k = 10; k >= 0 && e == hipSuccess; k--) {
        const int first = start[k];
        const int count = (k == 0 ? start[11] : start[k - 1]) - first;
        e = launch_eval_group((const uint64_t *)boards, k, first, count, (uint4 *)out, A.S, T, st);
    }
    (void)hipFreeAsync(A.base, st);
    if (e != hipSuccess) return hip_fail(e, "eval launch");
    return 0;
}

}  // extern "C"
