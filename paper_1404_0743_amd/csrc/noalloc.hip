// noalloc.hip -- the allocation-free variant of pentago_eval_batch, for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops).  Its scratch (the roots' binning arrays, the work
// queue counters and the global DAG layer slots of roots with 9 or 10 empty
// cells) lives in one fixed device array instead of a stream-ordered
// allocation; the kernels are the ones pentago_eval_batch runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "internal.h"

namespace pg {

// Largest batch of the allocation-free call, and the number of workgroups of
// the 8-10 empty-cell class that own a global layer slot (the others take
// only roots with 8 empty cells, whose layers fit in LDS).
constexpr size_t kNoAllocMaxBoards = (size_t)1 << 20;
constexpr int kNoAllocSlots = 64;

constexpr size_t kNoAllocLayerBytes = (size_t)kNoAllocSlots * 2 * 4 * kDagGlobalLayer * sizeof(uint4);
constexpr size_t kNoAllocIntsOff = kNoAllocLayerBytes;             // count, start, cursor: 64 ints
constexpr size_t kNoAllocCounterOff = kNoAllocIntsOff + 256;       // 4 queue counters
constexpr size_t kNoAllocOrderOff = kNoAllocCounterOff + 256;      // order: int per root
constexpr size_t kNoAllocEmptiesOff = kNoAllocOrderOff + 4 * kNoAllocMaxBoards;  // u8 per root
constexpr size_t kNoAllocBytes = kNoAllocEmptiesOff + kNoAllocMaxBoards;

// One copy per device, held until the process ends.  Host code never uses
// this name as an address: it is resolved per device with
// hipGetSymbolAddress in pentago_init and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_mutex;
static void *g_scratch[kMaxDevices];
static int g_grid[kMaxDevices];

}  // namespace pg

using namespace pg;

extern "C" {

int pentago_init(void)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PENTAGO_ERANGE, "device index beyond 63");
    DevTables T;
    int rc = device_tables(&T);
    if (rc) return rc;
    int grid = 0;
    rc = eval_grid(&grid);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_scratch[dev]) return 0;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(PENTAGO_EDEVICE, "hipGetSymbolAddress(scratch) gave NULL");
    g_grid[dev] = grid;
    g_scratch[dev] = p;
    return 0;
}

int pentago_eval_batch_noalloc(const pentago_board *boards, size_t n, pentago_superinfo *out,
                               int32_t *status, void *hip_stream)
{
    if (n && (!boards || !out)) return fail(PENTAGO_EINVAL, "NULL boards or out");
    if (n > kNoAllocMaxBoards)
        return fail(PENTAGO_ERANGE, "more than 2^20 boards in one allocation-free call");
    if (n == 0) return 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PENTAGO_ERANGE, "device index beyond 63");
    DevTables T;
    if (device_tables_ready(&T)) return fail(PENTAGO_EINVAL, "pentago_init has not run on this device");
    char *base;
    int grid;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        base = (char *)g_scratch[dev];
        grid = g_grid[dev];
    }
    if (!base) return fail(PENTAGO_EINVAL, "pentago_init has not run on this device");
    EvalScratch S;
    S.global_layers = (uint4 *)base;
    S.count = (int *)(base + kNoAllocIntsOff);
    S.start = S.count + 16;
    S.cursor = S.count + 32;
    S.counter = (unsigned long long *)(base + kNoAllocCounterOff);
    S.order = (int *)(base + kNoAllocOrderOff);
    S.empties = (uint8_t *)(base + kNoAllocEmptiesOff);
    S.global_slots = std::min(kNoAllocSlots, grid);
    const hipStream_t st = (hipStream_t)hip_stream;
    // the binning pass clears the per-class counts and the persistent launch
    // its queue counters with small kernels: nothing from an earlier call is
    // read before it is rewritten
    e = launch_eval_bin((const uint64_t *)boards, n, S, status, (uint4 *)out, T, st);
    if (e == hipSuccess)
        e = launch_eval_persistent_slots((const uint64_t *)boards, n, (uint4 *)out, S, grid,
                                         S.global_slots, T, st);
    if (e != hipSuccess) return hip_fail(e, "eval launch");
    return 0;
}

}  // extern "C"
