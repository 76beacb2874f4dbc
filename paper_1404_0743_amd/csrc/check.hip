// check.hip -- checks of solved tables: the counts of won, tied and lost
// (entry, rotation) pairs of a table, which Section VII uses to check every
// computed slice, and the entries whose win set is not inside their not-lose
// set, which no solved table has (the value is win + notlose - 1, so win
// without not-lose encodes nothing).
#include <atomic>
#include <string>

#include "device_common.h"
#include "internal.h"

namespace pg {

// out[0..3] += wins, ties, losses (bits over every entry's 256 rotations) and
// invalid entries of table[0, n).  Lane i reads entry i whole (four 16-byte
// loads; a wave's loads cover 4 KB), grid-stride; one atomic per wave.
__global__ void __launch_bounds__(256) table_counts_kernel(const uint4 *table, uint64_t n, unsigned long long *out)
{
    unsigned long long win = 0, tie = 0, loss = 0, bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256u) {
        const uint4 *p = table + 4 * i;
        const uint4 w0 = p[0], w1 = p[1], n0 = p[2], n1 = p[3];
        const uint32_t W[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
        const uint32_t N[8] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, n1.z, n1.w};
        uint32_t cw = 0, ct = 0, cn = 0, inv = 0;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            cw += __popc(W[k]);
            ct += __popc(N[k] & ~W[k]);
            cn += __popc(N[k]);
            inv |= W[k] & ~N[k];
        }
        win += cw;
        tie += ct;
        loss += 256u - cn;
        bad += inv != 0u;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        win += __shfl_xor(win, off, 64);
        tie += __shfl_xor(tie, off, 64);
        loss += __shfl_xor(loss, off, 64);
        bad += __shfl_xor(bad, off, 64);
    }
    if ((threadIdx.x & 63u) == 0) {
        atomicAdd(out, win);
        atomicAdd(out + 1, tie);
        atomicAdd(out + 2, loss);
        atomicAdd(out + 3, bad);
    }
}

static hipError_t launch_table_counts(const uint4 *table, uint64_t n, unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, s, out, 4);
    if (n > 0) {
        const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 4096);
        hipLaunchKernelGGL(table_counts_kernel, dim3((unsigned)blocks), dim3(256), 0, s, table, n, out);
    }
    return hipGetLastError();
}

static std::atomic<int> g_validate{0};

// The entries of table[0, n) whose win set is not inside their not-lose set
// (synchronises st).
static int count_invalid(const uint4 *table, uint64_t n, hipStream_t st, unsigned long long *bad)
{
    unsigned long long *dev = nullptr;
    hipError_t e = hipMallocAsync((void **)&dev, 32, st);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(check)");
    unsigned long long host[4] = {0, 0, 0, 0};
    e = launch_table_counts(table, n, dev, st);
    if (e == hipSuccess) e = hipMemcpyAsync(host, dev, sizeof(host), hipMemcpyDeviceToHost, st);
    (void)hipFreeAsync(dev, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "table check");
    *bad = host[3];
    return 0;
}

// With validation on: every child table J reads must be a valid table.
int validate_children(const SweepJob &J, hipStream_t st)
{
    if (!g_validate.load()) return 0;
    uint64_t entries = 1;
    for (int j = 0; j < 4; j++) entries *= (uint64_t)J.m[j];
    for (int j = 0; j < 4; j++) {
        if (!J.child[j]) continue;
        const uint64_t centries = entries / (uint64_t)J.m[j] * (uint64_t)J.cm[j];
        unsigned long long bad = 0;
        const int rc = count_invalid(J.child[j], centries, st, &bad);
        if (rc) return rc;
        if (bad)
            return fail(PENTAGO_EINVAL, "child table of quadrant " + std::to_string(j) + " has " +
                                            std::to_string(bad) + " entries whose win set is not inside not-lose");
    }
    return 0;
}

}  // namespace pg

using namespace pg;

extern "C" {

int pentago_table_counts(const pentago_superinfo *table, uint64_t n, uint64_t *out, void *hip_stream)
{
    if (!out || (n && !table)) return fail(PENTAGO_EINVAL, "NULL table or out");
    const hipError_t e =
        launch_table_counts((const uint4 *)table, n, (unsigned long long *)out, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "pentago_table_counts");
    return 0;
}

int pentago_validate_table(const pentago_superinfo *table, uint64_t n, void *hip_stream)
{
    if (n && !table) return fail(PENTAGO_EINVAL, "NULL table");
    unsigned long long bad = 0;
    const int rc = count_invalid((const uint4 *)table, n, (hipStream_t)hip_stream, &bad);
    if (rc) return rc;
    if (bad) return fail(PENTAGO_EINVAL, std::to_string(bad) + " entries have a win set not inside not-lose");
    return 0;
}

int pentago_set_validate(int on)
{
    g_validate.store(on ? 1 : 0);
    return 0;
}

}  // extern "C"
