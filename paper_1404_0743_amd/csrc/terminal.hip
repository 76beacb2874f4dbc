// terminal.hip -- sections of full boards (36 stones): every entry's value is
// f_c - f_cbar for the side to move c (Section II), so the table is the pair
// W = F_c & ~F_o, N = F_c | ~F_o of five-sets over L (Section III), with no
// children.
//
// The five-set factors into six pair terms, each a function of the patterns
// of two quadrants (five_assemble in set256.h).  A first small kernel builds
// every pair term of the section (for full boards each quadrant class has at
// most 34 patterns, so all of them take under 300 KB; they are kept per
// section geometry, see launch_terminal); the entry kernel then
// takes one quarter of an 8^4 block per workgroup (Section IV layout: the
// entries with block-local index i0 in [2q, 2q + 2), a contiguous range of the
// table), copies the pair terms its patterns use into LDS and assembles each
// entry's two five-sets from 12 table reads.
#include "device_common.h"

#include <array>
#include <map>
#include <mutex>

namespace pg {

// Pair terms of a section, per colour x (0: the side to move, 1: the other
// side): t_ab[x][i_a][i_b] over the class indices of quadrants a and b; t23
// holds three uint4 per pair.
struct TermPairs {
    uint4 *t01, *t02, *t03, *t12, *t13, *t23;
    int m[4];
};

__device__ __forceinline__ LineMasks pattern_lines(const SweepJob &J, const DevTables &T, int j, int idx, int x)
{
    const QInfo q = T.qinfo[J.qb[j] + idx];
    // x = 0: the side to move's stones
    const unsigned m = (x == 0) == (J.mover == 1) ? q.bm : q.wm;
    return T.lm[j * 512 + m];
}

__global__ void __launch_bounds__(256) terminal_pairs_kernel(SweepJob J, DevTables T, TermPairs Q)
{
    const int m0 = J.m[0], m1 = J.m[1], m2 = J.m[2], m3 = J.m[3];
    const int n01 = m0 * m1, n02 = m0 * m2, n03 = m0 * m3, n12 = m1 * m2, n13 = m1 * m3, n23 = m2 * m3;
    const int per = n01 + n02 + n03 + n12 + n13 + n23;
    const int it = blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= 2 * per) return;
    const int x = it >= per;
    int k = it - per * x;
    if (k < n01) {
        Q.t01[x * n01 + k] = pair01(pattern_lines(J, T, 0, k / m1, x), pattern_lines(J, T, 1, k % m1, x));
        return;
    }
    k -= n01;
    if (k < n02) {
        Q.t02[x * n02 + k] = pair02(pattern_lines(J, T, 0, k / m2, x), pattern_lines(J, T, 2, k % m2, x));
        return;
    }
    k -= n02;
    if (k < n03) {
        Q.t03[x * n03 + k] = pair03(pattern_lines(J, T, 0, k / m3, x), pattern_lines(J, T, 3, k % m3, x));
        return;
    }
    k -= n03;
    if (k < n12) {
        Q.t12[x * n12 + k] = pair12(pattern_lines(J, T, 1, k / m2, x), pattern_lines(J, T, 2, k % m2, x));
        return;
    }
    k -= n12;
    if (k < n13) {
        Q.t13[x * n13 + k] = pair13(pattern_lines(J, T, 1, k / m3, x), pattern_lines(J, T, 3, k % m3, x));
        return;
    }
    k -= n13;
    uint4 t[3];
    pair23(pattern_lines(J, T, 2, k / m3, x), pattern_lines(J, T, 3, k % m3, x), t);
    uint4 *dst = Q.t23 + 3 * (x * n23 + k);
    dst[0] = t[0];
    dst[1] = t[1];
    dst[2] = t[2];
}

// LDS of one tile: the pair terms of its patterns (quadrant 0 relative to
// the tile's first index, the others relative to the block).
struct TermLds {
    uint4 t01[2][2 * 8];
    uint4 t02[2][2 * 8];
    uint4 t03[2][2 * 8];
    uint4 t12[2][8 * 8];
    uint4 t13[2][8 * 8];
    uint4 t23[2][8 * 8][3];
};

template <int NT>
__global__ void __launch_bounds__(NT) terminal_kernel(SweepJob J, TermPairs Q)
{
    __shared__ TermLds L;
    // tile -> (block, quarter): blocks in row-major order of block coordinates
    const uint32_t quarter = blockIdx.x & 3u, blk = blockIdx.x >> 2;
    const int nb3 = (J.m[3] + 7) >> 3, nb2 = (J.m[2] + 7) >> 3, nb1 = (J.m[1] + 7) >> 3;
    uint32_t r = blk;
    int B[4];
    B[3] = (int)(r % (uint32_t)nb3); r /= (uint32_t)nb3;
    B[2] = (int)(r % (uint32_t)nb2); r /= (uint32_t)nb2;
    B[1] = (int)(r % (uint32_t)nb1); r /= (uint32_t)nb1;
    B[0] = (int)r;
    int s[4];
#pragma unroll
    for (int j = 0; j < 4; j++) s[j] = min(8, J.m[j] - 8 * B[j]);
    const int first0 = 2 * (int)quarter;
    if (first0 >= s[0]) return;  // a quarter beyond a thin block's extent (whole workgroup)
    const int n0 = min(2, s[0] - first0);
    const int inner = s[1] * s[2] * s[3];
    const int n = n0 * inner;
    int bidx[4] = {8 * B[0], 8 * B[1], 8 * B[2], 8 * B[3]};
    const uint32_t base = block_offset(J.m, bidx) + (uint32_t)(first0 * inner);
    const int m0 = Q.m[0], m1 = Q.m[1], m2 = Q.m[2], m3 = Q.m[3];
    const int a0 = 8 * B[0] + first0, a1 = 8 * B[1], a2 = 8 * B[2], a3 = 8 * B[3];

    // the tile's pair terms: 3 x 16 slots over (Q0, Qj) and 3 x 64 over the
    // other pairs, per colour; slots beyond the block's extent are not read
    for (int it = threadIdx.x; it < 2 * 240; it += NT) {
        const int x = it >= 240, k = it - 240 * x;
        if (k < 48) {
            const int which = k >> 4, a = (k >> 3) & 1, b = k & 7;
            if (a >= n0) continue;
            if (which == 0) {
                if (b < s[1]) L.t01[x][k & 15] = Q.t01[(x * m0 + a0 + a) * m1 + a1 + b];
            } else if (which == 1) {
                if (b < s[2]) L.t02[x][k & 15] = Q.t02[(x * m0 + a0 + a) * m2 + a2 + b];
            } else {
                if (b < s[3]) L.t03[x][k & 15] = Q.t03[(x * m0 + a0 + a) * m3 + a3 + b];
            }
        } else {
            const int kk = k - 48, which = kk >> 6, a = (kk >> 3) & 7, b = kk & 7;
            if (which == 0) {
                if (a < s[1] && b < s[2]) L.t12[x][kk & 63] = Q.t12[(x * m1 + a1 + a) * m2 + a2 + b];
            } else if (which == 1) {
                if (a < s[1] && b < s[3]) L.t13[x][kk & 63] = Q.t13[(x * m1 + a1 + a) * m3 + a3 + b];
            } else if (a < s[2] && b < s[3]) {
                const uint4 *src = Q.t23 + 3 * ((x * m2 + a2 + a) * m3 + a3 + b);
                L.t23[x][kk & 63][0] = src[0];
                L.t23[x][kk & 63][1] = src[1];
                L.t23[x][kk & 63][2] = src[2];
            }
        }
    }
    __syncthreads();

    // entries: a wave takes 64 consecutive entries; quad lane l of quad q
    // computes entry 16 l + q, so that after the quad transpose store p writes
    // entries 16 p .. 16 p + 15 (1 KB in order)
    const int lane = threadIdx.x & 63, l4 = lane & 3, q = lane >> 2;
    const uint32_t d3 = 0xffffffffu / (uint32_t)s[3] + 1u, d2 = 0xffffffffu / (uint32_t)s[2] + 1u,
                   d1 = 0xffffffffu / (uint32_t)s[1] + 1u;
    for (int g0 = (threadIdx.x >> 6) * 64; g0 < n; g0 += NT) {
        const uint32_t e = (uint32_t)min(g0 + 16 * l4 + q, n - 1);  // a spare lane repeats the last entry
        // e -> (i0, i1, i2, i3) row-major over (n0, s1, s2, s3); a divisor of 1
        // has no 32-bit multiplier
        const uint32_t e3 = s[3] > 1 ? __umulhi(e, d3) : e, i3 = e - e3 * (uint32_t)s[3];
        const uint32_t e2 = s[2] > 1 ? __umulhi(e3, d2) : e3, i2 = e3 - e2 * (uint32_t)s[2];
        const uint32_t i0 = s[1] > 1 ? __umulhi(e2, d1) : e2, i1 = e2 - i0 * (uint32_t)s[1];
        Set256 F[2];
#pragma unroll
        for (int x = 0; x < 2; x++) {
            const uint4 t23[3] = {L.t23[x][8 * i2 + i3][0], L.t23[x][8 * i2 + i3][1], L.t23[x][8 * i2 + i3][2]};
            F[x] = five_assemble(L.t01[x][8 * i0 + i1], L.t02[x][8 * i0 + i2], L.t12[x][8 * i1 + i2],
                                 L.t03[x][8 * i0 + i3], L.t13[x][8 * i1 + i3], t23);
        }
        uint4 v[4];
        v[0] = make_uint4(F[0].w[0] & ~F[1].w[0], F[0].w[1] & ~F[1].w[1], F[0].w[2] & ~F[1].w[2], F[0].w[3] & ~F[1].w[3]);
        v[1] = make_uint4(F[0].w[4] & ~F[1].w[4], F[0].w[5] & ~F[1].w[5], F[0].w[6] & ~F[1].w[6], F[0].w[7] & ~F[1].w[7]);
        v[2] = make_uint4(F[0].w[0] | ~F[1].w[0], F[0].w[1] | ~F[1].w[1], F[0].w[2] | ~F[1].w[2], F[0].w[3] | ~F[1].w[3]);
        v[3] = make_uint4(F[0].w[4] | ~F[1].w[4], F[0].w[5] | ~F[1].w[5], F[0].w[6] | ~F[1].w[6], F[0].w[7] | ~F[1].w[7]);
        quad_transpose(v, l4);
#pragma unroll
        for (int p = 0; p < 4; p++)
            if (g0 + 16 * p + q < n) store_stream(J.out + 4 * ((size_t)base + g0 + 16 * p + q) + l4, v[p]);
    }
}

// Pair terms depend only on the section's four (black, white) classes and
// the side to move, so they are built once per device and geometry and kept: the first call builds them on its stream and
// records an event that later calls on other streams wait for.  At most
// kPairCacheMax geometries are kept; beyond that a call builds its own in
// stream-ordered scratch.
constexpr int kPairCacheMax = 64;

struct PairEntry {
    void *buf;
    hipEvent_t ready;
};

static std::mutex g_pair_mutex;
static std::map<std::array<int, 10>, PairEntry> g_pairs;

static TermPairs pair_layout(const SweepJob &J, void *buf)
{
    const size_t m0 = J.m[0], m1 = J.m[1], m2 = J.m[2], m3 = J.m[3];
    TermPairs Q;
    Q.t01 = (uint4 *)buf;
    Q.t02 = Q.t01 + 2 * m0 * m1;
    Q.t03 = Q.t02 + 2 * m0 * m2;
    Q.t12 = Q.t03 + 2 * m0 * m3;
    Q.t13 = Q.t12 + 2 * m1 * m2;
    Q.t23 = Q.t13 + 2 * m1 * m3;
    for (int j = 0; j < 4; j++) Q.m[j] = J.m[j];
    return Q;
}

static size_t pair_bytes(const SweepJob &J)
{
    const size_t m0 = J.m[0], m1 = J.m[1], m2 = J.m[2], m3 = J.m[3];
    return 2 * (m0 * m1 + m0 * m2 + m0 * m3 + m1 * m2 + m1 * m3 + 3 * m2 * m3) * sizeof(uint4);
}

static void launch_pairs(const SweepJob &J, const DevTables &T, const TermPairs &Q, hipStream_t s)
{
    const size_t m0 = J.m[0], m1 = J.m[1], m2 = J.m[2], m3 = J.m[3];
    const size_t items = 2 * (m0 * m1 + m0 * m2 + m0 * m3 + m1 * m2 + m1 * m3 + m2 * m3);
    hipLaunchKernelGGL(terminal_pairs_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, J, T, Q);
}

hipError_t launch_terminal(const SweepJob &J, const DevTables &T, hipStream_t s)
{
    int nb = 1;
    for (int j = 0; j < 4; j++) nb *= (J.m[j] + 7) / 8;
    if (nb == 0) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::array<int, 10> key{dev};
    for (int j = 0; j < 4; j++) {
        key[1 + j] = J.qb[j];
        key[5 + j] = J.m[j];
    }
    key[9] = J.mover;
    void *own = nullptr;
    TermPairs Q;
    {
        std::lock_guard<std::mutex> lock(g_pair_mutex);
        auto it = g_pairs.find(key);
        if (it != g_pairs.end()) {
            Q = pair_layout(J, it->second.buf);
            e = hipStreamWaitEvent(s, it->second.ready, 0);
            if (e != hipSuccess) return e;
        } else if ((int)g_pairs.size() < kPairCacheMax) {
            PairEntry P{nullptr, nullptr};
            e = hipMalloc(&P.buf, pair_bytes(J));
            if (e != hipSuccess) return e;
            e = hipEventCreateWithFlags(&P.ready, hipEventDisableTiming);
            if (e != hipSuccess) {
                (void)hipFree(P.buf);
                return e;
            }
            Q = pair_layout(J, P.buf);
            launch_pairs(J, T, Q, s);
            e = hipEventRecord(P.ready, s);
            if (e != hipSuccess) return e;
            g_pairs[key] = P;
        } else {
            e = hipMallocAsync(&own, pair_bytes(J), s);
            if (e != hipSuccess) return e;
            Q = pair_layout(J, own);
            launch_pairs(J, T, Q, s);
        }
    }
    const unsigned tiles = (unsigned)(4 * nb);
    if (J.threads == 512)
        hipLaunchKernelGGL(terminal_kernel<512>, dim3(tiles), dim3(512), 0, s, J, Q);
    else
        hipLaunchKernelGGL(terminal_kernel<256>, dim3(tiles), dim3(256), 0, s, J, Q);
    e = hipGetLastError();
    if (own) (void)hipFreeAsync(own, s);
    return e;
}

}  // namespace pg
