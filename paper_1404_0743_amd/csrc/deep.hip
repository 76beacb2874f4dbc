// deep.hip -- the endgame solver for one deep root (Section VIII: positions
// outside the database are solved from scratch, rotations folded in by rmax
// only; the paper's serial solver evaluates an 18-stone position in 16 s on
// one CPU thread).  Where the batched solver keeps a root's whole DAG in one
// workgroup's LDS (up to 10 empty cells), this one spreads each layer of one
// root over the whole GPU, with the layers in HBM: an 18-empty root has
// 86,574,831 nodes, at most 17,153,136 in one layer.
//
// Node (t, cmask, omask) of a root with e empty cells is the root with t more
// stones: the root's side to move on the cells of cmask (ceil(t/2) of them),
// the other side on omask (floor(t/2)), cells numbered 0..e-1.  Its index in
// layer t is rank(cmask) * C(e - |cmask|, |omask|) + rank'(omask), with rank
// the colex rank of a subset of the e cells (sum of C(c_i, i + 1) over its
// cells c_0 < c_1 < ...) and rank' the colex rank of omask among the cells
// not in cmask.  Layers are solved from t = e down to 0, each node keeping for
// its parents A = F_parent(node) | rmax(not N), B = F_parent(node) | rmax(not
// W) (64 B), as in the batched solver.
#include "device_common.h"
#include "internal.h"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <set>

namespace pg {

constexpr int kDeepMaxEmpty = 20;

static __constant__ uint32_t c_binom[kDeepMaxEmpty + 2][kDeepMaxEmpty + 2];

struct DeepJob {
    int e;                        // empty cells of the root
    int t;                        // layer
    int mover;                    // side to move at the root (1 black, 2 white)
    unsigned cm0[4], om0[4];      // the root's stones of the mover and the other side
    int slot_q[kDeepMaxEmpty];    // quadrant and local cell of each empty cell
    int slot_l[kDeepMaxEmpty];
    uint32_t nsub_c, nsub_o;      // subsets of the mover's / other side's size in layer t
    uint32_t nodes;               // nodes of layer t
    uint4 *ftab;                  // five-sets: [nsub_c] of the mover's subsets, then [nsub_o]
    const uint4 *prev;            // A/B records of layer t + 1
    uint4 *cur;                   // A/B records of layer t
    uint4 *out;                   // the root's W/N (t = 0)
    int parity;                   // -1: all of L; 0 / 1: only the root's g with that parity of sum g_i
};

// Parity-halved records (Section VIII: rmax flips the parity of
// g0 + g1 + g2 + g3, so a root's values of one parity need each layer's
// terms of one parity only, alternating from layer to layer).  Bit
// g0 + 4 g1 + 16 (g2 & 1) of word (g2 >> 1) + 2 g3 has parity
// popcount(bit & 0x15) + g3 (mod 2); kEvenBits marks the even bits of the
// words with g3 even (0, 1, 4, 5).  Words w and w ^ 2 differ in g3 by one,
// so the bits of one parity of both fit one word: a 256-bit set of that
// parity packs into 4 words, and a node's A/B record into 32 B.
constexpr uint32_t kEvenBits = 0x5a5aa5a5u;

// Mask of the bits of parity par in the words with g3 even.
__device__ __forceinline__ uint32_t parity_bits(int par) { return par ? ~kEvenBits : kEvenBits; }

// Pack the bits of parity par of x (words 0, 1, 4, 5 with 2, 3, 6, 7).
__device__ __forceinline__ uint4 pack_parity(const Set256 &x, int par)
{
    const uint32_t m = parity_bits(par);
    return make_uint4((x.w[0] & m) | (x.w[2] & ~m), (x.w[1] & m) | (x.w[3] & ~m), (x.w[4] & m) | (x.w[6] & ~m),
                      (x.w[5] & m) | (x.w[7] & ~m));
}

// Unpack: both words of a pair take the packed word.  The bits of the other
// parity then hold values of no meaning; every use below is bitwise per g or
// goes through rmax, which reads them only for results of that other parity,
// and those are dropped again when the next record is packed.
__device__ __forceinline__ Set256 unpack_parity(uint4 v)
{
    Set256 x;
    x.w[0] = x.w[2] = v.x;
    x.w[1] = x.w[3] = v.y;
    x.w[4] = x.w[6] = v.z;
    x.w[5] = x.w[7] = v.w;
    return x;
}

typedef uint32_t BinomRow[kDeepMaxEmpty + 2];

__device__ __forceinline__ uint32_t colex_rank(unsigned mask, const BinomRow *bn)
{
    uint32_t r = 0;
    int i = 0;
    while (mask) {
        const int c = __builtin_ctz(mask);
        mask &= mask - 1;
        r += bn[c][i + 1];
        i++;
    }
    return r;
}

// The subset of {0..n-1} with k elements and colex rank r.
__device__ __forceinline__ unsigned colex_unrank(uint32_t r, int k, int n, const BinomRow *bn)
{
    unsigned mask = 0;
    for (int c = n - 1; c >= 0 && k > 0; c--) {
        const uint32_t b = bn[c][k];
        if (r >= b) {
            mask |= 1u << c;
            r -= b;
            k--;
        }
    }
    return mask;
}

// The k-th bit of m placed at the position of the k-th set bit of `within`
// (pdep).
__device__ __forceinline__ unsigned unpack_bits(unsigned m, unsigned within)
{
    unsigned r = 0;
    int i = 0;
    while (within) {
        const int c = __builtin_ctz(within);
        within &= within - 1;
        r |= ((m >> i) & 1u) << c;
        i++;
    }
    return r;
}

// Colex rank of omask among the cells not in cmask (rank of the packed
// subset): omask's cell c sits at c - popcount(cmask below c) among them.
__device__ __forceinline__ uint32_t rank_in_free(unsigned omask, unsigned cmask, const BinomRow *bn)
{
    uint32_t r = 0;
    int i = 0;
    while (omask) {
        const int c = __builtin_ctz(omask);
        omask &= omask - 1;
        r += bn[c - __popc(cmask & ((1u << c) - 1u))][i + 1];
        i++;
    }
    return r;
}

// The binomial table, copied to LDS by each workgroup: the lanes index it
// with different values, and from LDS those reads cost a few cycles instead
// of a dependent memory load each (the ranking loops chain them).
__device__ __forceinline__ const BinomRow *lds_binom(BinomRow *sb)
{
    for (int k = threadIdx.x; k < (kDeepMaxEmpty + 2) * (kDeepMaxEmpty + 2); k += blockDim.x)
        sb[k / (kDeepMaxEmpty + 2)][k % (kDeepMaxEmpty + 2)] = c_binom[k / (kDeepMaxEmpty + 2)][k % (kDeepMaxEmpty + 2)];
    __syncthreads();
    return sb;
}

// Five-set of every subset of the empty cells of the two sizes of layer t
// (the mover's ceil(t/2) cells, the other side's floor(t/2)), indexed by
// colex rank: each node then reads its two.
__global__ void __launch_bounds__(256) deep_five_kernel(DeepJob J, DevTables T)
{
    __shared__ BinomRow sb[kDeepMaxEmpty + 2];
    const BinomRow *bn = lds_binom(sb);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= J.nsub_c + J.nsub_o) return;
    const bool mine = i < J.nsub_c;
    const int k = mine ? (J.t + 1) >> 1 : J.t >> 1;
    const unsigned m = colex_unrank(mine ? i : i - J.nsub_c, k, J.e, bn);
    unsigned xm[4];
#pragma unroll
    for (int j = 0; j < 4; j++) xm[j] = mine ? J.cm0[j] : J.om0[j];
    for (int sl = 0; sl < J.e; sl++)
        if ((m >> sl) & 1) {
            const int q = J.slot_q[sl];
            const unsigned bit = 1u << J.slot_l[sl];
            xm[0] |= q == 0 ? bit : 0u;
            xm[1] |= q == 1 ? bit : 0u;
            xm[2] |= q == 2 ? bit : 0u;
            xm[3] |= q == 3 ? bit : 0u;
        }
    const Set256 F = board_five(T, xm);
    uint4 *dst = J.ftab + 2 * (size_t)i;
    dst[0] = make_uint4(F.w[0], F.w[1], F.w[2], F.w[3]);
    dst[1] = make_uint4(F.w[4], F.w[5], F.w[6], F.w[7]);
}

// One node of layer t per thread (Section II recurrence on Section III
// tables): OR the children's prepared terms, combine with the node's own
// five-sets, keep the terms its parents read (the root's W/N at t = 0).
// HALF: records of 32 B holding one parity (the root's parity J.parity).
template <bool HALF>
__global__ void __launch_bounds__(256) deep_node_kernel(DeepJob J, DevTables T)
{
    __shared__ BinomRow sb[kDeepMaxEmpty + 2];
    const BinomRow *bn = lds_binom(sb);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= J.nodes) return;
    const int e = J.e, t = J.t;
    const int sc = (t + 1) >> 1, so = t >> 1;
    const unsigned all = (1u << e) - 1u;
    const uint32_t per = bn[e - sc][so];
    const uint32_t r1 = i / per, r2 = i - r1 * per;
    const unsigned cmask = colex_unrank(r1, sc, e, bn);
    const unsigned omask = unpack_bits(colex_unrank(r2, so, e - sc, bn), all & ~cmask);
    // (cmask was unranked from r1, so r1 is its colex rank)
    const Set256 Fc = set_from(J.ftab + 2 * (size_t)r1);
    const Set256 Fo = set_from(J.ftab + 2 * ((size_t)J.nsub_c + colex_rank(omask, bn)));
    const bool xroot = (t & 1) == 0;   // the side to move at layer t is the root's mover
    const Set256 &Fx = xroot ? Fc : Fo;
    const Set256 &Fy = xroot ? Fo : Fc;
    Set256 Wnt = s_zero(), Nnt = s_zero();
    if (t == e) {
        Nnt = s_full();
    } else {
        // children: the side to move puts a stone on a free cell
        // child index rank(cmask') * C(e - |cmask'|, |omask'|) + rank of omask'
        // among the cells not in cmask': cmask grows when the root's mover
        // moves, else omask grows and cmask's rank is the same for all children
        const int cso = xroot ? so : so + 1;   // the other side's stones in layer t + 1
        const uint32_t rc = r1;
        const uint32_t per_c = xroot ? bn[e - sc - 1][cso] : bn[e - sc][cso];
        auto child_index = [&](int sl) -> uint32_t {
            const unsigned bit = 1u << sl;
            return xroot ? colex_rank(cmask | bit, bn) * per_c + rank_in_free(omask, cmask | bit, bn)
                         : rc * per_c + rank_in_free(omask | bit, cmask, bn);
        };
        // Every node of the layer has e - t free cells.  With 32 B records two
        // children go per step, both loads issued before either is used (an
        // odd count repeats the last child, which OR absorbs); with 64 B
        // records the pair's registers would cost occupancy, so one per step.
        const int nch = e - t;
        unsigned f = all & ~(cmask | omask);
        for (int k = 0; k < nch; k += HALF ? 2 : 1) {
            const int sa = __builtin_ctz(f);
            f &= f - 1;
            const uint32_t ca = child_index(sa);
            if (HALF) {
                const int sb = k + 1 < nch ? __builtin_ctz(f) : sa;
                f &= f - 1;
                const uint32_t cb = child_index(sb);
                const uint4 *pa = J.prev + 2 * (size_t)ca, *pb = J.prev + 2 * (size_t)cb;
                const uint4 a0 = pa[0], a1 = pa[1], b0 = pb[0], b1 = pb[1];
                s_or_into(Wnt, unpack_parity(a0));
                s_or_into(Nnt, unpack_parity(a1));
                s_or_into(Wnt, unpack_parity(b0));
                s_or_into(Nnt, unpack_parity(b1));
            } else {
                const uint4 *p = J.prev + 4 * (size_t)ca;
                s_or_into(Wnt, set_from(p));
                s_or_into(Nnt, set_from(p + 2));
            }
        }
    }
    Set256 W, N;
    combine(Fx, Fy, Wnt, Nnt, W, N);
    if (t == 0) {
        if (HALF) {
            // the root's entries of the other parity are cleared
            const uint32_t m = parity_bits(J.parity);
#pragma unroll
            for (int w = 0; w < 8; w++) {
                const uint32_t mw = (w & 2) ? ~m : m;
                W.w[w] &= mw;
                N.w[w] &= mw;
            }
        }
        store_info(J.out, W, N);
    } else if (HALF) {
        // a parent at parity p reads this record at p; layer t's records
        // carry the root's parity for odd t and the other one for even t
        Set256 A, B;
        child_terms(Fy, W, N, A, B);
        const int par = J.parity ^ ((t + 1) & 1);
        uint4 *p = J.cur + 2 * (size_t)i;
        p[0] = pack_parity(A, par);
        p[1] = pack_parity(B, par);
    } else {
        Set256 A, B;
        child_terms(Fy, W, N, A, B);
        uint4 *p = J.cur + 4 * (size_t)i;
        p[0] = make_uint4(A.w[0], A.w[1], A.w[2], A.w[3]);
        p[1] = make_uint4(A.w[4], A.w[5], A.w[6], A.w[7]);
        p[2] = make_uint4(B.w[0], B.w[1], B.w[2], B.w[3]);
        p[3] = make_uint4(B.w[4], B.w[5], B.w[6], B.w[7]);
    }
}

static uint64_t binom_host(int n, int k)
{
    if (k < 0 || k > n) return 0;
    uint64_t r = 1;
    for (int i = 1; i <= k; i++) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
    return r;
}

// Device bytes the deep solver needs for a root with e empty cells: two
// layers of records (64 B, or 32 B when halved by parity) and the largest
// pair of five-set tables.
size_t deep_scratch_bytes(int e, bool half)
{
    uint64_t layer = 0, sub = 0;
    for (int t = 0; t <= e; t++) {
        layer = std::max(layer, binom_host(e, t) * binom_host(t, (t + 1) / 2));
        sub = std::max(sub, binom_host(e, (t + 1) / 2) + binom_host(e, t / 2));
    }
    return 2 * (size_t)layer * (half ? 32 : 64) + (size_t)sub * 32 + 256;
}

}  // namespace pg

namespace pg {

// Empty cells of a board (-1 for an invalid code).
int board_empties(uint64_t packed)
{
    int e = 0;
    for (int j = 0; j < 4; j++) {
        int x = (int)((packed >> (16 * j)) & 0xffff);
        if (x >= 19683) return -1;
        for (int l = 0; l < 9; l++, x /= 3) e += x % 3 == 0;
    }
    return e;
}

// Enqueue the deep solve of one board (packed quadrant codes) on st.
int eval_deep_enqueue(uint64_t packed, uint4 *out, hipStream_t st, int parity)
{
    if (parity < -1 || parity > 1) return fail(PENTAGO_EINVAL, "parity must be 0 or 1");
    pentago_board board;
    for (int j = 0; j < 4; j++) board.q[j] = (uint16_t)((packed >> (16 * j)) & 0xffff);
    DevTables T;
    int rc = device_tables(&T);
    if (rc) return rc;
    DeepJob J;
    memset(&J, 0, sizeof(J));
    int nb = 0, nw = 0, e = 0;
    unsigned bm[4], wm[4];
    for (int j = 0; j < 4; j++) {
        if (board.q[j] >= 19683) return fail(PENTAGO_EINVAL, "invalid quadrant code");
        bm[j] = wm[j] = 0;
        int x = board.q[j];
        for (int l = 0; l < 9; l++, x /= 3) {
            if (x % 3 == 1) bm[j] |= 1u << l;
            if (x % 3 == 2) wm[j] |= 1u << l;
        }
        nb += __builtin_popcount(bm[j]);
        nw += __builtin_popcount(wm[j]);
        for (int l = 0; l < 9; l++)
            if (!(((bm[j] | wm[j]) >> l) & 1)) {
                if (e < kDeepMaxEmpty) {
                    J.slot_q[e] = j;
                    J.slot_l[e] = l;
                }
                e++;
            }
    }
    if (nb != nw && nb != nw + 1) return fail(PENTAGO_EINVAL, "invalid stone counts");
    if (e > kDeepMaxEmpty) return fail(PENTAGO_ERANGE, "more than 20 empty cells");
    J.e = e;
    J.mover = nb == nw ? 1 : 2;
    J.parity = parity;
    const bool half = parity >= 0;
    const size_t rec = half ? 32 : 64;
    for (int j = 0; j < 4; j++) {
        J.cm0[j] = J.mover == 1 ? bm[j] : wm[j];
        J.om0[j] = J.mover == 1 ? wm[j] : bm[j];
    }
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return hip_fail(err, "hipGetDevice");
    {
        // the binomial table, once per device
        static std::mutex mu;
        static std::set<int> ready;
        std::lock_guard<std::mutex> lock(mu);
        if (!ready.count(dev)) {
            uint32_t tab[kDeepMaxEmpty + 2][kDeepMaxEmpty + 2];
            for (int n = 0; n < kDeepMaxEmpty + 2; n++)
                for (int k = 0; k < kDeepMaxEmpty + 2; k++) tab[n][k] = (uint32_t)binom_host(n, k);
            err = hipMemcpyToSymbol(HIP_SYMBOL(c_binom), tab, sizeof(tab));
            if (err != hipSuccess) return hip_fail(err, "binomial table upload");
            ready.insert(dev);
        }
    }
    keep_pool(dev);
    uint64_t maxlayer = 0;
    for (int t = 0; t <= e; t++) maxlayer = std::max(maxlayer, binom_host(e, t) * binom_host(t, (t + 1) / 2));
    char *base = nullptr;
    err = hipMallocAsync((void **)&base, deep_scratch_bytes(e, half), st);
    if (err != hipSuccess) return hip_fail(err, "hipMallocAsync(deep scratch)");
    uint4 *buf[2] = {(uint4 *)base, (uint4 *)(base + (size_t)maxlayer * rec)};
    J.ftab = (uint4 *)(base + 2 * (size_t)maxlayer * rec);
    J.out = out;
    int cur = 0;
    for (int t = e; t >= 0 && err == hipSuccess; t--) {
        J.t = t;
        J.nsub_c = (uint32_t)binom_host(e, (t + 1) / 2);
        J.nsub_o = (uint32_t)binom_host(e, t / 2);
        J.nodes = (uint32_t)(binom_host(e, t) * binom_host(t, (t + 1) / 2));
        J.cur = buf[cur];
        J.prev = buf[cur ^ 1];
        const uint32_t nsub = J.nsub_c + J.nsub_o;
        hipLaunchKernelGGL(deep_five_kernel, dim3((nsub + 255) / 256), dim3(256), 0, st, J, T);
        err = hipGetLastError();
        if (err != hipSuccess) break;
        if (half)
            hipLaunchKernelGGL(deep_node_kernel<true>, dim3((J.nodes + 255) / 256), dim3(256), 0, st, J, T);
        else
            hipLaunchKernelGGL(deep_node_kernel<false>, dim3((J.nodes + 255) / 256), dim3(256), 0, st, J, T);
        err = hipGetLastError();
        cur ^= 1;
    }
    (void)hipFreeAsync(base, st);
    if (err != hipSuccess) return hip_fail(err, "deep endgame launch");
    return 0;
}

}  // namespace pg

using namespace pg;

extern "C" int pentago_eval_deep(pentago_board board, pentago_superinfo *out, void *hip_stream)
{
    if (!out) return fail(PENTAGO_EINVAL, "out is NULL");
    const uint64_t packed = (uint64_t)board.q[0] | ((uint64_t)board.q[1] << 16) | ((uint64_t)board.q[2] << 32) |
                            ((uint64_t)board.q[3] << 48);
    return eval_deep_enqueue(packed, (uint4 *)out, (hipStream_t)hip_stream);
}

extern "C" int pentago_eval_deep_parity(pentago_board board, int parity, pentago_superinfo *out, void *hip_stream)
{
    if (!out) return fail(PENTAGO_EINVAL, "out is NULL");
    if (parity != 0 && parity != 1) return fail(PENTAGO_EINVAL, "parity must be 0 or 1");
    const uint64_t packed = (uint64_t)board.q[0] | ((uint64_t)board.q[1] << 16) | ((uint64_t)board.q[2] << 32) |
                            ((uint64_t)board.q[3] << 48);
    return eval_deep_enqueue(packed, (uint4 *)out, (hipStream_t)hip_stream, parity);
}
