// endgame.hip -- the endgame DAG solver (Section VIII) for batches of
// roots, its binning by empty cells, and the resident-section lookup.
#include "device_common.h"

namespace pg {

// ---------------------------------------------------------------------------
// Endgame DAG (Section VIII: the serial solver for boards beyond the
// database, rotations folded in by rmax only, no canonicalisation).
//
// For a root with e empty cells, node (t, cmask, omask) is the root with t
// more stones: the side to move at the root on the cells of cmask, the other
// side on omask.  Layers are solved from t = e (full board) down to t = 0.
// Each node keeps, for its parents, A = F_parent(node) | rmax(not N) and
// B = F_parent(node) | rmax(not W) (64 B) in a layer buffer.
// ---------------------------------------------------------------------------

// A root solved by a workgroup: two layers of node records (64 B each), then
// three five-set tables (the largest C(e, s) subsets, 32 B each): the two
// colours' tables of the current layer and, with 512 threads or more, the
// next layer's, computed while the current layer's nodes read the other two.
int dag_ftab_bytes(int e) { return 3 * dag_layout(e).max_subsets * 32; }

int dag_lds_bytes(int e)
{
    return 2 * dag_layout(e).max_layer * 64 + dag_ftab_bytes(e);
}

struct RootInfo {
    unsigned bm[4], wm[4];
    int code[4];
    int e;
    int mover;
    bool valid;
};

__device__ __forceinline__ RootInfo decode_root(uint64_t packed)
{
    RootInfo r;
    int nb = 0, nw = 0;
    r.valid = true;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        int code = (int)((packed >> (16 * j)) & 0xffff);
        r.code[j] = code;
        if (code >= 19683) { r.valid = false; code = 0; }
        unsigned bm = 0, wm = 0;
        int x = code;
        for (int l = 0; l < 9; l++) {
            const int dgt = x % 3;
            x /= 3;
            bm |= (unsigned)(dgt == 1) << l;
            wm |= (unsigned)(dgt == 2) << l;
        }
        r.bm[j] = bm;
        r.wm[j] = wm;
        nb += __popc(bm);
        nw += __popc(wm);
    }
    r.e = 36 - nb - nw;
    if (nb != nw && nb != nw + 1) r.valid = false;
    if (r.e > 10) r.valid = false;
    r.mover = nb == nw ? 1 : 2;
    return r;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Five-set of one board: the colour's stones xm0 plus the empty cells of
// subset m, stored as table entry r.  PL: the table is two planes of `smax`
// uint4 (entry r's halves at r and smax + r), else entries of two uint4.
template <bool PL>
__device__ __forceinline__ void five_entry(const DevTables &T, const unsigned xm0[4], unsigned m, int e,
                                           const int *s_slot_q, const int *s_slot_l, uint4 *tab, int smax,
                                           int r)
{
    unsigned xm[4] = {xm0[0], xm0[1], xm0[2], xm0[3]};
    for (int sl = 0; sl < e; sl++)
        if ((m >> sl) & 1) {
            const int q = s_slot_q[sl];
            const unsigned bit = 1u << s_slot_l[sl];
            xm[0] |= q == 0 ? bit : 0u;
            xm[1] |= q == 1 ? bit : 0u;
            xm[2] |= q == 2 ? bit : 0u;
            xm[3] |= q == 3 ? bit : 0u;
        }
    const Set256 F = board_five(T, xm);
    tab[PL ? r : 2 * r] = make_uint4(F.w[0], F.w[1], F.w[2], F.w[3]);
    tab[PL ? smax + r : 2 * r + 1] = make_uint4(F.w[4], F.w[5], F.w[6], F.w[7]);
}

// Solve one root with a group of GROUP threads: the whole workgroup (256 or
// 512) or a wave or part of one (64, 32, 16).  `buf0` and `buf1` hold
// two layers of A/B records, room for `cap` nodes each; `ftab` the five-set
// tables (three with 512 threads or more, else two); slot_q/slot_l (10 ints
// each, LDS) the root's empty cells.
//
// Five-sets: the nodes of layer t hold ceil(t/2) stones of the root's mover
// and floor(t/2) of the other side in the root's empty cells, and a colour's
// five-set depends only on which cells hold that colour.  So the five-set of
// every subset of the empty cells of those two sizes is tabled (C(e, s)
// boards per colour instead of one per node and colour), and each node reads
// its two.  From layer t to t - 1 one size stays (the mover's when t is
// even, the other side's when t is odd), so each layer tables one colour
// only: after the layer, over the table it replaces, or, with 512 threads or
// more, in the same pass as the layer's nodes, on the lanes the nodes leave
// free (a layer of 8 empty cells has up to 560 nodes, so the second pass of
// 512 lanes is mostly free), into the third table.
//
// Layouts: with 512 threads or more, records and tables are planes (node
// i's words 0-3 of A, 4-7 of A, 0-3 of B, 4-7 of B at [k * cap + i], so
// consecutive nodes take consecutive 16-byte slots); below, a node's record
// is four consecutive uint4 (measured: the planes' extra address arithmetic
// costs the smaller groups more than their LDS accesses gain).
template <int GROUP>
__device__ void solve_root(const RootInfo &R, const DevTables &T, uint4 *buf0, uint4 *buf1, int cap,
                           uint4 *ftab, uint4 *out, int *s_slot_q, int *s_slot_l)
{
    constexpr bool WG = GROUP >= 256;
    constexpr bool WIDE = GROUP >= 512;
    // GROUP < 64: a part of a wave; the other parts of the wave solve roots
    // with as many empty cells, so that every wave barrier below is reached
    // by all of them together
    const int lane = WG ? (int)threadIdx.x : (int)(threadIdx.x & (GROUP - 1));
    if (lane == 0) {
        int n = 0;
        for (int j = 0; j < 4; j++) {
            const unsigned empt = ~(R.bm[j] | R.wm[j]) & 0x1ffu;
            for (int l = 0; l < 9; l++)
                if ((empt >> l) & 1) {
                    s_slot_q[n] = j;
                    s_slot_l[n] = l;
                    n++;
                }
        }
    }
    if (WG) __syncthreads();
    else wave_sync();
    const int e = R.e;
    static_assert(kDagEdgeWords == 16, "edge records are two uint4");
    const uint4 *edges = T.dag_edge + 2 * T.dag_node_off[e];
    const uint16_t *smask = T.dag_sub_mask + T.dag_sub_off[e];
    const int *layer = T.dag_layer[e];
    const int *sstart = T.dag_sub_start[e];
    const int smax = T.dag_sub_max[e];
    // record piece j of node i, table half h of entry r
    const int rs = WIDE ? cap : 1, rn = WIDE ? 1 : 4;
    const int fs = WIDE ? smax : 1, fn = WIDE ? 1 : 2;
    // the root mover's stones and the other side's, per quadrant
    unsigned cm0[4], om0[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        cm0[j] = R.mover == 1 ? R.bm[j] : R.wm[j];
        om0[j] = R.mover == 1 ? R.wm[j] : R.bm[j];
    }
    // tables (2 * smax uint4 each): the root mover's subsets of the current
    // layer's size, the other side's, and (WIDE) the free one
    int tc = 0, to = 1, tf = 2;
    {
        const int sc = (e + 1) >> 1, so = e >> 1;
        const int nc = sstart[sc + 1] - sstart[sc], no = sstart[so + 1] - sstart[so];
        for (int i = lane; i < nc + no; i += GROUP) {
            const bool mine = i < nc;
            const int r = mine ? i : i - nc;
            five_entry<WIDE>(T, mine ? cm0 : om0, smask[sstart[mine ? sc : so] + r], e, s_slot_q, s_slot_l,
                             ftab + 2 * smax * (mine ? tc : to), smax, r);
        }
    }
    if (WG) __syncthreads();
    else wave_sync();
    uint4 *cur = buf0, *prev = buf1;
    for (int t = e; t >= 0; t--) {
        const int n0 = layer[t], nodes = layer[t + 1] - n0;
        const int x = (t & 1) ? 3 - R.mover : R.mover;   // side to move at layer t
        // the table that changes for layer t - 1: the mover's when t is odd
        const bool nmine = (t & 1) != 0;
        const int nsize = nmine ? t >> 1 : (t - 1) >> 1;
        const int nnext = t == 0 ? 0 : sstart[nsize + 1] - sstart[nsize];
        const uint4 *fc = ftab + 2 * smax * tc, *fo = ftab + 2 * smax * to;
        // the layer's nodes: each node's edge record (two 16-byte loads,
        // independent of one another) holds its five-set table entries and
        // the index of the child on each free slot; e - t children per node
        const int nfree = e - t;
        for (int k = lane; k < nodes + (WIDE ? nnext : 0); k += GROUP) {
            if (WIDE && k >= nodes) {
                const int r = k - nodes;
                five_entry<WIDE>(T, nmine ? cm0 : om0, smask[sstart[nsize] + r], e, s_slot_q, s_slot_l,
                                 ftab + 2 * smax * tf, smax, r);
                continue;
            }
            const int i = n0 + k;
            const uint4 ra = edges[2 * i], rb = edges[2 * i + 1];
            const uint32_t w[8] = {ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, rb.w};
            const uint32_t ic = w[0] & 0xffffu, io = w[0] >> 16;
            Set256 Fc, Fo;
            {
                const uint4 c0 = fc[fn * ic], c1 = fc[fn * ic + fs], o0 = fo[fn * io], o1 = fo[fn * io + fs];
                Fc.w[0] = c0.x; Fc.w[1] = c0.y; Fc.w[2] = c0.z; Fc.w[3] = c0.w;
                Fc.w[4] = c1.x; Fc.w[5] = c1.y; Fc.w[6] = c1.z; Fc.w[7] = c1.w;
                Fo.w[0] = o0.x; Fo.w[1] = o0.y; Fo.w[2] = o0.z; Fo.w[3] = o0.w;
                Fo.w[4] = o1.x; Fo.w[5] = o1.y; Fo.w[6] = o1.z; Fo.w[7] = o1.w;
            }
            const Set256 &Fx = x == R.mover ? Fc : Fo;
            const Set256 &Fy = x == R.mover ? Fo : Fc;
            Set256 Wnt = s_zero(), Nnt = s_zero();
            if (t == e) {
                Nnt = s_full();
            } else {
#pragma unroll
                for (int j = 0; j < 10; j++) {
                    if (j < nfree) {
                        const uint32_t ci = (w[1 + (j >> 1)] >> (16 * (j & 1))) & 0xffffu;
                        const uint4 *p = prev + rn * ci;
                        const uint4 a0 = p[0], a1 = p[rs], b0 = p[2 * rs], b1 = p[3 * rs];
                        Wnt.w[0] |= a0.x; Wnt.w[1] |= a0.y; Wnt.w[2] |= a0.z; Wnt.w[3] |= a0.w;
                        Wnt.w[4] |= a1.x; Wnt.w[5] |= a1.y; Wnt.w[6] |= a1.z; Wnt.w[7] |= a1.w;
                        Nnt.w[0] |= b0.x; Nnt.w[1] |= b0.y; Nnt.w[2] |= b0.z; Nnt.w[3] |= b0.w;
                        Nnt.w[4] |= b1.x; Nnt.w[5] |= b1.y; Nnt.w[6] |= b1.z; Nnt.w[7] |= b1.w;
                    }
                }
            }
            Set256 W, N;
            combine(Fx, Fy, Wnt, Nnt, W, N);
            if (t == 0) {
                store_info(out, W, N);
            } else {
                Set256 A, B;
                child_terms(Fy, W, N, A, B);
                uint4 *p = cur + rn * k;
                p[0] = make_uint4(A.w[0], A.w[1], A.w[2], A.w[3]);
                p[rs] = make_uint4(A.w[4], A.w[5], A.w[6], A.w[7]);
                p[2 * rs] = make_uint4(B.w[0], B.w[1], B.w[2], B.w[3]);
                p[3 * rs] = make_uint4(B.w[4], B.w[5], B.w[6], B.w[7]);
            }
        }
        if (WG) __syncthreads();
        else wave_sync();
        if (WIDE) {
            // the third table now holds the changing colour's; the old one is free
            const int old = nmine ? tc : to;
            if (nmine) tc = tf;
            else to = tf;
            tf = old;
        } else if (nnext > 0) {
            // the changing table, over the one it replaces
            for (int r = lane; r < nnext; r += GROUP)
                five_entry<WIDE>(T, nmine ? cm0 : om0, smask[sstart[nsize] + r], e, s_slot_q, s_slot_l,
                                 ftab + 2 * smax * (nmine ? tc : to), smax, r);
            if (WG) __syncthreads();
            else wave_sync();
        }
        uint4 *tmp = cur;
        cur = prev;
        prev = tmp;
    }
}

// Binning: each thread takes kBinPer boards (a workgroup 256 * kBinPer
// consecutive ones, coalesced per round), so that a workgroup's counts, kept
// in LDS, go to the global counters once per bin for that many boards: the
// global counters are twelve addresses, and every workgroup's atomics on
// them serialise.
constexpr int kBinPer = 8;

// Count roots per number of empty cells (index 11: invalid boards).
__global__ void __launch_bounds__(256)
    eval_count_kernel(const uint64_t *boards, size_t n, int *count, uint8_t *empties, int *status,
                      uint4 *out)
{
    __shared__ int lc[12];
    if (threadIdx.x < 12) lc[threadIdx.x] = 0;
    __syncthreads();
    for (int r = 0; r < kBinPer; r++) {
        const size_t i = ((size_t)blockIdx.x * kBinPer + r) * 256 + threadIdx.x;
        if (i >= n) break;
        const RootInfo R = decode_root(boards[i]);
        const int e = R.valid ? R.e : 11;
        empties[i] = (uint8_t)e;
        atomicAdd(&lc[e], 1);
        if (!R.valid) {
            const uint4 z = make_uint4(0, 0, 0, 0);
            out[4 * i] = z; out[4 * i + 1] = z; out[4 * i + 2] = z; out[4 * i + 3] = z;
        }
    }
    __syncthreads();
    if (threadIdx.x < 12 && lc[threadIdx.x]) {
        atomicAdd(&count[threadIdx.x], lc[threadIdx.x]);
        if (threadIdx.x == 11 && status) atomicAdd(status, lc[11]);
    }
}

// Bucket starts, most empty cells first.
__global__ void eval_scan_kernel(const int *count, int *start, int *cursor)
{
    if (threadIdx.x != 0) return;
    int acc = 0;
    for (int e = 10; e >= 0; e--) {
        start[e] = acc;
        cursor[e] = 0;
        acc += count[e];
    }
    start[11] = acc;
    cursor[11] = 0;
}

// Roots into their bins: positions inside the workgroup from LDS counters,
// one global reservation per bin per workgroup.
__global__ void __launch_bounds__(256)
    eval_scatter_kernel(const uint8_t *empties, size_t n, const int *start, int *cursor, int *order)
{
    __shared__ int lc[11], base[11];
    if (threadIdx.x < 11) lc[threadIdx.x] = 0;
    __syncthreads();
    int ee[kBinPer], local[kBinPer];
#pragma unroll
    for (int r = 0; r < kBinPer; r++) {
        const size_t i = ((size_t)blockIdx.x * kBinPer + r) * 256 + threadIdx.x;
        ee[r] = i < n ? empties[i] : 11;
        local[r] = ee[r] <= 10 ? atomicAdd(&lc[ee[r]], 1) : 0;
    }
    __syncthreads();
    if (threadIdx.x < 11 && lc[threadIdx.x]) base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], lc[threadIdx.x]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kBinPer; r++) {
        const size_t i = ((size_t)blockIdx.x * kBinPer + r) * 256 + threadIdx.x;
        if (ee[r] <= 10) order[start[ee[r]] + base[ee[r]] + local[r]] = (int)i;
    }
}

__global__ void zero_ints_kernel(int *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Persistent solve over all valid roots, most empty cells first.  The roots
// are binned by number of empty cells on the device; three persistent
// launches follow one another on the stream, one per LDS class, each taking
// roots from its own device work queue (no host synchronisation):
//   class 0: 8 to 10 empty cells, a workgroup per root (9 and 10 keep their
//            layers in the workgroup's slot of a global buffer; only the
//            first `slots` workgroups own a slot: they take the 9-10 queue
//            first, then join the others on the 8-empty queue);
//   class 1: 7 empty cells, a workgroup per root, a smaller LDS footprint;
//   class 2: up to kWaveMaxEmpties, synchronised per wave only: a wave
//            solves eight roots with up to 3 empty cells at once (8 lanes
//            each), four with 4 (16 lanes), two with 5 (32 lanes) or one
//            with 6, each on its own part of the wave's LDS.
constexpr int kWaveMaxEmpties = 6;
// two layers of the widest 6-empty layer, then the five-set tables (C(6,3) = 20)
constexpr int kWaveLdsBytes = 2 * 90 * 64 + 2 * 20 * 32;

template <int CLS, int NT>
__global__ void __launch_bounds__(NT)
    eval_persistent_kernel(const uint64_t *boards, const int *order, const int *start,
                           unsigned long long *counter, uint4 *out, uint4 *gl, int slots, DevTables T)
{
    extern __shared__ uint4 lds[];
    __shared__ long long s_item;
    __shared__ int s_slots[4][2][10];
    // bins are ordered by empty cells, most first: e occupies [start[e], start[e - 1])
    const int lo = CLS == 0 ? 0 : CLS == 1 ? start[7] : start[kWaveMaxEmpties];
    const int hi = CLS == 0 ? start[7] : CLS == 1 ? start[kWaveMaxEmpties] : start[11];
    if constexpr (CLS < 2) {
        // class 0: roots with 9 or 10 empty cells, [0, big), come from queue 3
        // and only go to workgroups that own a global layer slot; the rest of
        // the class, [big, hi), from queue 0.  Class 1 uses queue 1 only.
        const int big = CLS == 0 ? start[8] : lo;
        if (CLS == 0 && (int)blockIdx.x < slots) {
            uint4 *mine = gl + (size_t)blockIdx.x * 2 * 4 * kDagGlobalLayer;
            for (;;) {
                if (threadIdx.x == 0) s_item = (long long)atomicAdd(&counter[3], 1ull);
                __syncthreads();
                const long long item = s_item;
                __syncthreads();
                if (item >= big) break;
                const int root = order[item];
                const RootInfo R = decode_root(boards[root]);
                solve_root<NT>(R, T, mine, mine + 4 * kDagGlobalLayer, kDagGlobalLayer, lds, out + 4 * (size_t)root,
                                s_slots[0][0], s_slots[0][1]);
                __syncthreads();
            }
        }
        for (;;) {
            if (threadIdx.x == 0) s_item = (long long)atomicAdd(&counter[CLS], 1ull);
            __syncthreads();
            const long long item = big + s_item;
            __syncthreads();
            if (item >= hi) break;
            const int root = order[item];
            const RootInfo R = decode_root(boards[root]);
            solve_root<NT>(R, T, lds, lds + 4 * T.dag_max[R.e], T.dag_max[R.e], lds + 8 * T.dag_max[R.e],
                            out + 4 * (size_t)root, s_slots[0][0], s_slots[0][1]);
            __syncthreads();
        }
    } else {
        // A wave takes a chunk of K roots of one bin (K = 8 up to 3 empty
        // cells, 4 for 4, 2 for 5, 1 for 6: the widest layers have 6, 12, 30
        // and 90 nodes); the roots of a chunk have the same layers, so the wave
        // synchronises them together.  Chunks are numbered bin by bin, most
        // empty cells first; the last chunk of a bin repeats the bin's last
        // root where it runs short (the copy writes the same bytes).
        __shared__ int s_sub[4][8][2][kWaveMaxEmpties];
        (void)lo;
        (void)hi;
        const int w = threadIdx.x >> 6, wl = threadIdx.x & 63;
        uint4 *wb = lds + (size_t)w * (kWaveLdsBytes / 16);
        for (;;) {
            unsigned long long got = 0;
            if (wl == 0) got = atomicAdd(&counter[2], 1ull);
            const long long c = (long long)__shfl(got, 0, 64);
            int e = -1, K = 1, base = 0, last = 0;
            long long cum = 0;
            for (int b = kWaveMaxEmpties; b >= 0; b--) {
                const int blo = start[b], bhi = b == 0 ? start[11] : start[b - 1];
                const int kb = b <= 3 ? 8 : b == 4 ? 4 : b == 5 ? 2 : 1;
                const long long nch = (bhi - blo + kb - 1) / kb;
                if (e < 0 && c < cum + nch) {
                    e = b;
                    K = kb;
                    base = blo + (int)(c - cum) * kb;
                    last = bhi - 1;
                }
                cum += nch;
            }
            if (e < 0) break;
            const int g = wl / (64 / K);
            const int root = order[min(base + g, last)];
            const RootInfo R = decode_root(boards[root]);
            uint4 *o = out + 4 * (size_t)root;
            if (K == 8) {
                uint4 *sb = wb + g * 100;   // 1.6 KB each: layers of 6 nodes, tables of 3 subsets
                solve_root<8>(R, T, sb, sb + 4 * 6, 6, sb + 8 * 6, o, s_sub[w][g][0], s_sub[w][g][1]);
            } else if (K == 4) {
                uint4 *sb = wb + g * 200;   // 3.2 KB each: layers of 12 nodes, tables of 6 subsets
                solve_root<16>(R, T, sb, sb + 4 * 12, 12, sb + 8 * 12, o, s_sub[w][g][0], s_sub[w][g][1]);
            } else if (K == 2) {
                uint4 *sb = wb + g * 400;   // 6.4 KB each: layers of 30 nodes, tables of 10 subsets
                solve_root<32>(R, T, sb, sb + 4 * 30, 30, sb + 8 * 30, o, s_sub[w][g][0], s_sub[w][g][1]);
            } else {
                solve_root<64>(R, T, wb, wb + 4 * 90, 90, wb + 8 * 90, o, s_sub[w][0][0], s_sub[w][0][1]);
            }
            wave_sync();
        }
    }
}

// A batch whose roots all fall in one class (the server batches its searches
// by empty cells): the roots are taken in order from one device queue, with
// no binning pass.  Boards the class cannot hold get zero tables.
template <int CLS>
__global__ void __launch_bounds__(256)
    eval_direct_kernel(const uint64_t *boards, int n, unsigned long long *counter, uint4 *out,
                       uint4 *gl, DevTables T)
{
    extern __shared__ uint4 lds[];
    __shared__ long long s_item;
    __shared__ int s_slots[4][2][10];
    if (CLS < 2) {
        uint4 *mine = gl + (size_t)blockIdx.x * 2 * 4 * kDagGlobalLayer;
        for (;;) {
            if (threadIdx.x == 0) s_item = (long long)atomicAdd(counter, 1ull);
            __syncthreads();
            const long long item = s_item;
            __syncthreads();
            if (item >= n) break;
            const RootInfo R = decode_root(boards[item]);
            const bool ok = R.valid && (CLS == 0 ? (R.e >= 8 && (R.e == 8 || gl != nullptr)) : R.e == 7);
            if (!ok) {
                if (threadIdx.x < 4) out[4 * item + threadIdx.x] = make_uint4(0, 0, 0, 0);
            } else if (CLS == 0 && R.e > 8) {
                solve_root<256>(R, T, mine, mine + 4 * kDagGlobalLayer, kDagGlobalLayer, lds, out + 4 * (size_t)item,
                                s_slots[0][0], s_slots[0][1]);
            } else {
                solve_root<256>(R, T, lds, lds + 4 * T.dag_max[R.e], T.dag_max[R.e], lds + 8 * T.dag_max[R.e],
                                out + 4 * (size_t)item, s_slots[0][0], s_slots[0][1]);
            }
            __syncthreads();
        }
    } else {
        const int w = threadIdx.x >> 6;
        uint4 *wb = lds + (size_t)w * (kWaveLdsBytes / 16);
        for (;;) {
            unsigned long long got = 0;
            if ((threadIdx.x & 63) == 0) got = atomicAdd(counter, 1ull);
            const long long item = (long long)__shfl(got, 0, 64);
            if (item >= n) break;
            const RootInfo R = decode_root(boards[item]);
            if (!R.valid || R.e > kWaveMaxEmpties) {
                if ((threadIdx.x & 63) < 4) out[4 * item + (threadIdx.x & 3)] = make_uint4(0, 0, 0, 0);
            } else {
                solve_root<64>(R, T, wb, wb + 4 * 90, 90, wb + 8 * 90, out + 4 * (size_t)item, s_slots[w][0],
                               s_slots[w][1]);
            }
            wave_sync();
        }
    }
}

// Plain form: the roots of one empties group, one workgroup per root
// (grid-stride when the group needs global layer buffers).
__global__ void __launch_bounds__(256)
    eval_group_kernel(const uint64_t *boards, const int *order, int first, int count, uint4 *out,
                      uint4 *gl, int use_global, DevTables T)
{
    extern __shared__ uint4 lds[];
    __shared__ int s_slots[2][10];
    uint4 *mine = gl + (size_t)blockIdx.x * 2 * 4 * kDagGlobalLayer;
    for (int item = blockIdx.x; item < count; item += gridDim.x) {
        const int root = order[first + item];
        const RootInfo R = decode_root(boards[root]);
        if (use_global)
            solve_root<256>(R, T, mine, mine + 4 * kDagGlobalLayer, kDagGlobalLayer, lds, out + 4 * (size_t)root,
                            s_slots[0], s_slots[1]);
        else
            solve_root<256>(R, T, lds, lds + 4 * T.dag_max[R.e], T.dag_max[R.e], lds + 8 * T.dag_max[R.e],
                            out + 4 * (size_t)root, s_slots[0], s_slots[1]);
        __syncthreads();
    }
}

// Resident-section lookup (Section VIII: positions inside the database are
// read, not solved): each quadrant of the query is turned to its
// rotation-minimal pattern (k_j turns), the entry is read and shifted back by
// k_j along every dimension.  When the query's section is the image of the
// resident one under a board symmetry (Section IV keeps only one section of
// each D4 class), the query is first mapped back to its preimage in the
// resident section's frame, and the result is carried over to the query by
// the symmetry's table transform (no turns: h = 0).
__global__ void __launch_bounds__(256)
    lookup_kernel(const uint64_t *boards, const int *sec_of, int n, const ResidentSection *secs,
                  uint4 *out, DevTables T)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t b = boards[i];
    const int code = sec_of[i];
    const ResidentSection S = secs[code & 0xffffff];
    const int sym = code >> 24;
    int idx[4], k[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        // quadrant j of the query's preimage in the resident section's frame
        const int q = sym_quadrant(sym, j);
        const uint32_t c = (uint32_t)(b >> (16 * q)) & 0xffffu;
        const uint16_t cc = T.canon[sym ? T.symcode[sym * 19683 + c] : c];
        idx[j] = cc & 0xfff;
        k[j] = cc >> 12;
    }
    Set256 W, N;
    load_info(S.table + 4 * block_offset(S.m, idx), W, N);
#pragma unroll
    for (int j = 0; j < 4; j++) {
        W = shift_dim(W, j, k[j]);
        N = shift_dim(N, j, k[j]);
    }
    if (sym) {
        // the query is the symmetry's image of that preimage (Section III:
        // values are invariant under board symmetries)
        const int h0[4] = {0, 0, 0, 0};
        sym_apply_rt2(W, N, sym, h0);
    }
    store_info(out + 4 * (size_t)i, W, N);
}

hipError_t launch_lookup(const uint64_t *boards, const int *sec_of, int n,
                         const ResidentSection *secs, uint4 *out, const DevTables &T, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(lookup_kernel, dim3((n + 255) / 256), dim3(256), 0, s, boards, sec_of, n,
                       secs, out, T);
    return hipGetLastError();
}

hipError_t launch_eval_bin(const uint64_t *boards, size_t n, const EvalScratch &S, int *status,
                           uint4 *out, const DevTables &T, hipStream_t s)
{
    (void)T;
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, s, S.count, 16);
    if (n) {
        const unsigned g = (unsigned)((n + 256 * kBinPer - 1) / (256 * kBinPer));
        hipLaunchKernelGGL(eval_count_kernel, dim3(g), dim3(256), 0, s, boards, n, S.count,
                           S.empties, status, out);
    }
    hipLaunchKernelGGL(eval_scan_kernel, dim3(1), dim3(64), 0, s, S.count, S.start, S.cursor);
    if (n) {
        const unsigned g = (unsigned)((n + 256 * kBinPer - 1) / (256 * kBinPer));
        hipLaunchKernelGGL(eval_scatter_kernel, dim3(g), dim3(256), 0, s, S.empties, n, S.start,
                           S.cursor, S.order);
    }
    return hipGetLastError();
}

// Dynamic LDS of each persistent class.
static int eval_class_lds_bytes(int cls)
{
    if (cls == 0) return std::max(dag_lds_bytes(8), std::max(dag_ftab_bytes(9), dag_ftab_bytes(10)));
    if (cls == 1) return dag_lds_bytes(7);
    return 4 * kWaveLdsBytes;
}

// Dynamic LDS above 64 KiB has to be granted per kernel.
static hipError_t allow_lds(const void *kernel, int bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_eval_persistent(const uint64_t *boards, size_t n, uint4 *out,
                                  const EvalScratch &S, int grid, const DevTables &T,
                                  hipStream_t s)
{
    return launch_eval_persistent_slots(boards, n, out, S, grid, grid, T, s);
}

// Workgroup size of the persistent classes 0 and 1 (256 or 512 threads per
// root; class 2 solves roots by waves in 256-thread workgroups).
static int g_class_threads[2] = {512, 256};

void set_eval_class_threads(int c0, int c1)
{
    g_class_threads[0] = c0;
    g_class_threads[1] = c1;
}

void get_eval_class_threads(int *c0, int *c1)
{
    *c0 = g_class_threads[0];
    *c1 = g_class_threads[1];
}

template <int CLS, int NT>
static hipError_t launch_class(int g, int lds, hipStream_t s, const uint64_t *boards, const EvalScratch &S,
                               uint4 *out, int slots, const DevTables &T)
{
    const hipError_t e = allow_lds((const void *)eval_persistent_kernel<CLS, NT>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((eval_persistent_kernel<CLS, NT>), dim3(g), dim3(NT), lds, s, boards, S.order, S.start,
                       S.counter, out, S.global_layers, slots, T);
    return hipGetLastError();
}

template <int CLS, int NT>
static int class_blocks_per_cu(int lds)
{
    int per = 0;
    (void)allow_lds((const void *)eval_persistent_kernel<CLS, NT>, lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)eval_persistent_kernel<CLS, NT>, NT,
                                                     lds) != hipSuccess)
        return 1;
    return std::max(1, per);
}

hipError_t launch_eval_persistent_slots(const uint64_t *boards, size_t n, uint4 *out,
                                        const EvalScratch &S, int grid, int slots,
                                        const DevTables &T, hipStream_t s)
{
    (void)n;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (slots < 1 || slots > grid) return hipErrorInvalidValue;
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, s, S.counter, 4);
    // class 0: `grid` workgroups (two per CU: the LDS of an 8-empty root),
    // the first `slots` of them owning a global layer slot each
    const int lds0 = eval_class_lds_bytes(0), lds1 = eval_class_lds_bytes(1), lds2 = eval_class_lds_bytes(2);
    e = g_class_threads[0] == 512 ? launch_class<0, 512>(grid, lds0, s, boards, S, out, slots, T)
                                  : launch_class<0, 256>(grid, lds0, s, boards, S, out, slots, T);
    if (e != hipSuccess) return e;
    if (g_class_threads[1] == 512)
        e = launch_class<1, 512>(class_blocks_per_cu<1, 512>(lds1) * cus, lds1, s, boards, S, out, slots, T);
    else
        e = launch_class<1, 256>(class_blocks_per_cu<1, 256>(lds1) * cus, lds1, s, boards, S, out, slots, T);
    if (e != hipSuccess) return e;
    return launch_class<2, 256>(class_blocks_per_cu<2, 256>(lds2) * cus, lds2, s, boards, S, out, slots, T);
}

hipError_t launch_eval_direct(const uint64_t *boards, int n, uint4 *out, int cls,
                              unsigned long long *counter, uint4 *global_layers, int grid,
                              const DevTables &T, hipStream_t s)
{
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const void *kern[3] = {(const void *)eval_direct_kernel<0>, (const void *)eval_direct_kernel<1>,
                           (const void *)eval_direct_kernel<2>};
    const int lds = eval_class_lds_bytes(cls);
    e = allow_lds(kern[cls], lds);
    if (e != hipSuccess) return e;
    int g = grid;  // class 0 owns the global layer slots: one per workgroup of `grid`
    if (cls > 0) {
        int per = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern[cls], 256, lds);
        if (e != hipSuccess) return e;
        g = std::max(1, per) * cus;
    }
    // no more workgroups than the batch can use
    g = std::min(g, cls == 2 ? (n + 3) / 4 : n);
    if (g <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, s, counter, 1);
    switch (cls) {
    case 0: hipLaunchKernelGGL(eval_direct_kernel<0>, dim3(g), dim3(256), lds, s, boards, n, counter, out,
                               global_layers, T); break;
    case 1: hipLaunchKernelGGL(eval_direct_kernel<1>, dim3(g), dim3(256), lds, s, boards, n, counter, out,
                               global_layers, T); break;
    default: hipLaunchKernelGGL(eval_direct_kernel<2>, dim3(g), dim3(256), lds, s, boards, n, counter, out,
                                global_layers, T); break;
    }
    return hipGetLastError();
}

hipError_t launch_eval_group(const uint64_t *boards, int e, int first, int count, uint4 *out,
                             const EvalScratch &S, const DevTables &T, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const bool global = e > 8;
    const int grid = global ? std::min(count, S.global_slots) : count;
    const int lds = global ? dag_ftab_bytes(e) : dag_lds_bytes(e);
    const hipError_t err = allow_lds((const void *)eval_group_kernel, lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(eval_group_kernel, dim3(grid), dim3(256), lds, s,
                       boards, S.order, first, count, out, S.global_layers, global ? 1 : 0, T);
    return hipGetLastError();
}

}  // namespace pg
