// kernels.hip -- HIP kernels for gfx950: the section sweep (Sections II-IV)
// and the endgame DAG solver (Section VIII).
//
// Data layout in HBM: a section table is entries x 64 B superinfos (win
// words then not-lose words) in the 8^4-blocked order of Section IV.  One
// lane owns one entry and keeps each 256-bit set in eight VGPRs, so every
// set operation is plain per-lane integer work; nothing here is a dense
// contraction, so there is no MFMA.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace pg {

__constant__ uint32_t c_pow3[10] = {1, 3, 9, 27, 81, 243, 729, 2187, 6561, 19683};

// Entry offset in the 8^4-blocked layout (see pentago_section_offset).  The
// host rejects sections of 2^32 entries or more, so 32-bit arithmetic holds.
__device__ __forceinline__ uint32_t block_offset(const int *m, const int *idx)
{
    uint32_t B[4], r[4], s[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        B[j] = (uint32_t)idx[j] >> 3;
        r[j] = (uint32_t)idx[j] & 7u;
        s[j] = min(8u, (uint32_t)m[j] - 8u * B[j]);
    }
    const uint32_t m23 = (uint32_t)m[2] * (uint32_t)m[3];
    uint32_t off = 8u * B[0] * (uint32_t)m[1] * m23;
    off += s[0] * 8u * B[1] * m23;
    off += s[0] * s[1] * 8u * B[2] * (uint32_t)m[3];
    off += s[0] * s[1] * s[2] * 8u * B[3];
    off += ((r[0] * s[1] + r[1]) * s[2] + r[2]) * s[3] + r[3];
    return off;
}

// block_offset along a line of dimension D: with every index but idx[D]
// fixed, the offset is c0 + c1 * B + c2 * s + c3 * r for B = idx[D] >> 3,
// r = idx[D] & 7 and s = min(8, m[D] - 8 B) (the extent of that block).
template <int D>
__device__ __forceinline__ uint4 line_offset_coeffs(const int *m, const int *idx)
{
    uint32_t B[4], r[4], s[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        B[j] = (uint32_t)idx[j] >> 3;
        r[j] = (uint32_t)idx[j] & 7u;
        s[j] = min(8u, (uint32_t)m[j] - 8u * B[j]);
    }
    uint32_t c0 = 0, c1 = 8, c2 = 0, c3 = 1;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        uint32_t lo = 1, lo_d = 1, hi_m = 1, hi_s = 1, hi_s_d = 1;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            if (i < j) { lo *= s[i]; if (i != D) lo_d *= s[i]; }
            if (i > j) { hi_m *= (uint32_t)m[i]; hi_s *= s[i]; if (i != D) hi_s_d *= s[i]; }
        }
        if (j < D) {
            c0 += lo * 8u * B[j] * hi_m;   // whole blocks before, in dimensions < D
            c2 += r[j] * hi_s_d;           // in-block index terms that carry s_D
        } else if (j == D) {
            c1 = lo * 8u * hi_m;
            c3 = hi_s;
        } else {
            c2 += lo_d * 8u * B[j] * hi_m;  // whole blocks in dimensions > D carry s_D
            c0 += r[j] * hi_s;
        }
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ void load_info(const uint4 *p, Set256 &W, Set256 &N)
{
    const uint4 a = p[0], b = p[1], c = p[2], d = p[3];
    W.w[0] = a.x; W.w[1] = a.y; W.w[2] = a.z; W.w[3] = a.w;
    W.w[4] = b.x; W.w[5] = b.y; W.w[6] = b.z; W.w[7] = b.w;
    N.w[0] = c.x; N.w[1] = c.y; N.w[2] = c.z; N.w[3] = c.w;
    N.w[4] = d.x; N.w[5] = d.y; N.w[6] = d.z; N.w[7] = d.w;
}

__device__ __forceinline__ void store_info(uint4 *p, const Set256 &W, const Set256 &N)
{
    p[0] = make_uint4(W.w[0], W.w[1], W.w[2], W.w[3]);
    p[1] = make_uint4(W.w[4], W.w[5], W.w[6], W.w[7]);
    p[2] = make_uint4(N.w[0], N.w[1], N.w[2], N.w[3]);
    p[3] = make_uint4(N.w[4], N.w[5], N.w[6], N.w[7]);
}

__device__ __forceinline__ Set256 board_five(const DevTables &T, const unsigned xm[4])
{
    const LineMasks l0 = T.lm[0 * 512 + xm[0]];
    const LineMasks l1 = T.lm[1 * 512 + xm[1]];
    const LineMasks l2 = T.lm[2 * 512 + xm[2]];
    const LineMasks l3 = T.lm[3 * 512 + xm[3]];
    return five_set(l0, l1, l2, l3);
}

// ---------------------------------------------------------------------------
// Section sweep
// ---------------------------------------------------------------------------

// Index helpers: runtime dimension numbers only ever select among the four
// registers (never index a local array, which would go to scratch).
struct Idx4 {
    int v[4];
};

__device__ __forceinline__ int get4(const Idx4 &x, int j)
{
    return j == 0 ? x.v[0] : j == 1 ? x.v[1] : j == 2 ? x.v[2] : x.v[3];
}

__device__ __forceinline__ void set4(Idx4 &x, int j, int val)
{
#pragma unroll
    for (int i = 0; i < 4; i++)
        if (i == j) x.v[i] = val;
}

__device__ __forceinline__ int mdim(const SweepJob &J, int j)
{
    return j == 0 ? J.m[0] : j == 1 ? J.m[1] : j == 2 ? J.m[2] : J.m[3];
}

// A child entry's contribution, prepared once per child entry of a staged
// line and used by every parent of the line that reaches it (Section III:
// rmax is translation invariant, so it commutes with the canonicalising
// shift; the immediate-win set of the placement is the child's own five-set
// of the parent's colour, shifted the same way).
//   A = F_c(child) | rmax(not N_child),  B = F_c(child) | rmax(not W_child)
// JD is the child's dimension (the quadrant that received the stone).
template <int JD>
__device__ __forceinline__ void child_entry_terms(const SweepJob &J, const DevTables &T,
                                                  const Idx4 &idx, Set256 &A, Set256 &B)
{
    const int c = J.mover;
    unsigned cm_[4], om_[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const QInfo q = T.qinfo[(j == JD ? J.cqb[j] : J.qb[j]) + idx.v[j]];
        cm_[j] = c == 1 ? q.bm : q.wm;
        om_[j] = c == 1 ? q.wm : q.bm;
    }
    Set256 W, N;
    if ((J.odmask >> JD) & 1) {
        // a full board with the other side to move: value f_o - f_c (Section II)
        const Set256 Fc = board_five(T, cm_);
        const Set256 Fo = board_five(T, om_);
#pragma unroll
        for (int i = 0; i < 8; i++) {
            W.w[i] = Fo.w[i] & ~Fc.w[i];
            N.w[i] = Fo.w[i] | ~Fc.w[i];
        }
    } else {
        int cshape[4] = {J.m[0], J.m[1], J.m[2], J.m[3]};
        cshape[JD] = J.cm[JD];
        load_info(J.child[JD] + 4 * block_offset(cshape, idx.v), W, N);
    }
    const Set256 Fc = board_five(T, cm_);
    child_terms(Fc, W, N, A, B);
}

__device__ __forceinline__ Set256 set_from(const uint4 *p)
{
    Set256 x;
    const uint4 u = p[0], v = p[1];
    x.w[0] = u.x; x.w[1] = u.y; x.w[2] = u.z; x.w[3] = u.w;
    x.w[4] = v.x; x.w[5] = v.y; x.w[6] = v.z; x.w[7] = v.w;
    return x;
}

// ---------------------------------------------------------------------------
// Five-in-a-row sets along a line (Section III five-sets, Section IV lines).
//
// Inside a tile every entry of one line shares the patterns of the three
// quadrants other than D; only quadrant D varies.  The sweep works in an
// internal layout where dimension D is exchanged with dimension 3, so for a
// fixed turn k of quadrant D the five-set is one 64-bit word pair over the
// other three dimensions:
//   F[k] = U | OR over lines l through D that quadrant D completes at k of O_l
// where U collects the lines missing D and O_l is the product of l's
// cylinders in the other quadrants it touches.  The 17 lines through D are
// split into the three chunks of quadrant D's LineMasks (6 slots each), and
// each chunk gets a 64-entry table over subsets of its lines, so F[k] is
// three table reads.  The selectors (which lines D completes at k) depend
// only on D's pattern and come from T.sel.
// ---------------------------------------------------------------------------

// LDS layout of one tile.  Per tile: the selectors of every position along D
// for both colours, stored as [turn k][position] pairs (sel_c, sel_o) with a
// row stride that puts the four turns of one position in different banks;
// the children of every position; the selectors of the child positions.  Per
// line: the chunk tables for both colours, the partial sets (18 chunk lines +
// U) for both colours and the LineMasks of the 4 quadrants for both colours.
// Child records (A then B in the internal layout, 2 dwords of padding) are
// indexed [child position][line], so consecutive lanes of the child pass
// write consecutive records.
constexpr int kOSlots = 19;                    // 18 chunk lines + U
constexpr int kLutStride = 2 * 3 * 64 + 1;    // uint2 per line; +1 staggers the banks of lines
constexpr int kRecWords = 18;

struct PosChild {
    uint16_t nchild, child[9];   // child index | k << 12 per empty cell
};
struct ChildPosRec {
    uint4 sel_c, sel_o;
};

__host__ __device__ __forceinline__ int sel_stride(int mD) { return ((mD + 15) & ~31) + 16; }

struct TileLds {
    ChildPosRec *cpos;  // [cmD]
    uint2 *sel;         // [4][sel_stride(mD)]
    uint2 *lut;         // [G][kLutStride]
    uint2 *O;           // [G][2][kOSlots]
    uint32_t *rec;      // [cmD][G][kRecWords]
    LineMasks *lmq;     // [G][2][4]
    uint4 *loff;        // [G] line_offset_coeffs of each line
    PosChild *pch;      // [mD]
};

__host__ __device__ __forceinline__ int tile_lds_bytes(int G, int mD, int cmD, TileLds *L, char *base)
{
    int off = 0;
    if (L) L->cpos = (ChildPosRec *)(base + off);
    off += cmD * (int)sizeof(ChildPosRec);
    if (L) L->sel = (uint2 *)(base + off);
    off += 4 * sel_stride(mD) * 8;
    if (L) L->lut = (uint2 *)(base + off);
    off += G * kLutStride * 8;
    if (L) L->O = (uint2 *)(base + off);
    off += G * 2 * kOSlots * 8;
    if (L) L->rec = (uint32_t *)(base + off);
    off += cmD * G * kRecWords * 4;
    if (L) L->lmq = (LineMasks *)(base + off);
    off += G * 8 * (int)sizeof(LineMasks);
    if (L) L->loff = (uint4 *)(base + off);
    off += G * 16;
    if (L) L->pch = (PosChild *)(base + off);
    off += mD * (int)sizeof(PosChild);
    return off;
}

__device__ __forceinline__ TileLds tile_lds(void *base, int G, int mD, int cmD)
{
    TileLds L;
    tile_lds_bytes(G, mD, cmD, &L, (char *)base);
    return L;
}

// A line reference: quadrant j (bits 0-1), LineMasks field f (bits 2-3) and
// nibble i (bits 4-7); 0xff stands for no quadrant.  ref_cyl gives the
// cylinder over the internal dimension of quadrant j of the turns after
// which the line's cells in quadrant j hold the colour (all of L for 0xff).
// Branch-free, as the lanes of a wave carry different references.
template <int D>
__device__ __forceinline__ uint2 ref_cyl(const LineMasks *lmq, uint32_t ref)
{
    const bool none = ref == 0xffu;
    const uint32_t j = ref & 3, f = (ref >> 2) & 3;
    const uint32_t fld = ((const uint32_t *)(lmq + j))[none ? 0 : f];
    const uint32_t m = none ? 0xfu : (fld >> (4 * (ref >> 4))) & 0xfu;
    // internal position of quadrant j when D is exchanged with 3
    const uint32_t p = j == 3 ? (uint32_t)D : j;
    const uint32_t c0 = m * 0x1111u;          // p = 0: a set of g0, every g1
    const uint32_t c1 = spread1(m) * 0xfu;    // p = 1: a set of g1, every g0
    const uint32_t h = p == 0 ? c0 : c1;
    const uint32_t lo = ((m & 1u) ? 0x0000ffffu : 0u) | ((m & 2u) ? 0xffff0000u : 0u);
    const uint32_t hi = ((m & 4u) ? 0x0000ffffu : 0u) | ((m & 8u) ? 0xffff0000u : 0u);
    const uint32_t hh = h | (h << 16);
    return p == 2 && !none ? make_uint2(lo, hi) : make_uint2(hh, hh);
}

// Product of the cylinders of up to three references (refs: one per byte).
template <int D>
__device__ __forceinline__ uint2 ref_product3(const LineMasks *lmq, uint32_t refs)
{
    const uint2 a = ref_cyl<D>(lmq, refs & 0xffu);
    const uint2 b = ref_cyl<D>(lmq, (refs >> 8) & 0xffu);
    const uint2 c = ref_cyl<D>(lmq, (refs >> 16) & 0xffu);
    return make_uint2(a.x & b.x & c.x, a.y & b.y & c.y);
}

// Five-set of a board of the line from the line's chunk tables and the
// selectors of its quadrant-D pattern (internal layout).
__device__ __forceinline__ Set256 five_lut(const uint2 *lut, const uint4 sel)
{
    Set256 F;
    const uint32_t s4[4] = {sel.x, sel.y, sel.z, sel.w};
    const char *base = (const char *)lut;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const uint2 a = *(const uint2 *)(base + (s4[k] & 1023u));
        const uint2 b = *(const uint2 *)(base + ((s4[k] >> 10) & 1023u));
        const uint2 c = *(const uint2 *)(base + (s4[k] >> 20));
        F.w[2 * k] = a.x | b.x | c.x;
        F.w[2 * k + 1] = a.y | b.y | c.y;
    }
    return F;
}

// OR into acc the 8-word set at p shifted by k along internal dimension 3
// (a re-addressing of the four word pairs).
__device__ __forceinline__ void or_rotated(Set256 &acc, const uint32_t *p, int k)
{
#pragma unroll
    for (int g3 = 0; g3 < 4; g3++) {
        const uint2 v = *(const uint2 *)(p + 2 * ((g3 - k) & 3));
        acc.w[2 * g3] |= v.x;
        acc.w[2 * g3 + 1] |= v.y;
    }
}

// ---------------------------------------------------------------------------
// Stores of the parent pass.  Each lane computes one parent entry (64 B, four
// 16-byte pieces).  The four lanes of a quad then transpose their pieces in
// registers (two exchange stages of DPP quad permutations), so that in each
// of four store instructions the quad writes one whole entry and the 16 quads
// of a wave write 16 neighbouring entries: full, contiguous 1 KB stores.
// ---------------------------------------------------------------------------

template <int CTRL>
__device__ __forceinline__ uint32_t quad_perm(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, true);
}

// quad lanes [1,0,3,2] (X = 1) or [2,3,0,1] (X = 2)
template <int X>
__device__ __forceinline__ uint4 quad_xor(uint4 a)
{
    constexpr int ctrl = X == 1 ? 0xB1 : 0x4E;
    return make_uint4(quad_perm<ctrl>(a.x), quad_perm<ctrl>(a.y), quad_perm<ctrl>(a.z), quad_perm<ctrl>(a.w));
}

// One exchange stage: slot p of lane l takes slot p ^ X of lane l ^ X when
// bit X of l differs from bit X of p.
template <int X>
__device__ __forceinline__ void quad_stage(uint4 (&r)[4], int l)
{
    uint4 t[4];
#pragma unroll
    for (int p = 0; p < 4; p++) t[p] = quad_xor<X>(r[p ^ X]);
#pragma unroll
    for (int p = 0; p < 4; p++)
        if ((l ^ p) & X) r[p] = t[p];
}

// After this, slot p of quad lane l holds piece l of quad lane p's entry.
__device__ __forceinline__ void quad_transpose(uint4 (&r)[4], int l)
{
    quad_stage<2>(r, l);
    quad_stage<1>(r, l);
}

// Children of one parent along a dimension JD that is not staged: their
// A/B terms were prepared per child entry by prep_kernel, in the parent's
// internal layout (64 B each, in the child section's blocked order).
template <int D, int JD>
__device__ __forceinline__ void direct_children(const SweepJob &J, const DevTables &T,
                                                const Idx4 &idx, const QInfo &q, Set256 &Wnt,
                                                Set256 &Nnt)
{
    int cshape[4] = {J.m[0], J.m[1], J.m[2], J.m[3]};
    cshape[JD] = J.cm[JD];
    constexpr int ip = JD == 3 ? D : JD;
    unsigned empt = ~(unsigned)(q.bm | q.wm) & 0x1ffu;
    while (empt) {
        const int cell = __builtin_ctz(empt);
        empt &= empt - 1;
        const uint16_t cc = T.canon[q.code + J.mover * c_pow3[cell]];
        Idx4 cidx = idx;
        cidx.v[JD] = cc & 0xfff;
        const uint4 *p = J.prep[JD] + 4 * block_offset(cshape, cidx.v);
        s_or_into(Wnt, shift_dim(set_from(p), ip, cc >> 12));
        s_or_into(Nnt, shift_dim(set_from(p + 2), ip, cc >> 12));
    }
}

// A/B terms of every entry of the child section along JD (for dimensions
// that a sweep does not stage in LDS), written in the internal layout of the
// parent's sweep (dimension J.d exchanged with 3).
template <int JD>
__device__ __forceinline__ void prep_entry(const SweepJob &J, const DevTables &T, long long i)
{
    int cshape[4] = {J.m[0], J.m[1], J.m[2], J.m[3]};
    cshape[JD] = J.cm[JD];
    Idx4 idx;
    long long r = i;
    idx.v[3] = (int)(r % cshape[3]); r /= cshape[3];
    idx.v[2] = (int)(r % cshape[2]); r /= cshape[2];
    idx.v[1] = (int)(r % cshape[1]); r /= cshape[1];
    idx.v[0] = (int)r;
    Set256 A, B;
    child_entry_terms<JD>(J, T, idx, A, B);
    swap_with3_rt(A, J.d);
    swap_with3_rt(B, J.d);
    uint4 *p = J.prep_out[JD] + 4 * block_offset(cshape, idx.v);
    p[0] = make_uint4(A.w[0], A.w[1], A.w[2], A.w[3]);
    p[1] = make_uint4(A.w[4], A.w[5], A.w[6], A.w[7]);
    p[2] = make_uint4(B.w[0], B.w[1], B.w[2], B.w[3]);
    p[3] = make_uint4(B.w[4], B.w[5], B.w[6], B.w[7]);
}

__device__ __forceinline__ long long prep_count(const SweepJob &J, int jd)
{
    long long n = jd == 0 ? J.cm[0] : jd == 1 ? J.cm[1] : jd == 2 ? J.cm[2] : J.cm[3];
    for (int i = 0; i < 4; i++)
        if (i != jd) n *= (i == 0 ? J.m[0] : i == 1 ? J.m[1] : i == 2 ? J.m[2] : J.m[3]);
    return n;
}

template <int JD>
__global__ void __launch_bounds__(256) prep_kernel(SweepJob J, DevTables T)
{
    const long long n = prep_count(J, JD);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        prep_entry<JD>(J, T, i);
}

// Prep passes of many jobs in one launch: unit u = (job, dimension), its
// 256-entry chunks numbered from chunk_start[u].
__global__ void __launch_bounds__(256)
    prep_batch_kernel(const SweepJob *jobs, const int *unit, const long long *chunk_start, int nunits,
                      long long total, DevTables T)
{
    for (long long ch = blockIdx.x; ch < total; ch += gridDim.x) {
        int lo = 0, hi = nunits - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (chunk_start[mid] <= ch) lo = mid;
            else hi = mid - 1;
        }
        const int job = unit[lo] >> 2, jd = unit[lo] & 3;
        const SweepJob &J = jobs[job];
        const long long i = (ch - chunk_start[lo]) * 256 + threadIdx.x;
        if (i >= prep_count(J, jd)) continue;
        switch (jd) {
        case 0: prep_entry<0>(J, T, i); break;
        case 1: prep_entry<1>(J, T, i); break;
        case 2: prep_entry<2>(J, T, i); break;
        default: prep_entry<3>(J, T, i); break;
        }
    }
}

int sweep_lds_bytes(int G, int mD, int cmD)
{
    return tile_lds_bytes(G, mD, cmD, nullptr, nullptr);
}

template <int D>
__device__ void sweep_tile(const SweepJob &J, const DevTables &T, long long tile, void *lds_base)
{
    // tile = ((i_O1 * m_O2) + i_O2) * ngroups + group of G lines along E
    constexpr int E = D == 3 ? 2 : 3;
    constexpr int O1 = D == 0 ? 1 : 0;
    constexpr int O2 = D == 3 ? 1 : (D == 2 ? 1 : 2);
    // (32-bit: a section has fewer than 2^32 entries, so fewer tiles)
    const uint32_t t32 = (uint32_t)tile, ng = (uint32_t)J.ngroups, mo2 = (uint32_t)J.m[O2];
    const uint32_t rest = t32 / ng;
    const int grp = (int)(t32 - rest * ng);
    Idx4 base;
    base.v[D] = 0;
    base.v[O1] = (int)(rest / mo2);
    base.v[O2] = (int)(rest - (uint32_t)base.v[O1] * mo2);
    base.v[E] = grp * J.G;
    const int me = J.m[E];
    const int nlines = min(J.G, me - grp * J.G);
    const int c = J.mover;
    const bool staged = (J.emask >> D) & 1;
    const int cmD = J.cm[D];
    const int mD = J.m[D];
    const TileLds L = tile_lds(lds_base, J.G, mD, staged ? cmD : 0);
    // item it of the child pass -> (child position ic, line v): it / nlines
    // by a 16-bit reciprocal, exact for it < 8 * 420 and nlines <= 8
    const uint32_t rcp = (65536u + nlines - 1) / nlines;
    const bool load_children = staged && !((J.odmask >> D) & 1);
    int cshape[4] = {J.m[0], J.m[1], J.m[2], J.m[3]};
    cshape[D] = cmD;

    // The first child item of this thread is fetched from HBM now, so its
    // latency overlaps the table set-up below.
    uint4 pre[4] = {};
    if (load_children && (int)threadIdx.x < nlines * cmD) {
        const int it = threadIdx.x;
        const int ic = (int)(((uint32_t)it * rcp) >> 16);
        Idx4 idx = base;
        idx.v[E] = base.v[E] + (it - ic * nlines);
        idx.v[D] = ic;
        const uint4 *p = J.child[D] + 4 * block_offset(cshape, idx.v);
#pragma unroll
        for (int i = 0; i < 4; i++) pre[i] = p[i];
    }

    // Phase 0: per-line tables (LineMasks of the fixed quadrants, partial
    // sets, chunk tables), for both colours, and the per-position records.
    // Every work item is one small uniform task: a LineMasks, a position, one
    // line's cylinder product, one chunk table entry.
    for (int it = threadIdx.x; it < nlines * 8; it += blockDim.x) {
        const int v = it >> 3, x = ((it >> 2) & 1) + 1, j = it & 3;
        const int ij = get4(base, j) + (j == E ? v : 0);
        const int qbj = j == 0 ? J.qb[0] : j == 1 ? J.qb[1] : j == 2 ? J.qb[2] : J.qb[3];
        const QInfo q = T.qinfo[j == D ? 0 : qbj + ij];
        const LineMasks lm = T.lm[j * 512 + (x == 1 ? q.bm : q.wm)];
        const bool keep = j != D;
        L.lmq[it] = LineMasks{keep ? lm.a : 0u, keep ? lm.b : 0u, keep ? lm.c : 0u};
        if ((it & 7) == 0) {
            Idx4 li = base;
            li.v[E] = base.v[E] + v;
            L.loff[v] = line_offset_coeffs<D>(J.m, li.v);
        }
        if (j == 0) L.O[(2 * v + x - 1) * kOSlots + 18] = make_uint2(0, 0);  // U, ORed below
    }
    // positions along D, resolved once for all lines of the tile
    const int npos = mD + (staged ? cmD : 0);
    const int sst = sel_stride(mD);
    for (int it = threadIdx.x; it < npos; it += blockDim.x) {
        if (it < mD) {
            const QInfo q = T.qinfo[J.qb[D] + it];
            const unsigned mc = c == 1 ? q.bm : q.wm, mo = c == 1 ? q.wm : q.bm;
            const uint4 sc = T.sel[D * 512 + mc], so = T.sel[D * 512 + mo];
            L.sel[it] = make_uint2(sc.x, so.x);
            L.sel[sst + it] = make_uint2(sc.y, so.y);
            L.sel[2 * sst + it] = make_uint2(sc.z, so.z);
            L.sel[3 * sst + it] = make_uint2(sc.w, so.w);
            PosChild &r = L.pch[it];
            unsigned empt = staged ? ~(unsigned)(q.bm | q.wm) & 0x1ffu : 0u;
            int n = 0;
            while (empt) {
                const int cell = __builtin_ctz(empt);
                empt &= empt - 1;
                r.child[n++] = T.canon[q.code + c * c_pow3[cell]];
            }
            r.nchild = (uint16_t)n;
        } else {
            const QInfo q = T.qinfo[J.cqb[D] + (it - mD)];
            const unsigned mc = c == 1 ? q.bm : q.wm, mo = c == 1 ? q.wm : q.bm;
            ChildPosRec &cr = L.cpos[it - mD];
            cr.sel_c = T.sel[D * 512 + mc];
            cr.sel_o = T.sel[D * 512 + mo];
        }
    }
    __syncthreads();
    // partial sets: item (line, colour, l) for the 18 chunk slots and the 15
    // lines missing D (ORed into U); it / 33 by a 16-bit reciprocal, exact
    // for it < 33 * 16
    for (int it = threadIdx.x; it < nlines * 2 * 33; it += blockDim.x) {
        const int vx = (int)(((uint32_t)it * 1986u) >> 16), l = it - 33 * vx;
        const LineMasks *lmq = L.lmq + 4 * vx;
        // chunk slots carry two references (0xffff: unused slot), the lines
        // missing D three
        const uint32_t refs = l < 18 ? (uint32_t)T.chunk_ref[D * 18 + l] | 0xff0000u : T.u_ref[D * 15 + (l - 18)];
        uint2 pr = ref_product3<D>(lmq, refs);
        if (l < 18) {
            if ((refs & 0xffffu) == 0xffffu) pr = make_uint2(0, 0);
            L.O[kOSlots * vx + l] = pr;
        } else {
            uint32_t *u = (uint32_t *)(L.O + kOSlots * vx + 18);
            if (pr.x) atomicOr(u, pr.x);
            if (pr.y) atomicOr(u + 1, pr.y);
        }
    }
    __syncthreads();
    // chunk tables: item (line, colour, chunk, subset s of the chunk's first
    // 5 lines) writes entries s and s + 32 (the 6th line added); 32
    // consecutive lanes write 32 consecutive entries
    for (int it = threadIdx.x; it < nlines * 2 * 3 * 32; it += blockDim.x) {
        const int sigma = it & 31, g = it >> 5, vx = g / 3, ch = g - 3 * vx;
        const uint2 *O = L.O + kOSlots * vx + 6 * ch;
        uint2 r = ch == 0 ? L.O[kOSlots * vx + 18] : make_uint2(0, 0);
#pragma unroll
        for (int b = 0; b < 5; b++) {
            if ((sigma >> b) & 1) {
                const uint2 o = O[b];
                r.x |= o.x;
                r.y |= o.y;
            }
        }
        uint2 *dst = L.lut + kLutStride * (vx >> 1) + 192 * (vx & 1) + 64 * ch + sigma;
        const uint2 o5 = O[5];
        dst[0] = r;
        dst[32] = make_uint2(r.x | o5.x, r.y | o5.y);
    }
    __syncthreads();

    // Phase 1: stage the child line(s) of dimension D (Fig. 3 "gather"):
    // A = F_c(child) | rmax(not N_child), B = F_c(child) | rmax(not W_child).
    if (staged) {
        const int total = nlines * cmD;
        auto child_item = [&](int it, Set256 W, Set256 N) {
            const int ic = (int)(((uint32_t)it * rcp) >> 16);
            const int v = it - ic * nlines;
            const ChildPosRec &cp = L.cpos[ic];
            const uint2 *lut = L.lut + kLutStride * v;
            const Set256 Fc = five_lut(lut + 192 * (c - 1), cp.sel_c);
            if ((J.odmask >> D) & 1) {
                const Set256 Fo = five_lut(lut + 192 * (2 - c), cp.sel_o);
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    W.w[i] = Fo.w[i] & ~Fc.w[i];
                    N.w[i] = Fo.w[i] | ~Fc.w[i];
                }
            } else {
                swap_with3<D>(W);
                swap_with3<D>(N);
            }
            Set256 A, B;
            child_terms(Fc, W, N, A, B);
            uint32_t *r = L.rec + kRecWords * (ic * J.G + v);
#pragma unroll
            for (int i = 0; i < 8; i += 2) {
                *(uint2 *)(r + i) = make_uint2(A.w[i], A.w[i + 1]);
                *(uint2 *)(r + 8 + i) = make_uint2(B.w[i], B.w[i + 1]);
            }
        };
        // the first item of each thread uses the prefetched entry
        if ((int)threadIdx.x < total) child_item(threadIdx.x, set_from(pre), set_from(pre + 2));
        for (int it = threadIdx.x + blockDim.x; it < total; it += blockDim.x) {
            Set256 W, N;
            if (load_children) {
                const int ic = (int)(((uint32_t)it * rcp) >> 16);
                Idx4 idx = base;
                idx.v[E] = base.v[E] + (it - ic * nlines);
                idx.v[D] = ic;
                load_info(J.child[D] + 4 * block_offset(cshape, idx.v), W, N);
            } else {
                W = s_zero();
                N = s_zero();
            }
            child_item(it, W, N);
        }
        __syncthreads();
    }

    // Phase 2: every parent entry of the tile (Fig. 3 "compute").  A wave
    // takes 64 parents that are consecutive in memory order (for D = 3 along
    // D, the fastest index of a block; otherwise along the lines, dimension
    // 3); quad lane l of quad q computes parent 16 l + q, so after the quad
    // transpose store p writes parents 16 p .. 16 p + 15.
    const int lane = threadIdx.x & 63, l4 = lane & 3, q = lane >> 2;
    const int nwaves = blockDim.x >> 6;
    const int nparents = nlines * mD;
    // P / div as a multiply-high by ceil(2^32 / div): exact for P < 2^32 / div
    // (P < 8 * 420 here); div = 1 has no 32-bit multiplier and is kept apart
    const uint32_t div = D == 3 ? (uint32_t)mD : (uint32_t)nlines;
    const uint32_t magic = div > 1 ? 0xffffffffu / div + 1u : 0u;
    for (int g0 = (threadIdx.x >> 6) * 64; g0 < nparents; g0 += nwaves * 64) {
        const int P = min(g0 + 16 * l4 + q, nparents - 1);  // a spare lane repeats the last parent
        const int hiq = div > 1 ? (int)__umulhi((uint32_t)P, magic) : P;
        const int loq = P - hiq * (int)div;
        const int v = D == 3 ? hiq : loq;
        const int iD = D == 3 ? loq : hiq;
        Idx4 idx = base;
        idx.v[E] = base.v[E] + v;
        idx.v[D] = iD;
        Set256 Wnt = s_zero(), Nnt = J.emask == 0 ? s_full() : s_zero();
        if (staged) {
            const PosChild &pr = L.pch[iD];
            const uint32_t *line = L.rec + kRecWords * v;
            const int n = pr.nchild;
            for (int e = 0; e < n; e++) {
                const uint32_t cc = pr.child[e];
                const uint32_t *r = line + kRecWords * J.G * (cc & 0xfff);
                or_rotated(Wnt, r, cc >> 12);
                or_rotated(Nnt, r + 8, cc >> 12);
            }
        }
        // Children along the other dimensions with empty cells.
        if (J.emask & ~(1 << D)) {
            QInfo qi[4];
#pragma unroll
            for (int j = 0; j < 4; j++) qi[j] = T.qinfo[J.qb[j] + idx.v[j]];
            if (D != 0 && (J.emask & 1)) direct_children<D, 0>(J, T, idx, qi[0], Wnt, Nnt);
            if (D != 1 && (J.emask & 2)) direct_children<D, 1>(J, T, idx, qi[1], Wnt, Nnt);
            if (D != 2 && (J.emask & 4)) direct_children<D, 2>(J, T, idx, qi[2], Wnt, Nnt);
            if (D != 3 && (J.emask & 8)) direct_children<D, 3>(J, T, idx, qi[3], Wnt, Nnt);
        }
        const uint2 *lut = L.lut + kLutStride * v;
        const uint2 s0 = L.sel[iD], s1 = L.sel[sst + iD], s2 = L.sel[2 * sst + iD], s3 = L.sel[3 * sst + iD];
        const Set256 Fc = five_lut(lut + 192 * (c - 1), make_uint4(s0.x, s1.x, s2.x, s3.x));
        const Set256 Fo = five_lut(lut + 192 * (2 - c), make_uint4(s0.y, s1.y, s2.y, s3.y));
        Set256 W, N;
        combine(Fc, Fo, Wnt, Nnt, W, N);
        swap_with3<D>(W);
        swap_with3<D>(N);
        uint4 r[4] = {make_uint4(W.w[0], W.w[1], W.w[2], W.w[3]), make_uint4(W.w[4], W.w[5], W.w[6], W.w[7]),
                      make_uint4(N.w[0], N.w[1], N.w[2], N.w[3]), make_uint4(N.w[4], N.w[5], N.w[6], N.w[7])};
        quad_transpose(r, l4);
        const uint4 lc = L.loff[v];
        const uint32_t bD = (uint32_t)iD >> 3;
        const uint32_t sD = min(8u, (uint32_t)mD - 8u * bD), rD = (uint32_t)iD & 7u;
        // for D = 3 every coefficient but c0 is below 2^13 (products of block
        // extents), so 24-bit multiplies are exact
        const uint32_t off = D == 3 ? lc.x + __umul24(lc.y, bD) + __umul24(lc.z, sD) + rD
                                    : lc.x + lc.y * bD + lc.z * sD + lc.w * rD;
        const uint32_t offs[4] = {quad_perm<0x00>(off), quad_perm<0x55>(off), quad_perm<0xAA>(off),
                                  quad_perm<0xFF>(off)};
#pragma unroll
        for (int p = 0; p < 4; p++)
            if (g0 + 16 * p + q < nparents) J.out[4 * offs[p] + l4] = r[p];
    }
}

template <int D, int NT>
__global__ void __launch_bounds__(NT, NT == 512 ? 6 : 1) sweep_kernel(SweepJob J, DevTables T)
{
    extern __shared__ uint4 lds[];
    sweep_tile<D>(J, T, blockIdx.x, (void *)lds);
}

// Many sections in one persistent launch: workgroups take tiles from a
// device counter; tile_start[j] is the first global tile of job j.
__global__ void __launch_bounds__(256)
    sweep_batch_kernel(const SweepJob *jobs, const long long *tile_start, int njobs,
                       long long total, unsigned long long *counter, DevTables T)
{
    extern __shared__ uint4 lds[];
    __shared__ long long s_tile;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (long long)atomicAdd(counter, 1ull);
        __syncthreads();
        const long long t = s_tile;
        __syncthreads();
        if (t >= total) break;
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_start[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const SweepJob &J = jobs[lo];
        const long long local = t - tile_start[lo];
        switch (J.d) {
        case 0: sweep_tile<0>(J, T, local, (void *)lds); break;
        case 1: sweep_tile<1>(J, T, local, (void *)lds); break;
        case 2: sweep_tile<2>(J, T, local, (void *)lds); break;
        default: sweep_tile<3>(J, T, local, (void *)lds); break;
        }
        __syncthreads();
    }
}

__global__ void zero_counter_kernel(unsigned long long *c, int n)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

hipError_t launch_prep(const SweepJob &job, int j, const DevTables &T, hipStream_t s)
{
    long long n = job.cm[j];
    for (int i = 0; i < 4; i++)
        if (i != j) n *= job.m[i];
    const unsigned grid = (unsigned)std::min<long long>((n + 255) / 256, 65536);
    if (n == 0) return hipSuccess;
    switch (j) {
    case 0: hipLaunchKernelGGL(prep_kernel<0>, dim3(grid), dim3(256), 0, s, job, T); break;
    case 1: hipLaunchKernelGGL(prep_kernel<1>, dim3(grid), dim3(256), 0, s, job, T); break;
    case 2: hipLaunchKernelGGL(prep_kernel<2>, dim3(grid), dim3(256), 0, s, job, T); break;
    default: hipLaunchKernelGGL(prep_kernel<3>, dim3(grid), dim3(256), 0, s, job, T); break;
    }
    return hipGetLastError();
}

hipError_t launch_sweep(const SweepJob &job, const DevTables &T, hipStream_t s)
{
    if (job.ntiles == 0) return hipSuccess;
    const dim3 grid((unsigned)job.ntiles), block(job.threads);
    if (job.threads == 512) {
        switch (job.d) {
        case 0: hipLaunchKernelGGL((sweep_kernel<0, 512>), grid, block, job.lds_bytes, s, job, T); break;
        case 1: hipLaunchKernelGGL((sweep_kernel<1, 512>), grid, block, job.lds_bytes, s, job, T); break;
        case 2: hipLaunchKernelGGL((sweep_kernel<2, 512>), grid, block, job.lds_bytes, s, job, T); break;
        default: hipLaunchKernelGGL((sweep_kernel<3, 512>), grid, block, job.lds_bytes, s, job, T); break;
        }
    } else if (job.threads == 256) {
        switch (job.d) {
        case 0: hipLaunchKernelGGL((sweep_kernel<0, 256>), grid, block, job.lds_bytes, s, job, T); break;
        case 1: hipLaunchKernelGGL((sweep_kernel<1, 256>), grid, block, job.lds_bytes, s, job, T); break;
        case 2: hipLaunchKernelGGL((sweep_kernel<2, 256>), grid, block, job.lds_bytes, s, job, T); break;
        default: hipLaunchKernelGGL((sweep_kernel<3, 256>), grid, block, job.lds_bytes, s, job, T); break;
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_prep_batch(const SweepJob *dev_jobs, const int *dev_unit,
                             const long long *dev_chunk_start, int nunits, long long total_chunks,
                             const DevTables &T, hipStream_t s)
{
    if (nunits == 0 || total_chunks == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<long long>(total_chunks, 1 << 16);
    hipLaunchKernelGGL(prep_batch_kernel, dim3(grid), dim3(256), 0, s, dev_jobs, dev_unit,
                       dev_chunk_start, nunits, total_chunks, T);
    return hipGetLastError();
}

int sweep_batch_blocks_per_cu(int lds_bytes)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_batch_kernel, 256, lds_bytes) != hipSuccess)
        return 1;
    return std::max(1, n);
}

hipError_t launch_sweep_batch(const SweepJob *dev_jobs, const long long *dev_tile_start, int njobs,
                              long long total_tiles, int lds_bytes, unsigned long long *dev_counter,
                              int grid, const DevTables &T, hipStream_t s)
{
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, s, dev_counter, 1);
    hipLaunchKernelGGL(sweep_batch_kernel, dim3(grid), dim3(256), lds_bytes, s, dev_jobs,
                       dev_tile_start, njobs, total_tiles, dev_counter, T);
    return hipGetLastError();
}

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

// Per root: two layers of node records (64 B each), then the layer's
// five-set tables (two colours x the largest C(e, s) subsets, 32 B each).
int dag_ftab_bytes(int e) { return 2 * dag_layout(e).max_subsets * 32; }

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

// Solve one root with a group of GROUP threads: the whole workgroup (256) or
// one wave (64).  `buf0` and `buf1` hold two layers of A/B records (64 B per
// node); `ftab` the five-set tables of the current layer; slot_q/slot_l (10
// ints each, LDS) the root's empty cells.
//
// Five-sets: the nodes of layer t hold ceil(t/2) stones of the root's mover
// and floor(t/2) of the other side in the root's empty cells, and a colour's
// five-set depends only on which cells hold that colour.  So each layer first
// computes the five-set of every subset of the empty cells of those two sizes
// (C(e, s) boards per colour instead of one per node and colour: 581 boards
// against 4246 for 8 empty cells), and each node reads its two.
template <int GROUP>
__device__ void solve_root(const RootInfo &R, const DevTables &T, uint4 *buf0, uint4 *buf1,
                           uint4 *ftab, uint4 *out, int *s_slot_q, int *s_slot_l)
{
    const int lane = GROUP == 256 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
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
    if (GROUP == 256) __syncthreads();
    else wave_sync();
    const int e = R.e;
    const uint32_t *nodes = T.dag_node + T.dag_node_off[e];
    const uint16_t *rank = T.dag_rank + T.dag_rank_off[e];
    const uint16_t *smask = T.dag_sub_mask + T.dag_sub_off[e];
    const uint16_t *srank = T.dag_sub_rank + T.dag_sub_off[e];
    const int *layer = T.dag_layer[e];
    const int smax = T.dag_sub_max[e];
    // the root mover's stones and the other side's, per quadrant
    unsigned cm0[4], om0[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        cm0[j] = R.mover == 1 ? R.bm[j] : R.wm[j];
        om0[j] = R.mover == 1 ? R.wm[j] : R.bm[j];
    }
    uint4 *cur = buf0, *prev = buf1;
    for (int t = e; t >= 0; t--) {
        const int n0 = layer[t], n1 = layer[t + 1];
        const int x = (t & 1) ? 3 - R.mover : R.mover;   // side to move at layer t
        const int xdigit = (t & 1) ? 2 : 1;              // slot digit of x's stones
        // five-set tables of the layer: entries [0, nc) for the root mover's
        // subsets of size ceil(t/2), [smax, smax + no) for the other side's
        const int sc = (t + 1) >> 1, so = t >> 1;
        const int nc = T.dag_sub_start[e][sc + 1] - T.dag_sub_start[e][sc];
        const int no = T.dag_sub_start[e][so + 1] - T.dag_sub_start[e][so];
        for (int i = lane; i < nc + no; i += GROUP) {
            const bool mine = i < nc;
            const int r = mine ? i : i - nc;
            const unsigned m = smask[T.dag_sub_start[e][mine ? sc : so] + r];
            unsigned xm[4] = {mine ? cm0[0] : om0[0], mine ? cm0[1] : om0[1], mine ? cm0[2] : om0[2],
                              mine ? cm0[3] : om0[3]};
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
            uint4 *dst = ftab + 2 * ((mine ? 0 : smax) + r);
            dst[0] = make_uint4(F.w[0], F.w[1], F.w[2], F.w[3]);
            dst[1] = make_uint4(F.w[4], F.w[5], F.w[6], F.w[7]);
        }
        if (GROUP == 256) __syncthreads();
        else wave_sync();
        for (int i = n0 + lane; i < n1; i += GROUP) {
            const uint32_t nd = nodes[i];
            const unsigned cmask = nd & 0xffffu, omask = nd >> 16;
            int code = 0;
            for (int sl = e - 1; sl >= 0; sl--)
                code = 3 * code + (((cmask >> sl) & 1) ? 1 : ((omask >> sl) & 1) ? 2 : 0);
            const Set256 Fc = set_from(ftab + 2 * srank[cmask]);
            const Set256 Fo = set_from(ftab + 2 * (smax + srank[omask]));
            const Set256 &Fx = x == R.mover ? Fc : Fo;
            const Set256 &Fy = x == R.mover ? Fo : Fc;
            Set256 Wnt = s_zero(), Nnt = s_zero();
            if (t == e) {
                Nnt = s_full();
            } else {
                const unsigned free = ~(cmask | omask) & ((1u << e) - 1u);
                unsigned f = free;
                while (f) {
                    const int sl = __builtin_ctz(f);
                    f &= f - 1;
                    const int ci = rank[code + xdigit * (int)c_pow3[sl]];
                    const uint4 *p = prev + 4 * ci;
                    s_or_into(Wnt, set_from(p));
                    s_or_into(Nnt, set_from(p + 2));
                }
            }
            Set256 W, N;
            combine(Fx, Fy, Wnt, Nnt, W, N);
            if (t == 0) {
                store_info(out, W, N);
            } else {
                Set256 A, B;
                child_terms(Fy, W, N, A, B);
                uint4 *p = cur + 4 * (i - n0);
                p[0] = make_uint4(A.w[0], A.w[1], A.w[2], A.w[3]);
                p[1] = make_uint4(A.w[4], A.w[5], A.w[6], A.w[7]);
                p[2] = make_uint4(B.w[0], B.w[1], B.w[2], B.w[3]);
                p[3] = make_uint4(B.w[4], B.w[5], B.w[6], B.w[7]);
            }
        }
        if (GROUP == 256) __syncthreads();
        else wave_sync();
        uint4 *tmp = cur;
        cur = prev;
        prev = tmp;
    }
}

// Count roots per number of empty cells (index 11: invalid boards).  Counts
// are gathered per workgroup in LDS first, so each workgroup adds to the
// global counters once per bin (a million lanes adding to twelve global
// counters directly serialise on them).
__global__ void __launch_bounds__(256)
    eval_count_kernel(const uint64_t *boards, size_t n, int *count, uint8_t *empties, int *status,
                      uint4 *out)
{
    __shared__ int lc[12];
    if (threadIdx.x < 12) lc[threadIdx.x] = 0;
    __syncthreads();
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
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
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int e = i < n ? empties[i] : 11;
    const int local = e <= 10 ? atomicAdd(&lc[e], 1) : 0;
    __syncthreads();
    if (threadIdx.x < 11 && lc[threadIdx.x]) base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], lc[threadIdx.x]);
    __syncthreads();
    if (e <= 10) order[start[e] + base[e] + local] = (int)i;
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
//            layers in the workgroup's slot of a global buffer);
//   class 1: 7 empty cells, a workgroup per root, a smaller LDS footprint;
//   class 2: up to kWaveMaxEmpties, one wave per root, four per workgroup,
//            synchronised per wave only.
constexpr int kWaveMaxEmpties = 6;
// two layers of the widest 6-empty layer, then the five-set tables (C(6,3) = 20)
constexpr int kWaveLdsBytes = 2 * 90 * 64 + 2 * 20 * 32;

template <int CLS>
__global__ void __launch_bounds__(256)
    eval_persistent_kernel(const uint64_t *boards, const int *order, const int *start,
                           unsigned long long *counter, uint4 *out, uint4 *gl, DevTables T)
{
    extern __shared__ uint4 lds[];
    __shared__ long long s_item;
    __shared__ int s_slots[4][2][10];
    // bins are ordered by empty cells, most first: e occupies [start[e], start[e - 1])
    const int lo = CLS == 0 ? 0 : CLS == 1 ? start[7] : start[kWaveMaxEmpties];
    const int hi = CLS == 0 ? start[7] : CLS == 1 ? start[kWaveMaxEmpties] : start[11];
    if (CLS < 2) {
        const int big = start[8];  // roots with 9 or 10 empty cells: [0, big)
        uint4 *mine = gl + (size_t)blockIdx.x * 2 * 4 * kDagGlobalLayer;
        for (;;) {
            if (threadIdx.x == 0) s_item = (long long)atomicAdd(&counter[CLS], 1ull);
            __syncthreads();
            const long long item = lo + s_item;
            __syncthreads();
            if (item >= hi) break;
            const int root = order[item];
            const RootInfo R = decode_root(boards[root]);
            if (CLS == 0 && item < big)
                solve_root<256>(R, T, mine, mine + 4 * kDagGlobalLayer, lds, out + 4 * (size_t)root,
                                s_slots[0][0], s_slots[0][1]);
            else
                solve_root<256>(R, T, lds, lds + 4 * T.dag_max[R.e], lds + 8 * T.dag_max[R.e],
                                out + 4 * (size_t)root, s_slots[0][0], s_slots[0][1]);
            __syncthreads();
        }
    } else {
        const int w = threadIdx.x >> 6;
        uint4 *wb = lds + (size_t)w * (kWaveLdsBytes / 16);
        for (;;) {
            unsigned long long got = 0;
            if ((threadIdx.x & 63) == 0) got = atomicAdd(&counter[2], 1ull);
            const long long item = lo + (long long)__shfl(got, 0, 64);
            if (item >= hi) break;
            const int root = order[item];
            const RootInfo R = decode_root(boards[root]);
            solve_root<64>(R, T, wb, wb + 4 * 90, wb + 8 * 90, out + 4 * (size_t)root, s_slots[w][0],
                           s_slots[w][1]);
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
            solve_root<256>(R, T, mine, mine + 4 * kDagGlobalLayer, lds, out + 4 * (size_t)root,
                            s_slots[0], s_slots[1]);
        else
            solve_root<256>(R, T, lds, lds + 4 * T.dag_max[R.e], lds + 8 * T.dag_max[R.e],
                            out + 4 * (size_t)root, s_slots[0], s_slots[1]);
        __syncthreads();
    }
}

// Resident-section lookup (Section VIII: positions inside the database are
// read, not solved): each quadrant of the query is turned to its
// rotation-minimal pattern (k_j turns), the entry is read and shifted back by
// k_j along every dimension.
__global__ void __launch_bounds__(256)
    lookup_kernel(const uint64_t *boards, const int *sec_of, int n, const ResidentSection *secs,
                  uint4 *out, DevTables T)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t b = boards[i];
    const ResidentSection S = secs[sec_of[i]];
    int idx[4], k[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint16_t cc = T.canon[(b >> (16 * j)) & 0xffff];
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
        const unsigned g = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(eval_count_kernel, dim3(g), dim3(256), 0, s, boards, n, S.count,
                           S.empties, status, out);
    }
    hipLaunchKernelGGL(eval_scan_kernel, dim3(1), dim3(64), 0, s, S.count, S.start, S.cursor);
    if (n) {
        const unsigned g = (unsigned)((n + 255) / 256);
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
    (void)n;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const void *kern[3] = {(const void *)eval_persistent_kernel<0>, (const void *)eval_persistent_kernel<1>,
                           (const void *)eval_persistent_kernel<2>};
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, s, S.counter, 3);
    for (int c = 0; c < 3; c++) {
        const int lds = eval_class_lds_bytes(c);
        e = allow_lds(kern[c], lds);
        if (e != hipSuccess) return e;
        // class 0 owns the global layer slots: one per workgroup of `grid`
        int g = grid;
        if (c > 0) {
            int per = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern[c], 256, lds);
            if (e != hipSuccess) return e;
            g = std::max(1, per) * cus;
        }
        switch (c) {
        case 0: hipLaunchKernelGGL(eval_persistent_kernel<0>, dim3(g), dim3(256), lds, s, boards, S.order,
                                   S.start, S.counter, out, S.global_layers, T); break;
        case 1: hipLaunchKernelGGL(eval_persistent_kernel<1>, dim3(g), dim3(256), lds, s, boards, S.order,
                                   S.start, S.counter, out, S.global_layers, T); break;
        default: hipLaunchKernelGGL(eval_persistent_kernel<2>, dim3(g), dim3(256), lds, s, boards, S.order,
                                    S.start, S.counter, out, S.global_layers, T); break;
        }
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
