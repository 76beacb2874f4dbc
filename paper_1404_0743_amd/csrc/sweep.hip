// sweep.hip -- the section sweep (Sections II-IV, Fig. 3): one tile of G
// lines along the quadrant that receives stones per workgroup, the child
// prep pass for the other quadrants, and the batched persistent form.
#include "device_common.h"

namespace pg {

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

// Entry idx of child JD when the child is held as its representative under
// board symmetry J.csym[JD] (Section III: the table of an image is the
// representative's with dimensions moved, reflected for a reflection, and
// shifted): the representative's entry, and in h the turns that complete
// the transform (sym_apply).
template <int JD>
__device__ __forceinline__ const uint4 *child_rep_entry(const SweepJob &J, const DevTables &T, const int *idx,
                                                      int h[4])
{
    const uint16_t *map = T.symmap + J.csym[JD] * kPatterns;
    uint32_t e[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        e[k] = map[(k == JD ? J.cqb[k] : J.qb[k]) + idx[k]];
        h[k] = (int)(e[k] >> 12);
        e[k] &= 0xfffu;
    }
    const int *src = J.rsrc[JD];
    int sidx[4];
#pragma unroll
    for (int t = 0; t < 4; t++)
        sidx[t] = (int)(src[0] == t ? e[0] : src[1] == t ? e[1] : src[2] == t ? e[2] : e[3]);
    return J.child[JD] + 4 * block_offset(J.rm[JD], sidx);
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
        if (J.csym[JD]) {
            int h[4];
            load_info(child_rep_entry<JD>(J, T, idx.v, h), W, N);
            sym_apply_rt2(W, N, J.csym[JD], h);
        } else {
            int cshape[4] = {J.m[0], J.m[1], J.m[2], J.m[3]};
            cshape[JD] = J.cm[JD];
            load_info(J.child[JD] + 4 * block_offset(cshape, idx.v), W, N);
        }
    }
    const Set256 Fc = board_five(T, cm_);
    child_terms(Fc, W, N, A, B);
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
// only on D's pattern and come from T.pat_sel (T.sel per pattern).
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

// The same set, read instead of ORed (the first child of a parent).
__device__ __forceinline__ Set256 load_rotated(const uint32_t *p, int k)
{
    Set256 r;
#pragma unroll
    for (int g3 = 0; g3 < 4; g3++) {
        const uint2 v = *(const uint2 *)(p + 2 * ((g3 - k) & 3));
        r.w[2 * g3] = v.x;
        r.w[2 * g3 + 1] = v.y;
    }
    return r;
}

// Children of one parent along a dimension JD that is not staged: their
// A/B terms were prepared per child entry by prep_kernel, in the parent's
// internal layout (64 B each, in the child section's blocked order).
template <int D, int JD>
__device__ __forceinline__ void direct_children(const SweepJob &J, const DevTables &T,
                                                const Idx4 &idx, Set256 &Wnt, Set256 &Nnt)
{
    int cshape[4] = {J.m[0], J.m[1], J.m[2], J.m[3]};
    cshape[JD] = J.cm[JD];
    constexpr int ip = JD == 3 ? D : JD;
    // the parent's pattern along JD and its children: five words, one load
    // each (word 0: count | child 0 << 16, word i: children 2i - 1, 2i)
    const uint32_t *pw = (const uint32_t *)(T.pat_child + ((J.qb[JD] + idx.v[JD]) << 1) + J.mover - 1);
    uint32_t w[5];
#pragma unroll
    for (int i = 0; i < 5; i++) w[i] = pw[i];
    const int n = (int)(w[0] & 0xffffu);
#pragma unroll
    for (int k = 0; k < 9; k++) {
        if (k < n) {
            const uint32_t cc = (w[(k + 1) >> 1] >> (16 * ((k + 1) & 1))) & 0xffffu;
            Idx4 cidx = idx;
            cidx.v[JD] = cc & 0xfff;
            const uint4 *p = J.prep[JD] + 4 * block_offset(cshape, cidx.v);
            s_or_into(Wnt, shift_dim(set_from(p), ip, cc >> 12));
            s_or_into(Nnt, shift_dim(set_from(p + 2), ip, cc >> 12));
        }
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

// SYMC: the staged child is held as its representative (J.csym[D] != 0).
// STAGED: quadrant D has empty cells (every section but full boards, which
// the one-section sweep hands to the terminal kernel; only the batched forms
// run full boards here).
// Always inlined: the persistent kernels hold several instantiations, and a
// call would spill the caller's registers to scratch.
template <int D, bool SYMC = false, bool STAGED = true>
__device__ __forceinline__ void sweep_tile(const SweepJob &J, const DevTables &T, long long tile, void *lds_base)
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
    constexpr bool staged = STAGED;
    const int cmD = J.cm[D];
    const int mD = J.m[D];
    const TileLds L = tile_lds(lds_base, J.G, mD, staged ? cmD : 0);
    // item it of the child pass -> (child position ic, line v): it / nlines
    // by a 16-bit reciprocal, exact for it < 8 * 420 and nlines <= 8
    const uint32_t rcp = (65536u + nlines - 1) / nlines;
    const bool load_children = staged && !((J.odmask >> D) & 1);
    int cshape[4] = {J.m[0], J.m[1], J.m[2], J.m[3]};
    cshape[D] = cmD;

    // The line references of this thread's first partial-set item (below)
    // are fetched now, so that their latency overlaps phase 0.
    auto item_refs = [&](int it) -> uint32_t {
        const int l = it - 33 * (int)(((uint32_t)it * 1986u) >> 16);
        // chunk slots carry two references (0xffff: unused slot), the lines
        // missing D three
        return l < 18 ? (uint32_t)T.chunk_ref[D * 18 + l] | 0xff0000u : T.u_ref[D * 15 + (l - 18)];
    };
    const uint32_t refs0 = (int)threadIdx.x < nlines * 2 * 33 ? item_refs(threadIdx.x) : 0u;

    // The first child item of this thread is fetched from HBM now, so its
    // latency overlaps the table set-up below.
    uint4 pre[4] = {};
    int hpre[4] = {0, 0, 0, 0};
    if (load_children && (int)threadIdx.x < nlines * cmD) {
        const int it = threadIdx.x;
        const int ic = (int)(((uint32_t)it * rcp) >> 16);
        Idx4 idx = base;
        idx.v[E] = base.v[E] + (it - ic * nlines);
        idx.v[D] = ic;
        const uint4 *p = SYMC ? child_rep_entry<D>(J, T, idx.v, hpre) : J.child[D] + 4 * block_offset(cshape, idx.v);
#pragma unroll
        for (int i = 0; i < 4; i++) pre[i] = p[i];
    }

    // Phase 0: per-line tables (LineMasks of the fixed quadrants, partial
    // sets, chunk tables), for both colours, and the per-position records.
    // Every work item is one small uniform task: a LineMasks, a position, one
    // line's cylinder product, one chunk table entry.  The per-pattern
    // lookups come from tables indexed by pattern (one load each).
    for (int it = threadIdx.x; it < nlines * 8; it += blockDim.x) {
        const int v = it >> 3, x = ((it >> 2) & 1) + 1, j = it & 3;
        const int ij = get4(base, j) + (j == E ? v : 0);
        const int qbj = j == 0 ? J.qb[0] : j == 1 ? J.qb[1] : j == 2 ? J.qb[2] : J.qb[3];
        const bool keep = j != D;
        const LineMasks lm = T.pat_lm[((j * kPatterns + (keep ? qbj + ij : 0)) << 1) + x - 1];
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
        const int p = it < mD ? J.qb[D] + it : J.cqb[D] + (it - mD);
        const uint4 *ps = T.pat_sel + 2 * (((D * kPatterns + p) << 1) + c - 1);
        const uint4 sc = ps[0], so = ps[1];
        if (it < mD) {
            L.sel[it] = make_uint2(sc.x, so.x);
            L.sel[sst + it] = make_uint2(sc.y, so.y);
            L.sel[2 * sst + it] = make_uint2(sc.z, so.z);
            L.sel[3 * sst + it] = make_uint2(sc.w, so.w);
            if (staged) {
                L.pch[it] = T.pat_child[(p << 1) + c - 1];
            } else {
                L.pch[it].nchild = 0;
            }
        } else {
            ChildPosRec &cr = L.cpos[it - mD];
            cr.sel_c = sc;
            cr.sel_o = so;
        }
    }
    __syncthreads();
    // partial sets: item (line, colour, l) for the 18 chunk slots and the 15
    // lines missing D (ORed into U); it / 33 by a 16-bit reciprocal, exact
    // for it < 33 * 16
    for (int it = threadIdx.x; it < nlines * 2 * 33; it += blockDim.x) {
        const int vx = (int)(((uint32_t)it * 1986u) >> 16), l = it - 33 * vx;
        const LineMasks *lmq = L.lmq + 4 * vx;
        const uint32_t refs = it == (int)threadIdx.x ? refs0 : item_refs(it);
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
        if constexpr (SYMC) {
            // one call site of the transform: the first item of each thread
            // takes the prefetched representative entry, later items load
            for (int it = threadIdx.x; it < total; it += blockDim.x) {
                Set256 W = set_from(pre), N = set_from(pre + 2);
                int h[4] = {hpre[0], hpre[1], hpre[2], hpre[3]};
                if (it != (int)threadIdx.x) {
                    const int ic = (int)(((uint32_t)it * rcp) >> 16);
                    Idx4 idx = base;
                    idx.v[E] = base.v[E] + (it - ic * nlines);
                    idx.v[D] = ic;
                    load_info(child_rep_entry<D>(J, T, idx.v, h), W, N);
                }
                sym_apply_rt2(W, N, J.csym[D], h);
                child_item(it, W, N);
            }
        } else {
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
        Set256 Wnt, Nnt;
        if (staged) {
            // quadrant D has J.nchd >= 1 empty cells in every pattern of its
            // class: the first child starts the sums, a uniform loop adds the rest
            const PosChild &pr = L.pch[iD];
            const uint32_t *line = L.rec + kRecWords * v;
            const uint32_t c0 = pr.child[0];
            const uint32_t *r0 = line + kRecWords * J.G * (c0 & 0xfff);
            Wnt = load_rotated(r0, c0 >> 12);
            Nnt = load_rotated(r0 + 8, c0 >> 12);
            for (int e = 1; e < J.nchd; e++) {
                const uint32_t cc = pr.child[e];
                const uint32_t *r = line + kRecWords * J.G * (cc & 0xfff);
                or_rotated(Wnt, r, cc >> 12);
                or_rotated(Nnt, r + 8, cc >> 12);
            }
        } else {
            Wnt = s_zero();
            Nnt = J.emask == 0 ? s_full() : s_zero();
        }
        // Children along the other dimensions with empty cells.
        if (J.emask & ~(1 << D)) {
            if (D != 0 && (J.emask & 1)) direct_children<D, 0>(J, T, idx, Wnt, Nnt);
            if (D != 1 && (J.emask & 2)) direct_children<D, 1>(J, T, idx, Wnt, Nnt);
            if (D != 2 && (J.emask & 4)) direct_children<D, 2>(J, T, idx, Wnt, Nnt);
            if (D != 3 && (J.emask & 8)) direct_children<D, 3>(J, T, idx, Wnt, Nnt);
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
            if (g0 + 16 * p + q < nparents) store_stream(J.out + 4 * offs[p] + l4, r[p]);
    }
}

// 512 threads: at most 64 VGPRs (8 waves per SIMD, no scratch), so that four
// workgroups of tiles up to 40 KiB of LDS share a CU (the tile autotuner
// then takes 5 lines of 160 patterns for the headline section, against 7 at
// three workgroups per CU); the symmetry variant needs more registers.
template <int D, int NT, bool SYMC = false>
__global__ void __launch_bounds__(NT, NT == 512 ? (SYMC ? 5 : 8) : 1) sweep_kernel(SweepJob J, DevTables T)
{
    extern __shared__ uint4 lds[];
    uint32_t tile = blockIdx.x;
    if (J.order == 1) {
        // workgroups go to the 8 XCDs in turn: XCD x = b % 8 takes the x-th
        // contiguous range of tiles (ranges differ in size by at most one)
        const uint32_t n = (uint32_t)J.ntiles, per = n >> 3, rem = n & 7u, x = tile & 7u;
        tile = x * per + min(x, rem) + (tile >> 3);
    }
    sweep_tile<D, SYMC>(J, T, tile, (void *)lds);
}

// Many sections in one launch: workgroup b takes global tile b, found in
// the job whose tiles start at tile_start[j] <= b.  The hardware dispatcher
// hands out the tiles (measured faster than a persistent grid pulling tiles
// from a device counter: no queue atomic, no job table re-read per tile, and
// a new workgroup starts as soon as one ends).  SYMS: some staged children
// are held as their representatives (sweep_tile<D, true> for those jobs).
template <bool SYMS>
__device__ __forceinline__ void sweep_batch_tile(const SweepJob *jobs, const long long *tile_start, int njobs,
                                                 long long total, const DevTables &T)
{
    extern __shared__ uint4 lds[];
    const long long t = blockIdx.x;
    if (t >= total) return;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const SweepJob &J = jobs[lo];
    const long long local = t - tile_start[lo];
    const bool symc = SYMS && J.csym[J.d] != 0 && ((J.emask >> J.d) & 1) && !((J.odmask >> J.d) & 1);
    if (J.emask == 0) {
        sweep_tile<3, false, false>(J, T, local, (void *)lds);  // full boards
    } else if (symc) {
        switch (J.d) {
        case 0: sweep_tile<0, SYMS>(J, T, local, (void *)lds); break;
        case 1: sweep_tile<1, SYMS>(J, T, local, (void *)lds); break;
        case 2: sweep_tile<2, SYMS>(J, T, local, (void *)lds); break;
        default: sweep_tile<3, SYMS>(J, T, local, (void *)lds); break;
        }
    } else {
        switch (J.d) {
        case 0: sweep_tile<0>(J, T, local, (void *)lds); break;
        case 1: sweep_tile<1>(J, T, local, (void *)lds); break;
        case 2: sweep_tile<2>(J, T, local, (void *)lds); break;
        default: sweep_tile<3>(J, T, local, (void *)lds); break;
        }
    }
}

// NT = 256 or 512 threads per tile (the batch autotuner picks one per
// layer), at least 6 (5 with the symmetry variants) waves per SIMD: three
// 512-thread workgroups of tiles up to 52 KiB of LDS per CU, as the tuned
// single-section sweep, or twice as many 256-thread ones where the tiles
// are small (short lines leave most of 512 threads idle in every phase)
template <int NT>
__global__ void __launch_bounds__(NT, 6)
    sweep_batch_kernel(const SweepJob *jobs, const long long *tile_start, int njobs, long long total, DevTables T)
{
    sweep_batch_tile<false>(jobs, tile_start, njobs, total, T);
}

// The same over jobs whose children may be held as their representatives.
template <int NT>
__global__ void __launch_bounds__(NT, 5)
    sweep_batch_sym_kernel(const SweepJob *jobs, const long long *tile_start, int njobs, long long total,
                           DevTables T)
{
    sweep_batch_tile<true>(jobs, tile_start, njobs, total, T);
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
    const bool symc = job.csym[job.d & 3] != 0 && ((job.emask >> job.d) & 1) && !((job.odmask >> job.d) & 1);
    if (symc) {
        // the staged child read through a board symmetry
        if (job.threads == 512) {
            switch (job.d) {
            case 0: hipLaunchKernelGGL((sweep_kernel<0, 512, true>), grid, block, job.lds_bytes, s, job, T); break;
            case 1: hipLaunchKernelGGL((sweep_kernel<1, 512, true>), grid, block, job.lds_bytes, s, job, T); break;
            case 2: hipLaunchKernelGGL((sweep_kernel<2, 512, true>), grid, block, job.lds_bytes, s, job, T); break;
            default: hipLaunchKernelGGL((sweep_kernel<3, 512, true>), grid, block, job.lds_bytes, s, job, T); break;
            }
        } else if (job.threads == 256) {
            switch (job.d) {
            case 0: hipLaunchKernelGGL((sweep_kernel<0, 256, true>), grid, block, job.lds_bytes, s, job, T); break;
            case 1: hipLaunchKernelGGL((sweep_kernel<1, 256, true>), grid, block, job.lds_bytes, s, job, T); break;
            case 2: hipLaunchKernelGGL((sweep_kernel<2, 256, true>), grid, block, job.lds_bytes, s, job, T); break;
            default: hipLaunchKernelGGL((sweep_kernel<3, 256, true>), grid, block, job.lds_bytes, s, job, T); break;
            }
        } else {
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
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

hipError_t launch_sweep_batch(const SweepJob *dev_jobs, const long long *dev_tile_start, int njobs,
                              long long total_tiles, int lds_bytes, int threads, bool sym, const DevTables &T,
                              hipStream_t s)
{
    if (total_tiles <= 0) return hipSuccess;
    if (total_tiles > 0x7fffffffLL || (threads != 256 && threads != 512)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)total_tiles), block(threads);
    if (sym && threads == 512)
        hipLaunchKernelGGL(sweep_batch_sym_kernel<512>, grid, block, lds_bytes, s, dev_jobs, dev_tile_start, njobs,
                           total_tiles, T);
    else if (sym)
        hipLaunchKernelGGL(sweep_batch_sym_kernel<256>, grid, block, lds_bytes, s, dev_jobs, dev_tile_start, njobs,
                           total_tiles, T);
    else if (threads == 512)
        hipLaunchKernelGGL(sweep_batch_kernel<512>, grid, block, lds_bytes, s, dev_jobs, dev_tile_start, njobs,
                           total_tiles, T);
    else
        hipLaunchKernelGGL(sweep_batch_kernel<256>, grid, block, lds_bytes, s, dev_jobs, dev_tile_start, njobs,
                           total_tiles, T);
    return hipGetLastError();
}

}  // namespace pg
