// symmetry.hip -- board symmetries acting on sections and on their tables
// (Section III: the group G = L x| D4 of approximate symmetries, and the
// transform of a table when the representative of a board changes;
// Section IV: only sections whose counts are least under the board
// symmetries are computed, the others are images of those).
#include "device_common.h"
#include "internal.h"

#include <algorithm>
#include <cstring>

namespace pg {

// One workgroup takes a quarter of one 8^4 tile of the image section (up to
// 1024 entries; each wave 64 entries per step).  For the rotations a tile is
// an image block.  A reflection also permutes the patterns of every class
// (the mirror image of a rotation-minimal pattern is canonicalised again),
// so the eight image entries of a block along the image dimension G that
// receives the source's dimension 3 come from eight scattered source
// entries, and the other half of each 128-byte source line would be read by
// another workgroup.  For the reflections the tile therefore takes along G
// the image patterns whose sources form one source block along dimension 3
// (the inverse map syminv), and the image entries along G land in several
// image blocks, each written whole (64 bytes).  The tile's entries are
// enumerated with image dimension 3 fastest and next the dimension A = G
// (for symmetries that keep dimension 3 in place, dimension 2): so the two
// halves of every source line are read by one load instruction (halves
// read by different instructions, even of the same workgroup, are fetched
// from HBM twice).  Lane i works on entry
// 16 (i & 3) + (i >> 2) of its wave's 64: it finds its source entry, the
// quad loads its four source entries whole, transposes, transforms,
// transposes back and stores its four image entries whole.
template <int SYM>
__global__ void __launch_bounds__(256) transform_kernel(SymJob J, DevTables T)
{
    // Workgroups reach the 8 XCDs in turn (workgroup b on XCD b mod 8): the
    // four quarters of image block 8 k + x run on XCD x one after another.
    const uint32_t x = blockIdx.x & 7u, k = blockIdx.x >> 3;
    long long blk = (long long)(k >> 2) * 8 + x;
    const int quarter = (int)(k & 3u);
    if (blk >= J.nblocks) return;
    // enumeration order of the block's dimensions, slowest first
    constexpr int G = sym_quadrant(SYM, 3);
    constexpr bool GROUP = (SYM & 4) != 0;  // tile along G by source blocks
    constexpr int A = G == 3 ? 2 : G;
    constexpr int O1 = A == 0 ? 1 : 0;
    constexpr int O2 = (A == 2 || O1 == 2) ? (A == 1 || O1 == 1 ? 0 : 1) : 2;
    constexpr int D0 = O1 < O2 ? O1 : O2, D1 = O1 < O2 ? O2 : O1;
    int corner[4], s[4];
    {
        int B[4];
        B[3] = (int)(blk % J.nb[3]); blk /= J.nb[3];
        B[2] = (int)(blk % J.nb[2]); blk /= J.nb[2];
        B[1] = (int)(blk % J.nb[1]); blk /= J.nb[1];
        B[0] = (int)blk;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            corner[j] = 8 * B[j];
            s[j] = min(8, J.m[j] - corner[j]);
        }
    }
    const uint32_t base = block_offset(J.m, corner);
    const int vol = s[0] * s[1] * s[2] * s[3];
    // reflections: per entry t of the tile along G, the image pattern's block
    // offset with the tile's other corners, and its local index, its block's
    // extent along G and its symmap entry (r | s << 3 | map << 8)
    __shared__ uint32_t gbase[8], ginfo[8];
    if constexpr (GROUP) {
        if ((int)threadIdx.x < s[G]) {
            const int ig = T.syminv[SYM * kPatterns + J.qb[G] + corner[G] + (int)threadIdx.x];
            int c2[4] = {corner[0], corner[1], corner[2], corner[3]};
            c2[G] = ig & ~7;
            gbase[threadIdx.x] = block_offset(J.m, c2);
            ginfo[threadIdx.x] = (uint32_t)(ig & 7) | ((uint32_t)min(8, J.m[G] - (ig & ~7)) << 3) |
                                 ((uint32_t)T.symmap[SYM * kPatterns + J.qb[G] + ig] << 8);
        }
        __syncthreads();
    }
    const int end = min(vol, 1024 * (quarter + 1));
    // r / s for r < 4096 and s <= 8 as a multiply-high by ceil(2^16 / s):
    // the error stays below 1/16, under the 1/s gap to the next integer
    const uint32_t mg1 = (65535u + s[D1]) / s[D1], mg2 = (65535u + s[A]) / s[A],
                   mg3 = (65535u + s[3]) / s[3];
    const uint16_t *map = T.symmap + SYM * kPatterns;
    const int ql = (int)(threadIdx.x & 3u), qq = (int)((threadIdx.x & 63u) >> 2);
    for (int r0 = 1024 * quarter + 64 * (int)(threadIdx.x >> 6); r0 < end; r0 += 256) {
        // a spare lane past the end repeats the last entry (never stored)
        const int r = min(r0 + 16 * ql + qq, end - 1);
        const uint32_t q3 = ((uint32_t)r * mg3) >> 16;
        const uint32_t q2 = (q3 * mg2) >> 16;
        const uint32_t q1 = (q2 * mg1) >> 16;
        int loc[4];
        loc[D0] = (int)q1;
        loc[D1] = (int)(q2 - q1 * s[D1]);
        loc[A] = (int)(q3 - q2 * s[A]);
        loc[3] = (int)(r - q3 * s[3]);
        int sidx[4], h[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            // along G (reflections) the tile's entry loc[G] comes from LDS
            const uint32_t e = (GROUP && j == G) ? ginfo[loc[G]] >> 8 : map[J.qb[j] + corner[j] + loc[j]];
            h[j] = (int)(e >> 12);
            sidx[sym_source(SYM, j)] = (int)(e & 0xfffu);
        }
        uint32_t doff;
        if constexpr (GROUP) {
            const uint32_t gi = ginfo[loc[G]];
            int l[4] = {loc[0], loc[1], loc[2], loc[3]}, t[4] = {s[0], s[1], s[2], s[3]};
            l[G] = (int)(gi & 7u);
            t[G] = (int)((gi >> 3) & 15u);
            doff = gbase[loc[G]] + (uint32_t)(((l[0] * t[1] + l[1]) * t[2] + l[2]) * t[3] + l[3]);
        } else {
            doff = base + (uint32_t)(((loc[0] * s[1] + loc[1]) * s[2] + loc[2]) * s[3] + loc[3]);
        }
        const uint32_t off = block_offset(J.sm, sidx);
        const uint32_t offs[4] = {quad_perm<0x00>(off), quad_perm<0x55>(off), quad_perm<0xAA>(off),
                                  quad_perm<0xFF>(off)};
        uint4 v[4];
#pragma unroll
        for (int p = 0; p < 4; p++) v[p] = J.src[4 * (size_t)offs[p] + ql];  // piece ql of lane p's entry
        quad_transpose(v, ql);                                               // own entry, pieces 0..3
        Set256 W, N;
        W.w[0] = v[0].x; W.w[1] = v[0].y; W.w[2] = v[0].z; W.w[3] = v[0].w;
        W.w[4] = v[1].x; W.w[5] = v[1].y; W.w[6] = v[1].z; W.w[7] = v[1].w;
        N.w[0] = v[2].x; N.w[1] = v[2].y; N.w[2] = v[2].z; N.w[3] = v[2].w;
        N.w[4] = v[3].x; N.w[5] = v[3].y; N.w[6] = v[3].z; N.w[7] = v[3].w;
        sym_apply<SYM>(W, h);
        sym_apply<SYM>(N, h);
        v[0] = make_uint4(W.w[0], W.w[1], W.w[2], W.w[3]);
        v[1] = make_uint4(W.w[4], W.w[5], W.w[6], W.w[7]);
        v[2] = make_uint4(N.w[0], N.w[1], N.w[2], N.w[3]);
        v[3] = make_uint4(N.w[4], N.w[5], N.w[6], N.w[7]);
        quad_transpose(v, ql);  // slot p: piece ql of the entry of quad lane p
        const uint32_t doffs[4] = {quad_perm<0x00>(doff), quad_perm<0x55>(doff), quad_perm<0xAA>(doff),
                                   quad_perm<0xFF>(doff)};
#pragma unroll
        for (int p = 0; p < 4; p++)
            if (r0 + 16 * p + qq < end) store_stream(J.dst + 4 * (size_t)doffs[p] + ql, v[p]);
    }
}

hipError_t launch_transform(const SymJob &job, const DevTables &T, hipStream_t s)
{
    if (job.nchunks == 0) return hipSuccess;
    const dim3 grid((unsigned)job.nchunks), block(256);
    switch (job.sym) {
    case 0: hipLaunchKernelGGL(transform_kernel<0>, grid, block, 0, s, job, T); break;
    case 1: hipLaunchKernelGGL(transform_kernel<1>, grid, block, 0, s, job, T); break;
    case 2: hipLaunchKernelGGL(transform_kernel<2>, grid, block, 0, s, job, T); break;
    case 3: hipLaunchKernelGGL(transform_kernel<3>, grid, block, 0, s, job, T); break;
    case 4: hipLaunchKernelGGL(transform_kernel<4>, grid, block, 0, s, job, T); break;
    case 5: hipLaunchKernelGGL(transform_kernel<5>, grid, block, 0, s, job, T); break;
    case 6: hipLaunchKernelGGL(transform_kernel<6>, grid, block, 0, s, job, T); break;
    case 7: hipLaunchKernelGGL(transform_kernel<7>, grid, block, 0, s, job, T); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

pentago_section section_image(const pentago_section &s, int sym)
{
    pentago_section r;
    for (int q = 0; q < 4; q++) {
        r.black[sym_quadrant(sym, q)] = s.black[q];
        r.white[sym_quadrant(sym, q)] = s.white[q];
    }
    return r;
}

// Lexicographic order of the count tuples ((b0, w0), ..., (b3, w3)).
static bool section_less(const pentago_section &a, const pentago_section &b)
{
    for (int q = 0; q < 4; q++) {
        if (a.black[q] != b.black[q]) return a.black[q] < b.black[q];
        if (a.white[q] != b.white[q]) return a.white[q] < b.white[q];
    }
    return false;
}

void section_standardize(const pentago_section &s, pentago_section *rep, int *sym)
{
    pentago_section best = s;
    int bestd = 0;
    for (int d = 1; d < 8; d++) {
        const pentago_section img = section_image(s, d);
        if (section_less(img, best)) {
            best = img;
            bestd = d;
        }
    }
    *rep = best;
    *sym = sym_inverse(bestd);
}

// Mark the children of a sweep job as held by their representatives: for
// each quadrant with a child table, the symmetry taking the representative
// to the child, the representative's shape and which of its dimensions
// feeds each child dimension.
void set_child_syms(const pentago_section &s, const pentago_superinfo *const rep[4], SweepJob *J)
{
    for (int j = 0; j < 4; j++) {
        J->csym[j] = 0;
        if (!rep[j] || s.black[j] + s.white[j] == 9) continue;
        pentago_section r;
        int sym = 0;
        section_standardize(child_of(s, j), &r, &sym);
        J->csym[j] = sym;
        section_shape_of(r, J->rm[j]);
        for (int k = 0; k < 4; k++) J->rsrc[j][k] = sym_source(sym, k);
    }
}

int make_sym_job(const pentago_section &s, const pentago_superinfo *table, int sym,
                 pentago_superinfo *out, SymJob *J)
{
    if (!section_valid(s)) return fail(PENTAGO_EINVAL, "invalid section counts");
    if (sym < 0 || sym > 7) return fail(PENTAGO_EINVAL, "symmetry must be 0..7");
    if (!table || !out) return fail(PENTAGO_EINVAL, "table or out is NULL");
    const pentago_section img = section_image(s, sym);
    const HostTables &H = host_tables();
    memset(J, 0, sizeof(*J));
    J->sym = sym;
    section_shape_of(s, J->sm);
    section_shape_of(img, J->m);
    uint64_t entries = 1;
    J->nblocks = 1;
    for (int j = 0; j < 4; j++) {
        J->qb[j] = H.class_start[img.black[j]][img.white[j]];
        J->nb[j] = (J->m[j] + 7) / 8;
        J->nblocks *= J->nb[j];
        entries *= (uint64_t)J->m[j];
    }
    J->nchunks = 4 * 8 * ((J->nblocks + 7) / 8);
    if (entries >= (1ull << 32)) return fail(PENTAGO_ERANGE, "sections of 2^32 entries or more are not supported");
    const uintptr_t a = (uintptr_t)table, b = (uintptr_t)out, n = (uintptr_t)(entries * 64);
    if (a < b + n && b < a + n) return fail(PENTAGO_EINVAL, "out overlaps the source table");
    J->src = (const uint4 *)table;
    J->dst = (uint4 *)out;
    return 0;
}

}  // namespace pg

using namespace pg;

extern "C" {

int pentago_section_image(pentago_section s, int sym, pentago_section *image)
{
    if (!section_valid(s) || sym < 0 || sym > 7 || !image) return fail(PENTAGO_EINVAL, "invalid arguments");
    *image = section_image(s, sym);
    return 0;
}

int pentago_section_standardize(pentago_section s, pentago_section *rep, int *sym)
{
    if (!section_valid(s) || !rep || !sym) return fail(PENTAGO_EINVAL, "invalid arguments");
    section_standardize(s, rep, sym);
    return 0;
}

int pentago_section_transform(pentago_section s, const pentago_superinfo *table, int sym,
                              pentago_superinfo *out, void *hip_stream)
{
    DevTables T;
    int rc = device_tables(&T);
    if (rc) return rc;
    SymJob J;
    rc = make_sym_job(s, table, sym, out, &J);
    if (rc) return rc;
    const hipError_t e = launch_transform(J, T, (hipStream_t)hip_stream);
    return e == hipSuccess ? 0 : hip_fail(e, "transform launch");
}

int pentago_solve_section_d4(pentago_section s, const pentago_superinfo *const rep[4],
                             pentago_superinfo *out, void *hip_stream)
{
    if (!section_valid(s) || !rep) return fail(PENTAGO_EINVAL, "invalid arguments");
    DevTables T;
    int rc = device_tables(&T);
    if (rc) return rc;
    SweepJob J;
    rc = make_job(s, rep, out, &J, -1, 0);
    if (rc) return rc;
    set_child_syms(s, rep, &J);
    // the staged child read through a symmetry takes the kernel variant that
    // needs more registers (two 512-thread workgroups per CU), so the tile
    // shape tuned for the plain sweep, sized for four per CU, leaves LDS
    // unused: take 7 lines (measured on the headline geometry: 148 us
    // against 179 with the plain sweep's 5; 8 lines gave 176)
    if (J.csym[J.d] && ((J.emask >> J.d) & 1) && !((J.odmask >> J.d) & 1) && J.threads == 512) {
        const int cmd = J.cm[J.d];
        int G = 7;
        while (G > J.G && sweep_lds_bytes(G, J.m[J.d], cmd) > 65536) G--;
        if (G > J.G) {
            const int order = J.order;
            rc = make_job(s, rep, out, &J, J.d, G, 512, order);
            if (rc) return rc;
            set_child_syms(s, rep, &J);
        }
    }
    rc = validate_children(J, (hipStream_t)hip_stream);
    if (rc) return rc;
    return run_job(J, T, (hipStream_t)hip_stream);
}

int pentago_slice_sections(int stones, pentago_section *out, size_t cap, size_t *count)
{
    if (stones < 0 || stones > 36 || !count || (cap && !out)) return fail(PENTAGO_EINVAL, "invalid arguments");
    const int tb = (stones + 1) / 2, tw = stones / 2;
    size_t n = 0;
    pentago_section s;
    for (int b0 = 0; b0 <= 9; b0++)
        for (int w0 = 0; b0 + w0 <= 9; w0++)
            for (int b1 = 0; b1 <= 9; b1++)
                for (int w1 = 0; b1 + w1 <= 9; w1++)
                    for (int b2 = 0; b2 <= 9; b2++)
                        for (int w2 = 0; b2 + w2 <= 9; w2++) {
                            const int b3 = tb - b0 - b1 - b2, w3 = tw - w0 - w1 - w2;
                            if (b3 < 0 || w3 < 0 || b3 + w3 > 9) continue;
                            const int bs[4] = {b0, b1, b2, b3}, ws[4] = {w0, w1, w2, w3};
                            for (int q = 0; q < 4; q++) {
                                s.black[q] = (uint8_t)bs[q];
                                s.white[q] = (uint8_t)ws[q];
                            }
                            pentago_section r;
                            int sym;
                            section_standardize(s, &r, &sym);
                            if (sym != 0 || memcmp(&r, &s, sizeof(s)) != 0) continue;
                            if (n < cap) out[n] = s;
                            n++;
                        }
    *count = n;
    return 0;
}

}  // extern "C"
