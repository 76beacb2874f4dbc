// device_common.h -- device helpers shared by the sweep and the endgame
// kernels: the blocked offset of Section IV, superinfo loads and stores, the
// five-set of a board from its quadrants' LineMasks.
//
// Data layout in HBM: a section table is entries x 64 B superinfos (win
// words then not-lose words) in the 8^4-blocked order of Section IV.  One
// lane owns one entry and keeps each 256-bit set in eight VGPRs, so every
// set operation is plain per-lane integer work; nothing here is a dense
// contraction, so there is no MFMA.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace pg {

static __constant__ uint32_t c_pow3[10] = {1, 3, 9, 27, 81, 243, 729, 2187, 6561, 19683};

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


__device__ __forceinline__ Set256 set_from(const uint4 *p)
{
    Set256 x;
    const uint4 u = p[0], v = p[1];
    x.w[0] = u.x; x.w[1] = u.y; x.w[2] = u.z; x.w[3] = u.w;
    x.w[4] = v.x; x.w[5] = v.y; x.w[6] = v.z; x.w[7] = v.w;
    return x;
}

// ---------------------------------------------------------------------------
// Whole-entry memory access by quads.  Each lane works on one entry (64 B,
// four 16-byte pieces).  The four lanes of a quad transpose their pieces in
// registers (two exchange stages of DPP quad permutations), so that in each
// of four load or store instructions the quad moves one whole entry; when
// quad q's lanes hold entries q, q + 16, q + 32, q + 48 of 64 neighbours,
// each instruction of a wave moves 16 neighbouring entries, 1 KB in order.
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
// bit X of l differs from bit X of p.  Written as keep ? own : moved, so that
// each dword is one select whose moved operand is the DPP source.
template <int X>
__device__ __forceinline__ uint32_t quad_pick(bool keep, uint32_t own, uint32_t other)
{
    constexpr int ctrl = X == 1 ? 0xB1 : 0x4E;
    // the exchange runs in every lane (a lane reads its partner's register),
    // the select after it
    const uint32_t moved = quad_perm<ctrl>(other);
    return keep ? own : moved;
}

template <int X>
__device__ __forceinline__ void quad_stage(uint4 (&r)[4], int l)
{
    const bool set = (l & X) != 0;
    uint4 t[4];
#pragma unroll
    for (int p = 0; p < 4; p++) {
        const bool keep = set == ((p & X) != 0);
        const uint4 o = r[p ^ X];
        t[p] = make_uint4(quad_pick<X>(keep, r[p].x, o.x), quad_pick<X>(keep, r[p].y, o.y),
                          quad_pick<X>(keep, r[p].z, o.z), quad_pick<X>(keep, r[p].w, o.w));
    }
#pragma unroll
    for (int p = 0; p < 4; p++) r[p] = t[p];
}

// After this, slot p of quad lane l holds piece l of quad lane p's entry.
__device__ __forceinline__ void quad_transpose(uint4 (&r)[4], int l)
{
    quad_stage<2>(r, l);
    quad_stage<1>(r, l);
}


// A 16-byte store that does not allocate in the caches, for results written
// once and not read again by the kernel that writes them (streaming writes:
// the lines go to HBM without displacing the inputs the kernel still reads).
__device__ __forceinline__ void store_stream(uint4 *p, uint4 v)
{
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    const v4u x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, (v4u *)p);
}

// Clear n work-queue counters (a kernel, not a memset, so the sequence can
// be captured in a graph).
static __global__ void zero_counter_kernel(unsigned long long *c, int n)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

}  // namespace pg
