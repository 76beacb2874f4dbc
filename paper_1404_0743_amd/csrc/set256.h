// set256.h -- 256-bit sets over L = Z4^4 and the rotation-abstracted
// primitives of Section III: rmax, the five-in-a-row set over L, and the
// cyclic shift f_b -> f_{gb} for g in L.
//
// A set lives in eight 32-bit words held by one lane: element
// g = g0 + 4*g1 + 16*g2 + 64*g3 is word g >> 5 = (g2 >> 1) + 2*g3, bit
// g & 31 = g0 + 4*g1 + 16*(g2 & 1).  So dimensions 0 and 1 are bit
// positions inside 16-bit halves, dimension 2 picks the half and the word of
// a pair, dimension 3 picks the word pair.  All functions are usable on the
// host too (the library's CPU self-checks call them there).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PG_HD __host__ __device__ __forceinline__

namespace pg {

struct Set256 {
    uint32_t w[8];
};

PG_HD Set256 s_zero()
{
    Set256 r;
#pragma unroll
    for (int i = 0; i < 8; i++) r.w[i] = 0;
    return r;
}

PG_HD Set256 s_full()
{
    Set256 r;
#pragma unroll
    for (int i = 0; i < 8; i++) r.w[i] = 0xffffffffu;
    return r;
}

PG_HD void s_or_into(Set256 &a, const Set256 &b)
{
#pragma unroll
    for (int i = 0; i < 8; i++) a.w[i] |= b.w[i];
}

PG_HD Set256 s_not(const Set256 &a)
{
    Set256 r;
#pragma unroll
    for (int i = 0; i < 8; i++) r.w[i] = ~a.w[i];
    return r;
}

PG_HD uint32_t rotr32(uint32_t x, int s) { return (x >> s) | (x << (32 - s)); }

// (m & a) | (~m & b): one v_bfi_b32
PG_HD uint32_t bfi(uint32_t m, uint32_t a, uint32_t b) { return (m & a) | (~m & b); }

// swap the two bytes of each 16-bit half
PG_HD uint32_t swap_bytes16(uint32_t x) { return ((x >> 8) & 0x00ff00ffu) | ((x << 8) & 0xff00ff00u); }

// rmin(X)(g) = AND over the 8 single-quadrant turns r of X(g + r), so that
// rmax(X) = not rmin(not X) (Section III's rmax, by De Morgan).  Along each
// dimension the two neighbours g_j +- 1 of g_j are exactly the two values of
// the other parity, so each dimension is "AND the two values of one parity,
// then hand the result to the other parity":
//   dimension 0 (bit pairs inside nibbles), dimension 1 (nibbles inside
//   16-bit halves), dimension 2 (halves and the two words of a pair),
//   dimension 3 (word pairs).
PG_HD Set256 rmin(const Set256 &x)
{
    Set256 r;
    uint32_t m2[4];
#pragma unroll
    for (int g3 = 0; g3 < 4; g3++) m2[g3] = rotr32(x.w[2 * g3] & x.w[2 * g3 + 1], 16);
    uint32_t m3[4];
#pragma unroll
    for (int p = 0; p < 2; p++) {
        m3[p] = x.w[2 + p] & x.w[6 + p];      // neighbours of g3 = 0 and 2
        m3[2 + p] = x.w[0 + p] & x.w[4 + p];  // neighbours of g3 = 1 and 3
    }
#pragma unroll
    for (int w = 0; w < 8; w++) {
        const int g3 = w >> 1, p = w & 1;
        const uint32_t u = x.w[w];
        // dimension 0: P holds (u0 & u2, u1 & u3) in bits 0, 1 of each nibble
        const uint32_t P = u & (u >> 2) & 0x33333333u;
        const uint32_t Q = ((P >> 1) & 0x11111111u) | ((P << 1) & 0x22222222u);
        const uint32_t n0 = Q | (Q << 2);
        // dimension 1: the same one level up, nibbles inside each half
        const uint32_t P1 = u & (u >> 8) & 0x00ff00ffu;
        const uint32_t Q1 = ((P1 >> 4) & 0x000f000fu) | ((P1 << 4) & 0x00f000f0u);
        const uint32_t n1 = Q1 | (Q1 << 8);
        r.w[w] = (n0 & n1) & (m2[g3] & m3[(g3 & 1) * 2 + p]);
    }
    return r;
}

// rmax(X)(g) = OR over the 8 single-quadrant turns r of X(g + r) (Section III).
PG_HD Set256 rmax(const Set256 &x) { return s_not(rmin(s_not(x))); }

// out(g) = in(g - k e_d): the table of a board whose quadrant d was turned k
// more times (Section III, transform f_b -> f_{gb} with g = k e_d).
PG_HD Set256 shift_dim(const Set256 &x, int d, int k)
{
    k &= 3;
    if (k == 0) return x;
    Set256 r;
    if (d == 0) {
        const uint32_t hi = 0x11111111u * ((0xfu << k) & 0xfu);
        const uint32_t lo = 0x11111111u * (0xfu >> (4 - k));
#pragma unroll
        for (int w = 0; w < 8; w++) r.w[w] = ((x.w[w] << k) & hi) | ((x.w[w] >> (4 - k)) & lo);
    } else if (d == 1) {
        const int s = 4 * k;
        const uint32_t hi = 0x00010001u * ((0xffffu << s) & 0xffffu);
        const uint32_t lo = 0x00010001u * (0xffffu >> (16 - s));
#pragma unroll
        for (int w = 0; w < 8; w++) r.w[w] = ((x.w[w] << s) & hi) | ((x.w[w] >> (16 - s)) & lo);
    } else if (d == 2) {
        // halves g2 = 0..3 of each word pair rotate by k: by two halves
        // (swap the words) then by one half (funnel shift by 16)
#pragma unroll
        for (int g3 = 0; g3 < 4; g3++) {
            uint32_t a = x.w[2 * g3], b = x.w[2 * g3 + 1];
            if (k & 2) { uint32_t t = a; a = b; b = t; }
            if (k & 1) {
                uint32_t na = (b >> 16) | (a << 16);
                uint32_t nb = (a >> 16) | (b << 16);
                a = na;
                b = nb;
            }
            r.w[2 * g3] = a;
            r.w[2 * g3 + 1] = b;
        }
    } else {
        // word pairs g3 rotate by k: by one pair then by two pairs
        uint32_t t[8];
#pragma unroll
        for (int w = 0; w < 8; w++) t[w] = (k & 1) ? x.w[(w + 6) & 7] : x.w[w];
#pragma unroll
        for (int w = 0; w < 8; w++) r.w[w] = (k & 2) ? t[(w + 4) & 7] : t[w];
    }
    return r;
}

// Exchange index bit I (inside a word, I < 5) with word-index bit B: the
// elements whose bit I is 1 and bit B is 0 trade places with those whose bit
// I is 0 and bit B is 1.
template <int I, int B>
PG_HD void swap_index_bits(Set256 &x)
{
    constexpr int s = 1 << I;
    constexpr uint32_t M = I == 0 ? 0x55555555u : I == 1 ? 0x33333333u : I == 2 ? 0x0f0f0f0fu
                         : I == 3 ? 0x00ff00ffu : 0x0000ffffu;
#pragma unroll
    for (int w = 0; w < 8; w++) {
        if ((w >> B) & 1) continue;
        const int w2 = w | (1 << B);
        const uint32_t t = ((x.w[w] >> s) ^ x.w[w2]) & M;
        x.w[w2] ^= t;
        x.w[w] ^= t << s;
    }
}

// Exchange dimensions D and 3 of L (self-inverse).  The sweep keeps the
// dimension of the quadrant that receives stones in the word-pair position,
// where a cyclic shift along it is a re-addressing of word pairs.
template <int D>
PG_HD void swap_with3(Set256 &x)
{
    if constexpr (D == 3) {
        return;
    } else if constexpr (D == 2) {
        // index bit 4 (half) <-> bit 6 (word bit 1); bit 5 (word bit 0) <-> bit 7 (word bit 2)
        swap_index_bits<4, 1>(x);
        uint32_t t = x.w[1]; x.w[1] = x.w[4]; x.w[4] = t;
        t = x.w[3]; x.w[3] = x.w[6]; x.w[6] = t;
    } else {
        swap_index_bits<2 * D, 1>(x);
        swap_index_bits<2 * D + 1, 2>(x);
    }
}

PG_HD void swap_with3_rt(Set256 &x, int D)
{
    switch (D) {
    case 0: swap_with3<0>(x); break;
    case 1: swap_with3<1>(x); break;
    case 2: swap_with3<2>(x); break;
    default: break;
    }
}

// ------------------------------------------------------------------------
// Board symmetries acting on tables (Section III: a change of the
// representative under G = L x| D4 transforms f_b into f_{gb} by cyclic
// shifts, transpositions of dimensions and reflections).
//
// sym = r + 4 f: mirror the board left-right when f is set, then turn the
// whole board r quarter turns counter-clockwise.  Quadrant q moves to
// sym_quadrant(sym, q); every quadrant's cells move by the same local map
// (mirror, then r turns), and a reflection reverses the sense of quadrant
// turns.  For a board b and its image b', the value of g.b equals the value
// of g'.b' where g'_{pi(i)} = sign * g_i (pi = sym_quadrant, sign -1 for a
// reflection); when b' is rotation-minimal only up to turns h of its
// quadrants, g' gains + h.  So the image table is
//   out(G) = in(g),  g_i = sign * (G_{pi(i)} - h_{pi(i)}),
// computed as: move dimension i to position pi(i), negate every dimension
// for a reflection, shift dimension j by h_j.
// ------------------------------------------------------------------------

PG_HD constexpr int sym_quadrant(int sym, int q)
{
    int qr = q >> 1, qc = q & 1;
    if (sym & 4) qc = 1 - qc;
    for (int t = 0; t < (sym & 3); t++) {
        const int nr = 1 - qc, nc = qr;  // a counter-clockwise quarter turn
        qr = nr;
        qc = nc;
    }
    return 2 * qr + qc;
}

// the quadrant that sym moves onto quadrant j
PG_HD constexpr int sym_source(int sym, int j)
{
    int q = 0;
    for (int i = 0; i < 4; i++)
        if (sym_quadrant(sym, i) == j) q = i;
    return q;
}

// Reflections are involutions; a rotation by r is undone by 4 - r.
PG_HD constexpr int sym_inverse(int sym) { return (sym & 4) ? sym : (4 - sym) & 3; }

// Exchanges with dimension 3 (swap_with3) that move dimension i to position
// sym_quadrant(sym, i): positions 0, 1, 2 are filled in turn, each with at
// most two exchanges.
struct SymSteps {
    int n;
    int a[6];
};

PG_HD constexpr SymSteps sym_steps(int sym)
{
    SymSteps st{0, {0, 0, 0, 0, 0, 0}};
    int at[4] = {0, 1, 2, 3};  // source dimension now at each position
    for (int t = 0; t < 3; t++) {
        const int want = sym_source(sym, t);
        if (at[t] == want) continue;
        if (at[3] != want) {
            int u = 0;
            for (int p = 0; p < 3; p++)
                if (at[p] == want) u = p;
            const int x = at[u];
            at[u] = at[3];
            at[3] = x;
            st.a[st.n++] = u;
        }
        const int x = at[t];
        at[t] = at[3];
        at[3] = x;
        st.a[st.n++] = t;
    }
    return st;
}

// out(g) = in(g with g_D replaced by -g_D): values 1 and 3 trade places.
template <int D>
PG_HD void negate_dim(Set256 &x)
{
    if constexpr (D == 0) {
#pragma unroll
        for (int w = 0; w < 8; w++) x.w[w] = bfi(0x55555555u, x.w[w], bfi(0x22222222u, x.w[w] >> 2, x.w[w] << 2));
    } else if constexpr (D == 1) {
#pragma unroll
        for (int w = 0; w < 8; w++) x.w[w] = bfi(0x0f0f0f0fu, x.w[w], bfi(0x00f000f0u, x.w[w] >> 8, x.w[w] << 8));
    } else if constexpr (D == 2) {
        // g2 = 1 (upper half of the even word) <-> g2 = 3 (upper half of the odd word)
#pragma unroll
        for (int g3 = 0; g3 < 4; g3++) {
            const uint32_t a = x.w[2 * g3], b = x.w[2 * g3 + 1];
            x.w[2 * g3] = bfi(0xffff0000u, b, a);
            x.w[2 * g3 + 1] = bfi(0xffff0000u, a, b);
        }
    } else {
        // word pair 1 <-> word pair 3
        uint32_t t = x.w[2]; x.w[2] = x.w[6]; x.w[6] = t;
        t = x.w[3]; x.w[3] = x.w[7]; x.w[7] = t;
    }
}

// The image table under board symmetry SYM (see above); h[j] are the turns
// of image quadrant j.
template <int SYM>
PG_HD void sym_apply(Set256 &x, const int h[4])
{
    constexpr SymSteps st = sym_steps(SYM);
#pragma unroll
    for (int i = 0; i < 6; i++) {
        if (i < st.n) {
            if (st.a[i] == 0) swap_with3<0>(x);
            else if (st.a[i] == 1) swap_with3<1>(x);
            else swap_with3<2>(x);
        }
    }
    if constexpr ((SYM & 4) != 0) {
        negate_dim<0>(x);
        negate_dim<1>(x);
        negate_dim<2>(x);
        negate_dim<3>(x);
    } else if constexpr (SYM != 0) {
        // a rotation by r turns every pattern without a symmetry of its own
        // by h = r: then the shifts are compile-time
        constexpr int r = SYM & 3;
        if (h[0] == r && h[1] == r && h[2] == r && h[3] == r) {
            x = shift_dim(x, 0, r);
            x = shift_dim(x, 1, r);
            x = shift_dim(x, 2, r);
            x = shift_dim(x, 3, r);
            return;
        }
    }
    x = shift_dim(x, 0, h[0]);
    x = shift_dim(x, 1, h[1]);
    x = shift_dim(x, 2, h[2]);
    x = shift_dim(x, 3, h[3]);
}

// Both sets of an entry (win, not-lose) under one runtime symmetry.
PG_HD void sym_apply_rt2(Set256 &a, Set256 &b, int sym, const int h[4])
{
    switch (sym & 7) {
    case 0: sym_apply<0>(a, h); sym_apply<0>(b, h); break;
    case 1: sym_apply<1>(a, h); sym_apply<1>(b, h); break;
    case 2: sym_apply<2>(a, h); sym_apply<2>(b, h); break;
    case 3: sym_apply<3>(a, h); sym_apply<3>(b, h); break;
    case 4: sym_apply<4>(a, h); sym_apply<4>(b, h); break;
    case 5: sym_apply<5>(a, h); sym_apply<5>(b, h); break;
    case 6: sym_apply<6>(a, h); sym_apply<6>(b, h); break;
    default: sym_apply<7>(a, h); sym_apply<7>(b, h); break;
    }
}

PG_HD void sym_apply_rt(Set256 &x, int sym, const int h[4])
{
    switch (sym & 7) {
    case 0: sym_apply<0>(x, h); break;
    case 1: sym_apply<1>(x, h); break;
    case 2: sym_apply<2>(x, h); break;
    case 3: sym_apply<3>(x, h); break;
    case 4: sym_apply<4>(x, h); break;
    case 5: sym_apply<5>(x, h); break;
    case 6: sym_apply<6>(x, h); break;
    default: sym_apply<7>(x, h); break;
    }
}

// ------------------------------------------------------------------------
// Five in a row over L (Section III: the set of g for which g.b has five in
// a row of one colour).
//
// Each of the 32 lines of the board touches two or three quadrants.  For a
// quadrant j and a line through it, mu = the 4-bit set of turns k of quadrant
// j after which the line's cells in quadrant j all hold the colour.  The line
// is complete at g iff g_j is in mu_j for every quadrant j it touches, so the
// five-set is a union of products of such 4-bit sets.  Lines are grouped by
// the quadrants they touch:
//   rows of the top half (Q0,Q1), rows of the bottom half (Q2,Q3),
//   columns of the left half (Q0,Q2), of the right half (Q1,Q3),
//   the two long diagonals (Q0,Q3), the two long anti-diagonals (Q1,Q2),
//   and four single lines touching three quadrants:
//   T013 (Q0,Q1,Q3), T023 (Q0,Q2,Q3), T012 (Q0,Q1,Q2), T123 (Q1,Q2,Q3).
//
// LineMasks of one quadrant and one colour pattern (a 9-bit stone mask):
//   a = its six lines of the first two-quadrant group, nibble i = line i
//   b = its six lines of the second group
//   c = nibbles 0,1: its two lines of the diagonal pair;
//       nibble 2: T013, 3: T023, 4: T012, 5: T123 (zero where the line misses it)
// First/second group per quadrant: Q0 (top rows, left columns),
// Q1 (top rows, right columns), Q2 (bottom rows, left columns),
// Q3 (bottom rows, right columns).  Diagonal pair: Q0,Q3 long diagonals;
// Q1,Q2 long anti-diagonals.
// ------------------------------------------------------------------------
struct LineMasks {
    uint32_t a, b, c;
};

PG_HD uint32_t nib(uint32_t x, int i) { return (x >> (4 * i)) & 0xfu; }

// bit y of m moves to bit 4y
PG_HD uint32_t spread1(uint32_t m)
{
    return (m & 1u) | ((m & 2u) << 3) | ((m & 4u) << 6) | ((m & 8u) << 9);
}

// {x + 4y : x in a, y in b}
PG_HD uint32_t prod16(uint32_t a, uint32_t b) { return a * spread1(b); }

// a set of g0 values, repeated for every g1 (16-bit half)
PG_HD uint32_t rep_g0(uint32_t m) { return m * 0x1111u; }
// a set of g1 values, every g0 (16-bit half)
PG_HD uint32_t fill_g1(uint32_t m) { return spread1(m) * 0xfu; }

PG_HD uint32_t union_pairs6(uint32_t lo, uint32_t hi)
{
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 6; i++) s |= prod16(nib(lo, i), nib(hi, i));
    return s;
}

PG_HD uint32_t union_pairs2(uint32_t lo, uint32_t hi)
{
    return prod16(nib(lo, 0), nib(hi, 0)) | prod16(nib(lo, 1), nib(hi, 1));
}

// The five-set factors over pairs of quadrants.  Every group of lines above
// depends on the patterns of two quadrants, and each three-quadrant line on
// a product of two quadrants' sets with a third quadrant's; so the five-set
// is assembled from six pair terms, each a function of two quadrants'
// LineMasks only, already laid out as the 32-bit words of a Set256 (word
// 2 g3 + p holds g2 = 2p in its low half and g2 = 2p + 1 in its high half,
// g0 + 4 g1 inside a half).  A tile of entries sharing patterns can build the
// pair terms once and assemble each entry from them.
//   pair01 (Q0,Q1): {S01, P012, P013} each repeated in both halves, 0
//   pair02 (Q0,Q2): E02 for p = 0, 1 (the left columns over g0, g2), and
//                   B for p = 0, 1 (T023's Q0 set where T023's Q2 set holds g2)
//   pair12 (Q1,Q2): E12 for p = 0, 1 (anti-diagonals over g1, g2), and
//                   C for p = 0, 1 (T123's Q1 set where its Q2 set holds g2)
//   pair03 (Q0,Q3): per g3, the long diagonals over g0 (both halves)
//   pair13 (Q1,Q3): per g3, the right columns over g1 (both halves)
//   pair23 (Q2,Q3): words 0-7: the bottom rows over g2, g3 as half-word masks;
//                   8-9: the halves where T012's Q2 set holds g2; 10: T013's
//                   Q3 set | T023's Q3 set << 4 | T123's Q3 set << 8; 11: 0
PG_HD uint32_t halves(uint32_t lo, uint32_t hi) { return (lo & 0xffffu) | (hi << 16); }
PG_HD uint32_t both_halves(uint32_t x) { return halves(x, x); }
PG_HD uint32_t bit_halfmask(uint32_t set, int i) { return (((set >> i) & 1u) ? 0x0000ffffu : 0u) | (((set >> (i + 1)) & 1u) ? 0xffff0000u : 0u); }

PG_HD uint4 pair01(const LineMasks &q0, const LineMasks &q1)
{
    const uint32_t S01 = union_pairs6(q0.a, q1.a);
    const uint32_t P012 = prod16(nib(q0.c, 4), nib(q1.c, 4));
    const uint32_t P013 = prod16(nib(q0.c, 2), nib(q1.c, 2));
    return make_uint4(both_halves(S01), both_halves(P012), both_halves(P013), 0u);
}

PG_HD uint4 pair02(const LineMasks &q0, const LineMasks &q2)
{
    const uint32_t S02 = union_pairs6(q0.b, q2.b);  // g0 + 4 g2
    const uint32_t b0 = rep_g0(nib(q0.c, 3)), b2 = nib(q2.c, 3);
    uint32_t e[2], b[2];
#pragma unroll
    for (int p = 0; p < 2; p++) {
        e[p] = halves(rep_g0(nib(S02, 2 * p)), rep_g0(nib(S02, 2 * p + 1)));
        b[p] = halves(((b2 >> (2 * p)) & 1u) ? b0 : 0u, ((b2 >> (2 * p + 1)) & 1u) ? b0 : 0u);
    }
    return make_uint4(e[0], e[1], b[0], b[1]);
}

PG_HD uint4 pair12(const LineMasks &q1, const LineMasks &q2)
{
    const uint32_t S12 = union_pairs2(q1.c, q2.c);  // g1 + 4 g2
    const uint32_t c1 = fill_g1(nib(q1.c, 5)), c2 = nib(q2.c, 5);
    uint32_t e[2], c[2];
#pragma unroll
    for (int p = 0; p < 2; p++) {
        e[p] = halves(fill_g1(nib(S12, 2 * p)), fill_g1(nib(S12, 2 * p + 1)));
        c[p] = halves(((c2 >> (2 * p)) & 1u) ? c1 : 0u, ((c2 >> (2 * p + 1)) & 1u) ? c1 : 0u);
    }
    return make_uint4(e[0], e[1], c[0], c[1]);
}

PG_HD uint4 pair03(const LineMasks &q0, const LineMasks &q3)
{
    const uint32_t S03 = union_pairs2(q0.c, q3.c);  // g0 + 4 g3
    return make_uint4(both_halves(rep_g0(nib(S03, 0))), both_halves(rep_g0(nib(S03, 1))),
                      both_halves(rep_g0(nib(S03, 2))), both_halves(rep_g0(nib(S03, 3))));
}

PG_HD uint4 pair13(const LineMasks &q1, const LineMasks &q3)
{
    const uint32_t S13 = union_pairs6(q1.b, q3.b);  // g1 + 4 g3
    return make_uint4(both_halves(fill_g1(nib(S13, 0))), both_halves(fill_g1(nib(S13, 1))),
                      both_halves(fill_g1(nib(S13, 2))), both_halves(fill_g1(nib(S13, 3))));
}

PG_HD void pair23(const LineMasks &q2, const LineMasks &q3, uint4 out[3])
{
    const uint32_t S23 = union_pairs6(q2.a, q3.a);  // g2 + 4 g3
    uint32_t w[12];
#pragma unroll
    for (int g3 = 0; g3 < 4; g3++)
#pragma unroll
        for (int p = 0; p < 2; p++) w[2 * g3 + p] = bit_halfmask(S23, 2 * p + 4 * g3);
    const uint32_t a2 = nib(q2.c, 4);
    w[8] = bit_halfmask(a2, 0);
    w[9] = bit_halfmask(a2, 2);
    w[10] = nib(q3.c, 2) | (nib(q3.c, 3) << 4) | (nib(q3.c, 5) << 8);
    w[11] = 0;
    out[0] = make_uint4(w[0], w[1], w[2], w[3]);
    out[1] = make_uint4(w[4], w[5], w[6], w[7]);
    out[2] = make_uint4(w[8], w[9], w[10], w[11]);
}

// all-ones when bit i of x is set, else 0
PG_HD uint32_t bit_mask(uint32_t x, int i) { return ((x >> i) & 1u) ? 0xffffffffu : 0u; }

PG_HD Set256 five_assemble(const uint4 &t01, const uint4 &t02, const uint4 &t12, const uint4 &t03,
                           const uint4 &t13, const uint4 (&t23)[3])
{
    const uint32_t e02[2] = {t02.x, t02.y}, bw[2] = {t02.z, t02.w};
    const uint32_t e12[2] = {t12.x, t12.y}, cw[2] = {t12.z, t12.w};
    const uint32_t z03[4] = {t03.x, t03.y, t03.z, t03.w}, z13[4] = {t13.x, t13.y, t13.z, t13.w};
    const uint32_t s23[8] = {t23[0].x, t23[0].y, t23[0].z, t23[0].w, t23[1].x, t23[1].y, t23[1].z, t23[1].w};
    const uint32_t a2m[2] = {t23[2].x, t23[2].y}, nb = t23[2].z;
    uint32_t Y[2], Z[4];
#pragma unroll
    for (int p = 0; p < 2; p++) Y[p] = e02[p] | e12[p] | t01.x | (t01.y & a2m[p]);
#pragma unroll
    for (int g3 = 0; g3 < 4; g3++) Z[g3] = z03[g3] | z13[g3] | (t01.z & bit_mask(nb, g3));
    Set256 r;
#pragma unroll
    for (int g3 = 0; g3 < 4; g3++) {
        const uint32_t bm = bit_mask(nb, 4 + g3), cm = bit_mask(nb, 8 + g3);
#pragma unroll
        for (int p = 0; p < 2; p++)
            r.w[2 * g3 + p] = Y[p] | Z[g3] | s23[2 * g3 + p] | (bw[p] & bm) | (cw[p] & cm);
    }
    return r;
}

// The five-set of one colour from the line masks of its four quadrants.
PG_HD Set256 five_set(const LineMasks &q0, const LineMasks &q1, const LineMasks &q2,
                      const LineMasks &q3)
{
    uint4 t23[3];
    pair23(q2, q3, t23);
    return five_assemble(pair01(q0, q1), pair02(q0, q2), pair12(q1, q2), pair03(q0, q3), pair13(q1, q3), t23);
}

// ------------------------------------------------------------------------
// Value assembly (Section II recurrence on Section III tables).
//   Fc, Fo     five-sets of the side to move and of the other side
//   Wnt, Nnt   OR over children of (immediate win | rmax(not child N)) and
//              (immediate win | rmax(not child W))
// Terminal elements (a five of either colour) score f_c - f_cbar; the rest
// take the children.  W = notFo & (Fc | Wnt), N = Fc | (notFo & Nnt).
// ------------------------------------------------------------------------
PG_HD void combine(const Set256 &Fc, const Set256 &Fo, const Set256 &Wnt, const Set256 &Nnt,
                   Set256 &W, Set256 &N)
{
#pragma unroll
    for (int i = 0; i < 8; i++) {
        W.w[i] = ~Fo.w[i] & (Fc.w[i] | Wnt.w[i]);
        N.w[i] = Fc.w[i] | (~Fo.w[i] & Nnt.w[i]);
    }
}

// The two sets a parent ORs in for one child t (side to move in t = the
// parent's opponent): A = F_parent(t) | rmax(not N_t), B = F_parent(t) | rmax(not W_t).
PG_HD void child_terms(const Set256 &Fparent_t, const Set256 &Wt, const Set256 &Nt, Set256 &A,
                       Set256 &B)
{
    // rmax(not X) = not rmin(X)
    const Set256 a = rmin(Nt);
    const Set256 b = rmin(Wt);
#pragma unroll
    for (int i = 0; i < 8; i++) {
        A.w[i] = Fparent_t.w[i] | ~a.w[i];
        B.w[i] = Fparent_t.w[i] | ~b.w[i];
    }
}

}  // namespace pg
