// tables.cpp -- construction of the host-side quadrant and DAG tables.
#include "tables.h"

#include <stdexcept>

#include <algorithm>
#include <mutex>

namespace pg {

int popcount9(unsigned x)
{
    int n = 0;
    for (; x; x &= x - 1) n++;
    return n;
}

static int pow3(int l)
{
    int p = 1;
    while (l-- > 0) p *= 3;
    return p;
}

// local cell after one counter-clockwise turn: (lr, lc) -> (2 - lc, lr)
static int turn_cell(int l)
{
    const int lr = l / 3, lc = l % 3;
    return 3 * (2 - lc) + lr;
}

// local cell after the left-right mirror: (lr, lc) -> (lr, 2 - lc)
static int mirror_cell(int l) { return 3 * (l / 3) + 2 - l % 3; }

static unsigned turn_mask(unsigned m, int k)
{
    for (int t = 0; t < k; t++) {
        unsigned r = 0;
        for (int l = 0; l < 9; l++)
            if (m >> l & 1) r |= 1u << turn_cell(l);
        m = r;
    }
    return m;
}

// The 32 lines of the board with the field/nibble each quadrant keeps them in
// (layout documented at LineMasks in set256.h).
struct LineDef {
    int cells[5];
    int group;  // 0 rows top, 1 rows bottom, 2 cols left, 3 cols right, 4 diag, 5 anti, 6.. triples
    int slot;   // index inside a two-quadrant group; triple id for groups >= 6
};

static std::vector<LineDef> all_lines()
{
    std::vector<LineDef> out;
    for (int r = 0; r < 6; r++)
        for (int c0 = 0; c0 < 2; c0++) {
            LineDef d;
            for (int i = 0; i < 5; i++) d.cells[i] = 6 * r + c0 + i;
            d.group = r < 3 ? 0 : 1;
            d.slot = 2 * (r % 3) + c0;
            out.push_back(d);
        }
    for (int c = 0; c < 6; c++)
        for (int r0 = 0; r0 < 2; r0++) {
            LineDef d;
            for (int i = 0; i < 5; i++) d.cells[i] = 6 * (r0 + i) + c;
            d.group = c < 3 ? 2 : 3;
            d.slot = 2 * (c % 3) + r0;
            out.push_back(d);
        }
    // diagonals down-right from (r0, c0)
    const int diag[4][2] = {{0, 0}, {1, 1}, {0, 1}, {1, 0}};
    for (int k = 0; k < 4; k++) {
        LineDef d;
        for (int i = 0; i < 5; i++) d.cells[i] = 6 * (diag[k][0] + i) + diag[k][1] + i;
        if (k < 2) { d.group = 4; d.slot = k; }
        else { d.group = 6; d.slot = k == 2 ? 0 : 1; }  // (0,1): T013, (1,0): T023
        out.push_back(d);
    }
    // anti-diagonals down-left from (r0, c0)
    const int anti[4][2] = {{0, 5}, {1, 4}, {0, 4}, {1, 5}};
    for (int k = 0; k < 4; k++) {
        LineDef d;
        for (int i = 0; i < 5; i++) d.cells[i] = 6 * (anti[k][0] + i) + anti[k][1] - i;
        if (k < 2) { d.group = 5; d.slot = k; }
        else { d.group = 6; d.slot = k == 2 ? 2 : 3; }  // (0,4): T012, (1,5): T123
        out.push_back(d);
    }
    return out;
}

// Field and nibble in which quadrant q keeps line d (layout at LineMasks).
static void line_slot(const LineDef &d, int *field, int *pos)
{
    if (d.group < 4) {
        *field = (d.group == 0 || d.group == 1) ? 0 : 1;
        *pos = d.slot;
    } else if (d.group < 6) {
        *field = 2;
        *pos = d.slot;
    } else {
        *field = 2;
        *pos = 2 + d.slot;
    }
}

static void build_line_masks(HostTables &t)
{
    t.lm.assign(4 * 512, LineMasks{0, 0, 0});
    const std::vector<LineDef> lines = all_lines();
    for (const LineDef &d : lines) {
        for (int q = 0; q < 4; q++) {
            unsigned cells = 0;
            for (int i = 0; i < 5; i++) {
                const int r = d.cells[i] / 6, c = d.cells[i] % 6;
                if (2 * (r / 3) + c / 3 == q) cells |= 1u << (3 * (r % 3) + c % 3);
            }
            if (!cells) continue;
            // which field/nibble of quadrant q's record holds this line
            int field, pos;
            line_slot(d, &field, &pos);
            for (unsigned m = 0; m < 512; m++) {
                unsigned mu = 0;
                for (int k = 0; k < 4; k++)
                    if ((turn_mask(m, k) & cells) == cells) mu |= 1u << k;
                LineMasks &rec = t.lm[q * 512 + m];
                uint32_t &f = field == 0 ? rec.a : field == 1 ? rec.b : rec.c;
                f |= mu << (4 * pos);
            }
        }
    }
}

static int line_quadrants(const LineDef &d)
{
    int m = 0;
    for (int i = 0; i < 5; i++) {
        const int r = d.cells[i] / 6, c = d.cells[i] % 6;
        m |= 1 << (2 * (r / 3) + c / 3);
    }
    return m;
}

static void build_line_structure(HostTables &t)
{
    t.sel.assign(4 * 512 * 4, 0);
    for (int j = 0; j < 4; j++)
        for (int m = 0; m < 512; m++) {
            const LineMasks &L = t.lm[j * 512 + m];
            const uint32_t f[3] = {L.a, L.b, L.c};
            for (int k = 0; k < 4; k++) {
                uint32_t off = 0;
                for (int ff = 0; ff < 3; ff++) {
                    uint32_t sigma = 0;
                    for (int sl = 0; sl < 6; sl++)
                        if ((f[ff] >> (4 * sl + k)) & 1) sigma |= 1u << sl;
                    // byte offset of entry sigma of chunk ff: 8 * (64 ff + sigma)
                    off |= (8u * (64u * ff + sigma)) << (10 * ff);
                }
                t.sel[(j * 512 + m) * 4 + k] = off;
            }
        }
    t.chunk_ref.assign(4 * 18, 0xffff);
    t.u_ref.assign(4 * 15, 0xffffffffu);
    const std::vector<LineDef> lines = all_lines();
    for (int D = 0; D < 4; D++) {
        int nu = 0;
        for (const LineDef &d : lines) {
            const int qm = line_quadrants(d);
            int field, pos;
            line_slot(d, &field, &pos);
            uint32_t refs = 0xffffffffu;
            int nr = 0;
            for (int j = 0; j < 4; j++) {
                if (!((qm >> j) & 1) || j == D) continue;
                const uint32_t ref = (uint32_t)(j | (field << 2) | (pos << 4));
                refs = (refs & ~(0xffu << (8 * nr))) | (ref << (8 * nr));
                nr++;
            }
            if ((qm >> D) & 1) t.chunk_ref[D * 18 + 6 * field + pos] = (uint16_t)(refs & 0xffff);
            else t.u_ref[D * 15 + nu++] = refs;
        }
    }
}

// Pattern maps of the 8 board symmetries (see HostTables::symmap).  With
// lam the local map of symmetry sym, an image pattern c' comes from the
// source pattern c = canonical form of lam^-1(c'); lam(c) is c' turned by
// some h, read off the canonicalising turn count of lam(c).
static void build_symmetry(HostTables &t)
{
    const int NC = 19683;
    std::vector<uint16_t> mirror1(NC);
    for (int code = 0; code < NC; code++) {
        int r = 0;
        for (int l = 0; l < 9; l++) r += (code / pow3(l)) % 3 * pow3(mirror_cell(l));
        mirror1[code] = (uint16_t)r;
    }
    auto turns = [&](int code, int k) {
        for (int i = 0; i < (k & 3); i++) code = t.turn1[code];
        return code;
    };
    t.symmap.assign(8 * kPatterns, 0);
    t.symcode.assign(8 * NC, 0);
    for (int sym = 0; sym < 8; sym++)
        for (int code = 0; code < NC; code++) {
            int x = turns(code, 4 - (sym & 3));
            if (sym & 4) x = mirror1[x];
            t.symcode[sym * NC + code] = (uint16_t)x;
        }
    for (int sym = 0; sym < 8; sym++) {
        const int r = sym & 3;
        const bool f = (sym & 4) != 0;
        for (int b = 0; b <= 9; b++)
            for (int w = 0; b + w <= 9; w++) {
                const int start = t.class_start[b][w];
                for (int i = 0; i < t.class_size[b][w]; i++) {
                    const int img = t.qinfo[start + i].code;
                    int x = turns(img, 4 - r);          // lam^-1 = mirror^f . turn^-r
                    if (f) x = mirror1[x];
                    const int src = t.canon[x] & 0xfff;
                    int y = t.qinfo[start + src].code;  // lam(c) = turn^r . mirror^f (c)
                    if (f) y = mirror1[y];
                    y = turns(y, r);
                    // y turned by K (its canonicalising count) is c', so y = c' turned -K
                    const int K = t.canon[y] >> 12;
                    if ((t.canon[y] & 0xfff) != i) throw std::logic_error("symmetry map");
                    t.symmap[sym * kPatterns + start + i] = (uint16_t)(src | (((4 - K) & 3) << 12));
                }
            }
    }
    // the inverse permutation of each class under each symmetry
    t.syminv.assign(8 * kPatterns, 0xffff);
    for (int sym = 0; sym < 8; sym++)
        for (int b = 0; b <= 9; b++)
            for (int w = 0; b + w <= 9; w++) {
                const int start = t.class_start[b][w];
                for (int i = 0; i < t.class_size[b][w]; i++) {
                    uint16_t &slot = t.syminv[sym * kPatterns + start + (t.symmap[sym * kPatterns + start + i] & 0xfff)];
                    if (slot != 0xffff) throw std::logic_error("symmetry map is not a permutation");
                    slot = (uint16_t)i;
                }
            }
}

static void build_pattern_lookups(HostTables &t)
{
    static const int pow3[9] = {1, 3, 9, 27, 81, 243, 729, 2187, 6561};
    t.pat_lm.assign(4 * kPatterns * 2, LineMasks{0, 0, 0});
    t.pat_sel.assign(4 * kPatterns * 2 * 2 * 4, 0);
    t.pat_child.assign(kPatterns * 2, PosChild{});
    for (int p = 0; p < kPatterns; p++) {
        const QInfo &q = t.qinfo[p];
        for (int x = 1; x <= 2; x++) {
            const unsigned mine = x == 1 ? q.bm : q.wm, other = x == 1 ? q.wm : q.bm;
            for (int j = 0; j < 4; j++) {
                t.pat_lm[(j * kPatterns + p) * 2 + x - 1] = t.lm[j * 512 + mine];
                uint32_t *ps = &t.pat_sel[((j * kPatterns + p) * 2 + x - 1) * 8];
                for (int w = 0; w < 4; w++) {
                    ps[w] = t.sel[(j * 512 + mine) * 4 + w];
                    ps[4 + w] = t.sel[(j * 512 + other) * 4 + w];
                }
            }
            PosChild &r = t.pat_child[p * 2 + x - 1];
            r.nchild = 0;
            for (int cell = 0; cell < 9; cell++)
                if (!(((q.bm | q.wm) >> cell) & 1u)) r.child[r.nchild++] = t.canon[q.code + x * pow3[cell]];
        }
    }
}

static void build(HostTables &t)
{
    const int NC = 19683;
    t.turn1.resize(NC);
    for (int code = 0; code < NC; code++) {
        int r = 0;
        for (int l = 0; l < 9; l++) r += (code / pow3(l)) % 3 * pow3(turn_cell(l));
        t.turn1[code] = (uint16_t)r;
    }
    std::vector<int> minc(NC), mink(NC);
    for (int code = 0; code < NC; code++) {
        int best = code, bk = 0, cur = code;
        for (int k = 1; k < 4; k++) {
            cur = t.turn1[cur];
            if (cur < best) { best = cur; bk = k; }
        }
        minc[code] = best;
        mink[code] = bk;
    }
    std::vector<int> index(NC, -1);
    t.qinfo.clear();
    for (int b = 0; b <= 9; b++)
        for (int w = 0; w <= 9; w++) {
            t.class_start[b][w] = (int)t.qinfo.size();
            t.class_size[b][w] = 0;
            if (b + w > 9) continue;
            for (int code = 0; code < NC; code++) {
                if (minc[code] != code) continue;
                unsigned bm = 0, wm = 0;
                for (int l = 0; l < 9; l++) {
                    const int dgt = (code / pow3(l)) % 3;
                    if (dgt == 1) bm |= 1u << l;
                    if (dgt == 2) wm |= 1u << l;
                }
                if (popcount9(bm) != b || popcount9(wm) != w) continue;
                index[code] = t.class_size[b][w]++;
                t.qinfo.push_back(QInfo{(uint16_t)code, (uint16_t)bm, (uint16_t)wm, 0});
            }
        }
    t.canon.resize(NC);
    for (int code = 0; code < NC; code++)
        t.canon[code] = (uint16_t)(index[minc[code]] | (mink[code] << 12));
    build_symmetry(t);
    build_line_masks(t);
    build_line_structure(t);
    build_pattern_lookups(t);
}

const HostTables &host_tables()
{
    static HostTables t;
    static std::once_flag once;
    std::call_once(once, [] { build(t); });
    return t;
}

static void build_dag(DagLayout &L, int e)
{
    L.e = e;
    int n3 = 1;
    for (int i = 0; i < e; i++) n3 *= 3;
    L.rank.assign(n3, 0xffff);
    L.layer_start.assign(e + 2, 0);
    L.node.clear();
    L.max_layer = 0;
    for (int t = 0; t <= e; t++) {
        L.layer_start[t] = (int)L.node.size();
        const int nc = (t + 1) / 2, no = t / 2;
        for (unsigned filled = 0; filled < (1u << e); filled++) {
            if (popcount9(filled) != t) continue;
            for (unsigned cm = filled;; cm = (cm - 1) & filled) {
                if (popcount9(cm) == nc) {
                    const unsigned om = filled & ~cm;
                    (void)no;
                    int code = 0;
                    for (int s = e - 1; s >= 0; s--) code = 3 * code + ((cm >> s & 1) ? 1 : (om >> s & 1) ? 2 : 0);
                    L.rank[code] = (uint16_t)(L.node.size() - L.layer_start[t]);
                    L.node.push_back(cm | (om << 16));
                }
                if (cm == 0) break;
            }
        }
        L.max_layer = std::max(L.max_layer, (int)L.node.size() - L.layer_start[t]);
    }
    L.layer_start[e + 1] = (int)L.node.size();
    L.sub_mask.clear();
    L.sub_rank.assign(1u << e, 0);
    L.sub_start.assign(e + 2, 0);
    L.max_subsets = 0;
    for (int sz = 0; sz <= e; sz++) {
        L.sub_start[sz] = (int)L.sub_mask.size();
        for (unsigned m = 0; m < (1u << e); m++)
            if (popcount9(m) == sz) {
                L.sub_rank[m] = (uint16_t)(L.sub_mask.size() - L.sub_start[sz]);
                L.sub_mask.push_back((uint16_t)m);
            }
        L.max_subsets = std::max(L.max_subsets, (int)L.sub_mask.size() - L.sub_start[sz]);
    }
    // per node: five-set table entries and child indices (the side to move
    // at layer t is the root's mover for even t, digit 1, else digit 2)
    L.edge.assign(L.node.size() * kDagEdgeWords, 0);
    for (int t = 0; t <= e; t++) {
        const int digit = (t & 1) ? 2 : 1;
        for (int i = L.layer_start[t]; i < L.layer_start[t + 1]; i++) {
            const unsigned cm = L.node[i] & 0xffffu, om = L.node[i] >> 16;
            uint16_t *rec = &L.edge[(size_t)i * kDagEdgeWords];
            rec[0] = L.sub_rank[cm];
            rec[1] = L.sub_rank[om];
            if (t == e) continue;
            int code = 0;
            for (int s2 = e - 1; s2 >= 0; s2--) code = 3 * code + ((cm >> s2 & 1) ? 1 : (om >> s2 & 1) ? 2 : 0);
            int pw = 1, k = 2;
            for (int sl = 0; sl < e; sl++, pw *= 3)
                if (!((cm | om) >> sl & 1)) rec[k++] = L.rank[code + digit * pw];
        }
    }
    L.sub_start[e + 1] = (int)L.sub_mask.size();
}

const DagLayout &dag_layout(int e)
{
    static DagLayout L[11];
    static std::once_flag once;
    std::call_once(once, [] {
        for (int k = 0; k <= 10; k++) build_dag(L[k], k);
    });
    return L[e];
}

}  // namespace pg
