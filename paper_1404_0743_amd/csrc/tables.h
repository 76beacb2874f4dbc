// tables.h -- quadrant tables of the library (Section IV: rotation-minimal
// quadrant patterns per (black, white) class and their ordering; Section III:
// per-quadrant line masks for the five-in-a-row sets over L).
#pragma once
#include <stdint.h>

#include <vector>

#include "set256.h"

namespace pg {

// Rotation-minimal quadrant patterns over all (black, white) classes.
constexpr int kPatterns = 4995;

// One rotation-minimal quadrant pattern.
struct QInfo {
    uint16_t code;   // ternary code, digit 0 empty / 1 black / 2 white at 3^local
    uint16_t bm, wm; // 9-bit black and white stone masks
    uint16_t pad;
};

// The children of a pattern when one side moves: per empty cell, in
// increasing cell order, the canonical child (class index | turns << 12).
struct alignas(4) PosChild {
    uint16_t nchild, child[9];
};

struct HostTables {
    int class_start[10][10];
    int class_size[10][10];
    std::vector<QInfo> qinfo;     // 4995 patterns, class by class, increasing code
    std::vector<uint16_t> canon;  // per code: index in its class | (k << 12), where
                                  // k = least number of turns taking the code to
                                  // its class representative
    std::vector<uint16_t> turn1;  // per code: code after one counter-clockwise turn
    std::vector<LineMasks> lm;    // [quadrant * 512 + stone mask]

    // Board symmetries (Section III: the group G of approximate symmetries
    // contains the 8 board symmetries, which move each quadrant onto a
    // quadrant, sym_quadrant in set256.h, and act on its nine cells by one
    // local map: a mirror when the symmetry is a reflection, then sym & 3
    // counter-clockwise turns).  symmap[sym * kPatterns + i], for pattern i
    // (qinfo order) of an image section: the index, within the same class, of
    // the source pattern whose local image is a turn of pattern i, | h << 12,
    // where that local image is pattern i turned h more times (h = 0..3).
    std::vector<uint16_t> symmap;  // [8 * kPatterns]
    // syminv[sym * kPatterns + start + u]: the pattern i of the class starting
    // at start whose symmap entry names source pattern u (symmap is a
    // permutation of each class)
    std::vector<uint16_t> syminv;  // [8 * kPatterns]
    // symcode[sym * 19683 + c]: the quadrant code that the local map of
    // symmetry sym takes to c (its preimage: mirror^f of c turned -r times).
    std::vector<uint16_t> symcode;  // [8 * 19683]

    // Line structure used by the sweep (five_lut in sweep.hip):
    // sel[(j * 512 + m) * 4 + k] describes the lines through quadrant j that
    // its stone mask m completes after k turns.  For each field f = a, b, c of
    // LineMasks the 6-bit set sigma_f (bit s iff nibble s of field f of
    // lm[j*512+m] contains k) is stored as the byte offset 8 * (64 f + sigma_f)
    // of its entry in a line's chunk tables, in bits [10 f, 10 f + 10) (the
    // third field takes 11 bits).
    std::vector<uint32_t> sel;    // [4 * 512 * 4]
    // chunk_ref[D * 18 + 6f + s]: the other quadrants of the line kept in
    // nibble s of field f of quadrant D's LineMasks, as up to two refs
    // (quadrant | field << 2 | nibble << 4), 0xff = none.
    std::vector<uint16_t> chunk_ref;  // [4 * 18]
    // u_ref[D * 15 + i]: the 15 lines that miss quadrant D, each as up to
    // three refs (byte per ref, 0xff = none).
    std::vector<uint32_t> u_ref;      // [4 * 15]

    // Per-pattern lookups of the sweep's tile set-up, each one load instead of
    // a chain (pattern record, then the table it indexes), for pattern p
    // (qinfo order), quadrant j and side x / mover c (1 black, 2 white):
    // pat_lm[(j * kPatterns + p) * 2 + x - 1] = lm[j * 512 + stones of x in p];
    // pat_sel[((j * kPatterns + p) * 2 + c - 1) * 2 + 0 / 1] = sel entries
    // (4 words each, k = 0..3) of the mover's / the other side's stones of p;
    // pat_child[p * 2 + c - 1] = the children of p when c moves.
    std::vector<LineMasks> pat_lm;     // [4 * kPatterns * 2]
    std::vector<uint32_t> pat_sel;     // [4 * kPatterns * 2 * 2 * 4]
    std::vector<PosChild> pat_child;   // [kPatterns * 2]
};

// Built once on first use (thread-safe).
const HostTables &host_tables();

// Endgame DAG layout for a board with e empty cells (the serial solver of
// Section VIII): node (t, cmask, omask) has t stones placed in the empty
// cells, alternately by the side to move (cmask, ceil(t/2) cells) and the
// other side (omask, floor(t/2) cells).  Layer t holds C(e,t)*C(t,floor(t/2))
// nodes.  Nodes are stored layer by layer; rank[] maps a ternary slot
// assignment (digit 1 = mover, 2 = other, base 3 over slots) to the node's
// index within its layer.
struct DagLayout {
    int e;
    std::vector<int> layer_start;   // e + 2 entries
    std::vector<uint32_t> node;     // cmask | omask << 16, layer by layer
    std::vector<uint16_t> rank;     // 3^e entries
    int max_layer;
    // subsets of the e slots by size: sub_mask lists the masks of size 0,
    // then size 1, ... (increasing within a size), sub_start[s] where size s
    // starts (e + 2 entries); sub_rank[mask] = its index within its size
    std::vector<uint16_t> sub_mask, sub_rank;
    std::vector<int> sub_start;
    int max_subsets;                // largest C(e, s)
    // per node (layer order), kDagEdgeWords u16: the ranks of cmask and
    // omask among the subsets of their sizes (their five-set table entries),
    // then the index in layer t + 1 of the child on each free slot, in
    // increasing slot order; unused words are 0
    std::vector<uint16_t> edge;
};

constexpr int kDagEdgeWords = 16;

const DagLayout &dag_layout(int e);

int popcount9(unsigned x);

}  // namespace pg
