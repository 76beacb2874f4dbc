// kernels.h -- device-side job descriptions shared by the kernels and the
// host launch code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "set256.h"
#include "tables.h"

namespace pg {

// Read-only tables in device memory (one copy per device).
struct DevTables {
    const uint16_t *canon;   // [19683] index in class | k << 12
    const QInfo *qinfo;      // [4995]
    const LineMasks *lm;     // [4 * 512]
    const uint4 *sel;        // [4 * 512]: per quadrant and stone mask, the selectors for k = 0..3
    const uint16_t *chunk_ref;  // [4 * 18]
    const uint32_t *u_ref;      // [4 * 15]
    const uint32_t *dag_node;   // all DAG layouts back to back (cmask | omask << 16)
    const uint16_t *dag_rank;   // all rank tables back to back
    const uint4 *dag_edge;      // all per-node edge records back to back (kDagEdgeWords u16 = 2 uint4 each)
    int dag_node_off[11];       // start of layout e in dag_node (and, in records, in dag_edge)
    int dag_rank_off[11];       // start of layout e in dag_rank
    int dag_layer[11][12];      // layer starts (relative) of layout e
    int dag_max[11];            // largest layer of layout e
    const uint16_t *dag_sub_mask;  // subsets of the e slots by size, all e back to back
    const uint16_t *dag_sub_rank;  // rank of a subset within its size, all e back to back
    int dag_sub_off[11];        // start of layout e in both (2^e entries each)
    int dag_sub_start[11][12];  // start of size s within layout e
    int dag_sub_max[11];        // largest C(e, s)
    const uint16_t *symmap;     // [8 * kPatterns]: source pattern | turns << 12 per symmetry
    const uint16_t *symcode;    // [8 * 19683]: preimage of a quadrant code under each symmetry
    const uint16_t *syminv;     // [8 * kPatterns]: image pattern per source pattern (inverse of symmap)
    const LineMasks *pat_lm;    // per-pattern lookups of the tile set-up (HostTables)
    const uint4 *pat_sel;
    const PosChild *pat_child;
};

// The table of the image section sym(s) from the table of s (Section III,
// transforms of tables under the board symmetries).
struct SymJob {
    int sym;
    int m[4];           // image shape
    int sm[4];          // source shape
    int qb[4];          // first QInfo index of each image quadrant class
    int nb[4];          // blocks of the image per dimension
    long long nblocks;  // image blocks
    long long nchunks;  // workgroups: 4 quarters of each block, blocks padded to a multiple of 8
    const uint4 *src;
    uint4 *dst;
};

// One section sweep (Section IV): a parent section, its child sections and
// the tiling of its entries into lines along dimension d (Fig. 3: a line of
// a parent depends on one line of the child section along the same dimension).
struct SweepJob {
    int m[4];          // parent shape
    int qb[4];         // first QInfo index of each parent quadrant class
    int cm[4];         // child extent along dimension j (0: quadrant j full)
    int cqb[4];        // first QInfo index of the child class of quadrant j
    const uint4 *child[4];
    const uint4 *prep[4];   // prepared child terms of dimensions not staged (read)
    uint4 *prep_out[4];     // where prep_kernel writes them (same buffers)
    uint4 *out;
    int mover;         // 1 black, 2 white
    int d;             // dimension whose child lines are staged in LDS
    int nchd;          // empty cells of quadrant d (children of every parent along d; 0: none)
    int emask;         // dimensions whose quadrant has empty cells
    int odmask;        // dimensions whose children are full boards evaluated on demand
    int e;             // dimension that groups G lines into a tile (3, or 2 when d == 3)
    int G;             // lines per tile
    int ngroups;       // ceil(m[e] / G)
    int o1, o2;        // the remaining two dimensions
    long long ntiles;
    int lds_bytes;     // dynamic LDS needed by one tile
    int threads;       // workgroup size of the one-section sweep (256 or 512)
    int order;         // tile order of the one-section sweep (0 natural, 1 by XCD)
    // Children held as their representatives under the board symmetries:
    // child[j] is then the table of a section whose image under symmetry
    // csym[j] is child j (0: child[j] is child j itself); rm[j] is that
    // section's shape and rsrc[j][k] its dimension that child dimension k
    // comes from.
    int csym[4];
    int rm[4][4];
    int rsrc[4][4];
};

// Host launchers (sweep.hip, endgame.hip, symmetry.hip).
hipError_t launch_sweep(const SweepJob &job, const DevTables &T, hipStream_t s);
hipError_t launch_transform(const SymJob &job, const DevTables &T, hipStream_t s);
// A section of full boards (no empty cell): one launch over half-blocks.
hipError_t launch_terminal(const SweepJob &job, const DevTables &T, hipStream_t s);
// Prepare the A/B child terms of dimension j (j in emask, j != d).
hipError_t launch_prep(const SweepJob &job, int j, const DevTables &T, hipStream_t s);
hipError_t launch_prep_batch(const SweepJob *dev_jobs, const int *dev_unit,
                             const long long *dev_chunk_start, int nunits, long long total_chunks,
                             const DevTables &T, hipStream_t s);
// One workgroup of `threads` (256 or 512) per tile of jobs [0, njobs)
// (tile_start: first global tile of each job).  sym: jobs whose children may
// be held as their representatives (csym).
hipError_t launch_sweep_batch(const SweepJob *dev_jobs, const long long *dev_tile_start, int njobs,
                              long long total_tiles, int lds_bytes, int threads, bool sym, const DevTables &T,
                              hipStream_t s);

// Endgame (Section VIII serial solver, one DAG per root).
struct EvalScratch {
    int *count;          // [16]: per empties count 0..10, [11] invalid
    int *start;          // [16]
    int *cursor;         // [16]
    int *order;          // [n] roots sorted by empties, most first
    uint8_t *empties;    // [n]
    unsigned long long *counter;  // work counter of the persistent launch
    uint4 *global_layers;         // DAG layers for roots with 9-10 empties
    int global_slots;             // number of roots the global layer buffer holds at once
};

hipError_t launch_eval_bin(const uint64_t *boards, size_t n, const EvalScratch &S, int *status,
                           uint4 *out, const DevTables &T, hipStream_t s);
hipError_t launch_eval_persistent(const uint64_t *boards, size_t n, uint4 *out,
                                  const EvalScratch &S, int grid, const DevTables &T,
                                  hipStream_t s);
// The same with only the first `slots` workgroups of class 0 owning a global
// layer slot (1 <= slots <= grid; global_layers holds `slots` slots).
hipError_t launch_eval_persistent_slots(const uint64_t *boards, size_t n, uint4 *out,
                                        const EvalScratch &S, int grid, int slots,
                                        const DevTables &T, hipStream_t s);
// Workgroup sizes of persistent endgame classes 0 and 1 (256 or 512), set
// by the endgame autotuner; process-wide.
void set_eval_class_threads(int c0, int c1);
void get_eval_class_threads(int *c0, int *c1);
hipError_t launch_eval_group(const uint64_t *boards, int e, int first, int count, uint4 *out,
                             const EvalScratch &S, const DevTables &T, hipStream_t s);

// One batch of roots of a single class (0: 8-10 empty cells, 9-10 needing
// global_layers; 1: 7; 2: up to 6), taken in order, no binning.
hipError_t launch_eval_direct(const uint64_t *boards, int n, uint4 *out, int cls,
                              unsigned long long *counter, uint4 *global_layers, int grid,
                              const DevTables &T, hipStream_t s);
int dag_lds_bytes(int e);
int dag_ftab_bytes(int e);

// A solved section kept resident for lookups.
// A lookup's section code: resident section index | symmetry << 24 (the
// query's section is the image of the resident one under that symmetry).
struct ResidentSection {
    const uint4 *table;
    int m[4];
};
hipError_t launch_lookup(const uint64_t *boards, const int *sec_of, int n,
                         const ResidentSection *secs, uint4 *out, const DevTables &T, hipStream_t s);
// Dynamic LDS of one sweep tile: G lines of mD parents, child lines of cmD
// entries (cmD = 0 when the staged dimension has no children).
int sweep_lds_bytes(int G, int mD, int cmD);

// Nodes of the largest layer of any supported root (10 empty cells).
constexpr int kDagGlobalLayer = 4200;

}  // namespace pg
