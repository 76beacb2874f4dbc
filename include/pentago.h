/*
 * pentago.h -- C ABI of the MI355X (gfx950) pentago retrograde library.
 *
 * The library computes exact rotation-abstracted values of pentago positions
 * (Irving, "Pentago is a First Player Win", arXiv:1404.0743):
 *   - the n+1 -> n layer sweep over one section or many sections
 *     (Section II recurrence, Section III rotation abstraction, Section IV
 *     sections and 8^4 blocks),
 *   - exact values of arbitrary boards solved to the full board (the serial
 *     endgame solver of Section VIII, rotations handled by rmax only),
 *   - a query server that answers boards from resident sections or by search.
 *
 * Conventions (fixed by this library; the paper leaves them open):
 *   cell        6*r + c, r counted downward, c rightward
 *   quadrant    2*(r/3) + c/3: 0 top-left, 1 top-right, 2 bottom-left, 3 bottom-right
 *   local cell  3*(r%3) + c%3; a quadrant pattern is the ternary code
 *               sum_l digit_l * 3^l with digit 0 empty, 1 black, 2 white
 *   one turn    90 degrees counter-clockwise: local (lr, lc) moves to (2-lc, lr)
 *   L = Z4^4    g = g0 + 4*g1 + 16*g2 + 64*g3, g_j counter-clockwise turns of quadrant j
 *   side to move  black when the black and white counts are equal, white when
 *               black has one more (Section II validity)
 *
 * Memory: every pointer named "device" is device memory of the current HIP
 * device, allocated and owned by the caller; the library only borrows it for
 * the call (or, for the server, until destroy).  Host pointers are read
 * during the call only.  Calls that take a hip_stream are stream-ordered and
 * asynchronous: they return after enqueueing, results are ready when the
 * stream reaches them.  A NULL stream means the default stream.
 *
 * Errors: every function returns 0 on success or a negative PENTAGO_E* code.
 * No C++ exception crosses this boundary.  pentago_strerror() names a code;
 * pentago_last_error() gives the detail of the calling thread's last failure.
 */
#ifndef PENTAGO_H
#define PENTAGO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PENTAGO_OK 0
#define PENTAGO_EINVAL (-1)   /* bad counts, board, index, size or NULL argument */
#define PENTAGO_ENOCHILD (-2) /* a child section table that is needed is NULL */
#define PENTAGO_ENOMEM (-3)   /* the library could not allocate its own scratch */
#define PENTAGO_ERANGE (-4)   /* a size beyond what the call supports */
#define PENTAGO_EAGAIN (-5)   /* try again: queue full, or result not ready */
#define PENTAGO_EDEVICE (-6)  /* a HIP runtime error; see pentago_last_error() */

/* A set of elements of L: bit g lives in w[g >> 6] at position g & 63. */
typedef struct {
    uint64_t w[4];
} pentago_set256;

/* The rotation-abstracted value of one board b (Section III): for every g in
 * L, win has bit g iff the side to move wins g.b, notlose has bit g iff it
 * does not lose.  64 bytes.  Invariant: win is a subset of notlose. */
typedef struct {
    pentago_set256 win, notlose;
} pentago_superinfo;

/* A concrete board: the ternary code of each quadrant (0 .. 19682). */
typedef struct {
    uint16_t q[4];
} pentago_board;

/* A section (Section IV): the boards with black[j] black and white[j]
 * white stones in quadrant j.  Valid iff black[j] + white[j] <= 9 for every j
 * and sum(black) - sum(white) is 0 or 1. */
typedef struct {
    uint8_t black[4], white[4];
} pentago_section;

/* ---------------------------------------------------------------- layout */

/* Shape of a section: shape[j] is the number of rotation-minimal patterns of
 * quadrant j's (black, white) class (Section IV, Fig. 4), entries their
 * product (number of superinfos), positions the number of boards
 * prod_j 9!/(b_j! w_j! (9-b_j-w_j)!).  Any output pointer may be NULL. */
int pentago_section_shape(pentago_section s, uint32_t shape[4], uint64_t *entries,
                          uint64_t *positions);

/* Offset (in superinfos) of entry idx in the section's table.  The table is
 * tiled in blocks of 8x8x8x8 entries (Section IV), smaller where a dimension
 * ends; blocks are stored in row-major order of block coordinates (dimension
 * 3 fastest), and the entries of a block row-major over its own extents. */
int pentago_section_offset(pentago_section s, const uint32_t idx[4], uint64_t *offset);

/* Board of entry idx: quadrant j holds the idx[j]-th rotation-minimal pattern
 * of its class, patterns ordered by increasing ternary code. */
int pentago_section_board(pentago_section s, const uint32_t idx[4], pentago_board *board);

/* The section whose table child[j] of pentago_solve_section must hold: s with
 * the side to move's count in quadrant j raised by one (Section IV: a stone
 * placed in quadrant j changes only that quadrant's index).  EINVAL if
 * quadrant j is full. */
int pentago_child_section(pentago_section s, int j, pentago_section *child);

/* ------------------------------------------------------- board symmetries */

/* The 8 board symmetries (Section III: with the quadrant turns L they form
 * the group G of approximate symmetries; values are unchanged by them).
 * sym = r + 4 f, 0 <= sym <= 7: mirror the board left-right when f is set
 * ((row, col) -> (row, 5 - col)), then turn the whole board r quarter turns
 * counter-clockwise ((row, col) -> (5 - col, row)).  Quadrant q moves to
 * quadrant pi(q): the rotation r = 1 sends 0 -> 2, 1 -> 0, 2 -> 3, 3 -> 1,
 * the mirror 0 <-> 1, 2 <-> 3.
 *
 * *image = the section holding the images of the boards of s: the counts of
 * quadrant q move to quadrant pi(q).  EINVAL for invalid counts or sym. */
int pentago_section_image(pentago_section s, int sym, pentago_section *image);

/* The sections of the slice with `stones` stones whose counts are least
 * among their images under the board symmetries (Section IV: the sections a
 * slice sweep computes), in lexicographic order of the count tuples.  Writes
 * at most cap of them to out; *count = how many there are (call with cap 0
 * to size out).  Host only.  EINVAL for stones outside 0..36. */
int pentago_slice_sections(int stones, pentago_section *out, size_t cap, size_t *count);

/* The representative of s under the board symmetries (Section IV: only
 * sections whose count tuple ((b0,w0),(b1,w1),(b2,w2),(b3,w3)) is least in
 * lexicographic order among its images are computed): *rep is that least
 * image and *sym a symmetry with pentago_section_image(*rep, *sym) == s
 * (sym = 0 when s is its own representative).  Host only. */
int pentago_section_standardize(pentago_section s, pentago_section *rep, int *sym);

/* The table of pentago_section_image(s, sym) from the table of s (Section
 * III: when the representative of a board changes, its table is shifted,
 * its dimensions transposed and, for a reflection, reversed).
 *   table  device, entries(s) x 64 B, blocked layout (read)
 *   out    device, entries(image) x 64 B (the same count), written completely;
 *          must not overlap table
 * Bit G of image entry e' is bit g of the source entry e whose boards map
 * onto e' (quadrant i of e goes to quadrant pi(i) of e', its pattern mirrored
 * for a reflection and turned to its rotation-minimal form), where
 * g_i = sign (G_pi(i) - h_pi(i)), sign = -1 for a reflection, and h_j turns
 * the local image of the source pattern to the pattern of e' (h_j = 1 for
 * every non-symmetric pattern under a rotation).  Stream-ordered and
 * asynchronous.  EINVAL for invalid counts, sym, NULL or overlapping
 * pointers; ERANGE for sections of 2^32 entries or more. */
int pentago_section_transform(pentago_section s, const pentago_superinfo *table, int sym,
                              pentago_superinfo *out, void *hip_stream);

/* ---------------------------------------------------------------- sweep */

/* The n+1 -> n sweep of one section (Section II recurrence on Section III
 * tables, Section IV data layout, Fig. 3 line structure).
 *   child[j]  device table of pentago_child_section(s, j) (entries x 64 B, in
 *             the blocked layout), or NULL when quadrant j is full.  When s
 *             has 35 stones its children are full boards: a NULL child[j] then
 *             selects on-demand evaluation of those boards.
 *   out       device, entries x 64 B, written completely.
 * Sections with 36 stones (no empty cell) are evaluated directly (f_c - f_cbar,
 * Section II).  out must not overlap any child table.  EINVAL for an invalid
 * section or NULL out; ENOCHILD for a missing child that is needed. */
int pentago_solve_section(pentago_section s, const pentago_superinfo *const child[4],
                          pentago_superinfo *out, void *hip_stream);

/* The sweep of section s with its children held only as their
 * representatives under the board symmetries (Section IV: only sections
 * whose counts are least among their images are computed).
 *   rep[j]  device table of the representative of pentago_child_section(s, j)
 *           (pentago_section_standardize), or NULL when quadrant j is full or
 *           its child is a 36-stone section evaluated on demand.
 *   out     as in pentago_solve_section; must not overlap any rep[j].
 * Each child entry the sweep needs is read from the representative's table
 * and transformed in registers as pentago_section_transform would (no
 * scratch memory, no extra pass).  The result is bit for bit the
 * pentago_solve_section result with the children themselves.  Errors as
 * pentago_solve_section. */
int pentago_solve_section_d4(pentago_section s, const pentago_superinfo *const rep[4],
                             pentago_superinfo *out, void *hip_stream);

/* Tile shape of the sweep: lines of the section along the staged quadrant
 * per tile (1..8), threads per workgroup (256 or 512), and the order in
 * which workgroups take tiles (0: tile = workgroup index; 1: each of the 8
 * XCDs of the GPU, which receive workgroups in turn, takes a contiguous range
 * of tiles). */
typedef struct {
    int32_t lines;
    int32_t threads;
    int32_t order;
} pentago_tile_shape;

/* The tile autotuner: times every tile shape the section admits with HIP
 * events on hip_stream, remembers the fastest for this section geometry
 * (later pentago_solve_section calls with the same geometry use it;
 * pentago_solve_sections uses its lines per tile) and leaves out holding the
 * sweep's result.  Synchronises the stream.  shape and best_ms may be NULL. */
int pentago_autotune_section(pentago_section s, const pentago_superinfo *const child[4],
                             pentago_superinfo *out, void *hip_stream, pentago_tile_shape *shape,
                             float *best_ms);

/* pentago_solve_section with an explicit tile shape (for tuning and tests).
 * ERANGE when the shape is outside the ranges above or its tile needs more
 * than 64 KiB of LDS; otherwise as pentago_solve_section (the result does not
 * depend on the shape). */
int pentago_solve_section_shape(pentago_section s, const pentago_superinfo *const child[4],
                                pentago_superinfo *out, void *hip_stream,
                                const pentago_tile_shape *shape);

/* One section of a batch: its counts, its four child tables as for
 * pentago_solve_section, and its output. */
typedef struct {
    pentago_section section;
    const pentago_superinfo *child[4];
    pentago_superinfo *out;
} pentago_section_job;

/* Many sections of one slice (all the same stone count) in one launch: the
 * tiles of every job form one grid (jobs whose tiles need more than 52 KiB of
 * LDS take a second launch beside it), after one batched prep launch for
 * children along dimensions that are not staged.  Results are bit-identical
 * to calling pentago_solve_section on each job.  Jobs must not write to any
 * table another job of the same call reads.  n <= 65536; ERANGE when a launch
 * would exceed 2^31 - 1 tiles. */
int pentago_solve_sections(const pentago_section_job *jobs, size_t n, void *hip_stream);

/* Autotuner of the batched sweep: times the jobs (as pentago_solve_sections,
 * or pentago_solve_sections_d4 when reps is nonzero) with each tile shape
 * the library supports, 256 or 512 threads per tile times a cap on a tile's
 * LDS bytes of 24, 32, 40 or 52 KiB (a tile above the cap takes fewer
 * lines), three timed launches each after a warm-up, and keeps the fastest
 * shape for every later batch of the same stone count in this process
 * (without tuning: 512 threads, 52 KiB).  The jobs' outputs hold their
 * results afterwards.  cap_bytes, threads and best_ms (each may be NULL)
 * receive the cap, the thread count and their time.  Synchronises
 * hip_stream. */
int pentago_autotune_sections(const pentago_section_job *jobs, size_t n, int reps, void *hip_stream,
                              int *cap_bytes, int *threads, float *best_ms);

/* The same with every job's children held as their representatives under
 * the board symmetries (child[j] as rep[j] of pentago_solve_section_d4): the
 * layer step of a whole-slice sweep that stores only D4-minimal sections
 * (Section IV).  Results are bit-identical to pentago_solve_section_d4 on
 * each job. */
int pentago_solve_sections_d4(const pentago_section_job *jobs, size_t n, void *hip_stream);

/* A sweep plan: the job table of one layer (as for pentago_solve_sections)
 * uploaded once, with the prepared-child buffers it needs, so that the layer
 * can be launched repeatedly, directly or from a captured hipGraph.  The
 * tables the jobs name are borrowed until pentago_plan_destroy.
 * pentago_plan_create synchronises the device while uploading. */
typedef struct pentago_sweep_plan pentago_sweep_plan;
int pentago_plan_create(const pentago_section_job *jobs, size_t n, pentago_sweep_plan **plan);
/* A plan whose jobs' children are representatives (as pentago_solve_sections_d4). */
int pentago_plan_create_d4(const pentago_section_job *jobs, size_t n, pentago_sweep_plan **plan);
/* Enqueue the layer on hip_stream: one batched prep launch (children along
 * dimensions that are not staged) and the sweep launch(es). */
int pentago_plan_launch(pentago_sweep_plan *plan, void *hip_stream);
/* The same work as one hipGraph: captured on the plan's own stream at the
 * first call, replayed on hip_stream at every call.  Launches of one plan
 * must not overlap. */
int pentago_plan_launch_graph(pentago_sweep_plan *plan, void *hip_stream);
/* Work tiles of the layer, workgroups launched (one per tile) and the
 * largest LDS bytes per workgroup. */
int pentago_plan_info(const pentago_sweep_plan *plan, long long *tiles, int *grid, int *lds_bytes);
/* Waits for the plan's work, then releases it. */
int pentago_plan_destroy(pentago_sweep_plan *plan);

/* ---------------------------------------------------------------- checks */

/* Counts over a solved table of n entries (Section VII checks every computed
 * slice by its numbers of won, tied and lost positions): out[0] wins, out[1]
 * ties, out[2] losses, each over every (entry, rotation g) pair, 256 per
 * entry (value = win + notlose - 1), and out[3] the entries whose win set is
 * not inside their not-lose set (no solved table has one).  table: device,
 * n x 64 B; out: 4 uint64 in device memory, written stream-ordered on
 * hip_stream.  EINVAL for a NULL out, or a NULL table with n > 0. */
int pentago_table_counts(const pentago_superinfo *table, uint64_t n, uint64_t *out, void *hip_stream);

/* 0 if every entry of table[0, n) has its win set inside its not-lose set,
 * else EINVAL (pentago_last_error() gives the number of bad entries).
 * Synchronises hip_stream. */
int pentago_validate_table(const pentago_superinfo *table, uint64_t n, void *hip_stream);

/* Debug-validate mode, off by default: while on, pentago_solve_section,
 * pentago_solve_section_d4, pentago_solve_sections(_d4) and
 * pentago_plan_create(_d4) first check every child table they are given as
 * pentago_validate_table does, and fail with EINVAL, launching nothing, if
 * one is not valid.  The checks synchronise the call's stream. */
int pentago_set_validate(int on);

/* ---------------------------------------------------------------- endgame */

/* Exact superinfo of n arbitrary boards, each solved to the full board over
 * all 256 quadrant rotations (the serial endgame solver of Section VIII: the
 * descendants of a board under placements only, rotations folded in by
 * rmax).  The side to move comes from the counts; boards that already show
 * five in a row are valid (those rotations are terminal).
 *   boards  device, n boards
 *   out     device, n x 64 B
 *   status  device int32 or NULL: incremented once per invalid board (a
 *           quadrant code >= 19683, counts that are not a valid position, or
 *           more than 10 empty cells); such a board's output is all zero.
 * Boards may have different numbers of empty cells: the library bins them on
 * the device (most empty cells first) and solves them in one persistent
 * launch per class of empty cells (8-10, 7, up to 6), each fed by a device
 * work queue.  ERANGE for n > 2^30. */
int pentago_eval_batch(const pentago_board *boards, size_t n, pentago_superinfo *out,
                       int32_t *status, void *hip_stream);

/* The endgame autotuner: times pentago_eval_batch on these boards with 256
 * and 512 threads per root for the workgroup-per-root classes (8-10 and 7
 * empty cells) and keeps the fastest pair for later calls (process-wide).
 * Leaves out holding the result; synchronises the stream.  threads (2 ints)
 * and best_ms may be NULL.  Errors as pentago_eval_batch. */
int pentago_autotune_eval(const pentago_board *boards, size_t n, pentago_superinfo *out, void *hip_stream,
                          int threads[2], float *best_ms);

/* The plain form of pentago_eval_batch: one launch per group of boards with
 * the same number of empty cells, one workgroup per board.  Same results.
 * Synchronises the stream once, to read the group sizes. */
int pentago_eval_batch_grouped(const pentago_board *boards, size_t n, pentago_superinfo *out,
                               int32_t *status, void *hip_stream);

/* Prepare the library on the current device: upload its read-only tables
 * (about 0.3 MB, once per device; every other call does this itself on first
 * use) and resolve the address of the fixed scratch array of
 * pentago_eval_batch_noalloc on this device.  Allocates.  Idempotent;
 * callers of the allocation-free call run it once per device beforehand. */
int pentago_init(void);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc):
 * pentago_eval_batch with no allocation of any kind.  Same arguments, same
 * results, same kernels.  Its scratch (binning arrays, queue counters and the
 * DAG layer slots of roots with 9 or 10 empty cells) is one fixed device array
 * of 39,649,792 bytes per device, held until the process ends and shared by
 * every call on that device: it keeps the last call's contents, and calls
 * that overlap on one device (on different streams or threads) race; the
 * caller serialises them.  Roots with 9 or 10 empty cells are solved by at
 * most 64 workgroups at a time.  ERANGE for n > 2^20 (before any device
 * work); EINVAL if pentago_init has not run on the current device. */
int pentago_eval_batch_noalloc(const pentago_board *boards, size_t n, pentago_superinfo *out,
                               int32_t *status, void *hip_stream);

/* Exact superinfo of one deep position, solved to the full board over all
 * 256 quadrant rotations (Section VIII: positions outside the database are
 * solved from scratch; the paper's serial solver evaluates an 18-stone
 * position in 16 s on one CPU thread).  The root's DAG (every way to fill its
 * e empty cells in alternating colours; 86,574,831 nodes for e = 18) is
 * solved layer by layer across the whole GPU, two layers at a time in HBM.
 *   out   device, 64 B.
 * Device scratch (two layers of 64 B records, 2 x max_t C(e,t) C(t,ceil(t/2))
 * x 64 B, plus the five-set table: 2.2 GB for e = 18, 17.0 GB for e = 20) is
 * allocated stream-ordered on hip_stream and released after the call's work.  Stream-ordered and asynchronous.  EINVAL for invalid codes or
 * stone counts; ERANGE for more than 20 empty cells; EDEVICE when the scratch
 * allocation fails. */
int pentago_eval_deep(pentago_board board, pentago_superinfo *out, void *hip_stream);

/* pentago_eval_deep for the rotations g of one parity of g0 + g1 + g2 + g3
 * only (Section VIII: rmax flips that parity, so each layer needs the terms
 * of one parity, alternating layer by layer, and its records shrink from 64
 * to 32 B).  A board's own value sits at g = 0, of parity 0.
 *   parity  0 or 1
 *   out     device, 64 B: win/not-lose bits of parity `parity` equal to
 *           pentago_eval_deep's; the bits of the other parity are zero.
 * Scratch as for pentago_eval_deep at half the layer bytes (32 B records:
 * 1.1 GB for e = 18, 8.5 GB for e = 20).  EINVAL for a parity other than 0 or 1, else the
 * errors of pentago_eval_deep. */
int pentago_eval_deep_parity(pentago_board board, int parity, pentago_superinfo *out, void *hip_stream);

/* ---------------------------------------------------------------- serving */

typedef struct pentago_server pentago_server;

typedef struct {
    uint64_t memory_budget;  /* bytes of device scratch the server may hold for searches */
    uint32_t max_inflight;   /* queries admitted but not yet polled */
    uint32_t max_batch;      /* queries per device batch */
    uint32_t streams;        /* HIP streams the server launches on (1..8) */
} pentago_serve_config;

typedef struct {
    uint64_t queries;        /* answered so far */
    uint64_t lookups;        /* answered from a resident section */
    uint64_t searches;       /* answered by on-device search */
    uint64_t batches;        /* device batches launched */
    double p50_us, p99_us;   /* latency from submit to result visible on the host */
    double queries_per_s;    /* answered queries over the time since the first submit */
    double lookup_p50_us, lookup_p99_us;  /* the same, lookups only (0 if none) */
    double search_p50_us, search_p99_us;  /* the same, searches only (0 if none) */
} pentago_serve_stats;

/* Create a server on the current device.  A background thread batches
 * submitted queries by kind and empties count and admits them while
 * in-flight slots and scratch memory allow (continuous batching). */
int pentago_serve_create(const pentago_serve_config *cfg, pentago_server **out);

/* Register a resident solved section (device table, borrowed until destroy).
 * Queries whose quadrant counts match a resident section, or the image of a
 * resident section under one of the 8 board symmetries (pentago_section_image;
 * Section IV stores one section per D4 class), are answered by lookup
 * (Section VIII: positions inside the database are read, not solved): the
 * query is mapped to its preimage in the resident section, whose entry is
 * read, turned back and transformed by the symmetry.  A section registered
 * itself always takes precedence over an image of another.  EINVAL while
 * queries are in flight: register sections first; ERANGE beyond 2^24
 * sections. */
int pentago_serve_add_section(pentago_server *srv, pentago_section s,
                              const pentago_superinfo *table);

/* Submit one board.  EAGAIN when max_inflight queries are pending; EINVAL
 * for an invalid board; ERANGE for more than 20 empty cells on a board that
 * no resident section holds.  Searches with up to 10 empty cells run in
 * batches on the batched endgame solver; with 11 to 20, one per batch on the
 * deep solver (pentago_eval_deep), on every search stream at once, each
 * one's scratch counted against the memory budget like a batch's.  A batch is admitted when a stream is idle and
 * its device scratch fits memory_budget next to the batches running (a
 * batch is always admitted when nothing runs, so no query waits forever).
 * Lookups are admitted before searches; with two or more streams the first
 * stream runs lookups only, so lookups never queue behind search batches;
 * among searches the class (empties group) with the oldest query goes first,
 * with at most one batch in flight per class (a class's queue grows while
 * its batch runs, so batch sizes follow the load). */
int pentago_serve_submit(pentago_server *srv, pentago_board board, uint64_t *ticket);

/* Fetch the result of a ticket into host memory.  EAGAIN while pending;
 * EINVAL for an unknown (or already fetched) ticket. */
int pentago_serve_poll(pentago_server *srv, uint64_t ticket, pentago_superinfo *out);

int pentago_serve_stats_get(pentago_server *srv, pentago_serve_stats *stats);

/* Clear the latency samples and counters (e.g. after a warm-up). */
int pentago_serve_reset_stats(pentago_server *srv);

/* Open-loop replay: submits boards[i] at arrival_s[i] seconds after the call
 * starts (busy-waiting for each arrival, retrying while the server answers
 * EAGAIN) and collects every result into results[i] (host) from a second
 * thread.  Returns when all results are in. */
int pentago_serve_replay(pentago_server *srv, const pentago_board *boards, const double *arrival_s,
                         size_t n, pentago_superinfo *results);

/* Stop the server thread, wait for the device, release everything. */
int pentago_serve_destroy(pentago_server *srv);

/* ---------------------------------------------------------------- misc */

const char *pentago_strerror(int code);
const char *pentago_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
