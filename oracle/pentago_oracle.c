/*
 * pentago_oracle.c -- plain, slow, obviously-correct CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The product path (the
 * HIP library) never calls, links or includes anything here, and this file
 * includes nothing from it.
 *
 * Everything follows Irving, "Pentago is a First Player Win" (arXiv:1404.0743):
 *   - the rules (Section I): 6x6 board, four 3x3 quadrants, place a stone then
 *     turn one quadrant by 90 degrees either way; five in a row wins; a five
 *     made by the placement wins at once; simultaneous fives or a full board
 *     without a five tie;
 *   - the value recurrence v_c / h_c and the validity predicate (Section II);
 *   - the rotation-abstracted table over L = Z4^4 with one win bit and one
 *     not-lose bit per element (Section III);
 *   - sections, rotation-minimal quadrant orderings and 8^4 blocks (Section IV,
 *     Fig. 4).
 * Boards are concrete 36-cell arrays; five-in-a-row is checked by scanning the
 * 32 explicit lines; every table bit is computed on its own rotated board.  No
 * bit tricks, no blocking beyond the layout definition, no reuse of results
 * across rotations except the memo table of the minimax search.
 *
 * Conventions (a reading; the paper leaves them open):
 *   cell      = 6*r + c, r counted downward, c rightward
 *   quadrant  = 2*(r/3) + c/3  (0 top-left, 1 top-right, 2 bottom-left, 3 bottom-right)
 *   local     = 3*(r%3) + c%3, ternary code = sum digit*3^local,
 *               digit 0 empty, 1 black, 2 white
 *   one turn  = 90 degrees counter-clockwise: local (lr,lc) moves to (2-lc, lr)
 *   g in L    = g0 + 4*g1 + 16*g2 + 64*g3, g_j = counter-clockwise turns of quadrant j
 *   table     = uint64[8] per entry: win words 0..3 then not-lose words 0..3,
 *               bit g lives in word g>>6 at position g&63
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define EMPTY 0
#define BLACK 1
#define WHITE 2

/* ------------------------------------------------------------------------ */
/* Rules primitives (Section I, Section II)                                   */
/* ------------------------------------------------------------------------ */

static int LINES[32][5];
static int NLINES = 0;

/* The 32 five-cell lines of a 6x6 board: 12 horizontal, 12 vertical and
   8 diagonal windows of length five (Section I: horizontal, vertical or
   diagonal). */
static void build_lines(void)
{
    int n = 0;
    for (int r = 0; r < 6; r++)
        for (int c0 = 0; c0 < 2; c0++, n++)
            for (int i = 0; i < 5; i++) LINES[n][i] = 6 * r + (c0 + i);
    for (int c = 0; c < 6; c++)
        for (int r0 = 0; r0 < 2; r0++, n++)
            for (int i = 0; i < 5; i++) LINES[n][i] = 6 * (r0 + i) + c;
    for (int r0 = 0; r0 < 2; r0++)
        for (int c0 = 0; c0 < 2; c0++, n++)
            for (int i = 0; i < 5; i++) LINES[n][i] = 6 * (r0 + i) + (c0 + i);
    for (int r0 = 0; r0 < 2; r0++)
        for (int c0 = 4; c0 < 6; c0++, n++)
            for (int i = 0; i < 5; i++) LINES[n][i] = 6 * (r0 + i) + (c0 - i);
    NLINES = n;
}

/* f_x(s) of Section II: 1 iff colour x has five in a row. */
int po_five(const uint8_t *b, int x)
{
    for (int l = 0; l < NLINES; l++) {
        int all = 1;
        for (int i = 0; i < 5; i++)
            if (b[LINES[l][i]] != x) { all = 0; break; }
        if (all) return 1;
    }
    return 0;
}

int po_lines(int *out)
{
    memcpy(out, LINES, sizeof(LINES));
    return NLINES;
}

static int cell_of(int quadrant, int local)
{
    int r = 3 * (quadrant / 2) + local / 3;
    int c = 3 * (quadrant % 2) + local % 3;
    return 6 * r + c;
}

/* Turn quadrant q counter-clockwise `turns` times (turns taken mod 4). */
void po_turn(uint8_t *b, int q, int turns)
{
    turns &= 3;
    for (int t = 0; t < turns; t++) {
        uint8_t old[9];
        for (int l = 0; l < 9; l++) old[l] = b[cell_of(q, l)];
        for (int lr = 0; lr < 3; lr++)
            for (int lc = 0; lc < 3; lc++) {
                int nr = 2 - lc, nc = lr;
                b[cell_of(q, 3 * nr + nc)] = old[3 * lr + lc];
            }
    }
}

/* g . s for g in L (Section III). */
void po_apply(const uint8_t *in, int g, uint8_t *out)
{
    memcpy(out, in, 36);
    for (int q = 0; q < 4; q++) po_turn(out, q, (g >> (2 * q)) & 3);
}

static void count_stones(const uint8_t *b, int *nb, int *nw)
{
    *nb = *nw = 0;
    for (int i = 0; i < 36; i++) {
        if (b[i] == BLACK) (*nb)++;
        else if (b[i] == WHITE) (*nw)++;
    }
}

/* Validity (Section II): black moves first, so black and white counts are
   equal on black's turn and black has one more on white's turn.  Returns the
   side to move, or 0 for an invalid board. */
int po_mover(const uint8_t *b)
{
    int nb, nw;
    count_stones(b, &nb, &nw);
    if (nb == nw) return BLACK;
    if (nb == nw + 1) return WHITE;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O2: minimax over the rules (Section II recurrence), memoised per search    */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t *key;
    int8_t *val;
    size_t mask, n;
} memo_t;

static void memo_init(memo_t *m, size_t cap)
{
    m->key = (uint64_t *)calloc(cap, sizeof(uint64_t));
    m->val = (int8_t *)calloc(cap, 1);
    m->mask = cap - 1;
    m->n = 0;
}

static void memo_free(memo_t *m)
{
    free(m->key);
    free(m->val);
}

static size_t memo_slot(const memo_t *m, uint64_t k)
{
    uint64_t h = k * 0x9E3779B97F4A7C15ull;
    return (size_t)(h >> 17) & m->mask;
}

static int memo_get(const memo_t *m, uint64_t k, int8_t *v)
{
    for (size_t i = memo_slot(m, k);; i = (i + 1) & m->mask) {
        if (m->key[i] == 0) return 0;
        if (m->key[i] == k) { *v = m->val[i]; return 1; }
    }
}

static void memo_put(memo_t *m, uint64_t k, int8_t v);

static void memo_grow(memo_t *m)
{
    memo_t big;
    memo_init(&big, 2 * (m->mask + 1));
    for (size_t i = 0; i <= m->mask; i++)
        if (m->key[i]) memo_put(&big, m->key[i], m->val[i]);
    memo_free(m);
    *m = big;
}

static void memo_put(memo_t *m, uint64_t k, int8_t v)
{
    if (2 * (m->n + 1) > m->mask + 1) memo_grow(m);
    for (size_t i = memo_slot(m, k);; i = (i + 1) & m->mask) {
        if (m->key[i] == 0) { m->key[i] = k; m->val[i] = v; m->n++; return; }
        if (m->key[i] == k) { m->val[i] = v; return; }
    }
}

static uint64_t board_key(const uint8_t *b)
{
    uint64_t k = 0;
    for (int i = 35; i >= 0; i--) k = 3 * k + b[i];
    return k + 1; /* 0 marks an empty slot */
}

/* v_c(s) of Section II with c the side to move.  Terminal: a five of either
   colour or a full board, value f_c - f_cbar.  Otherwise the maximum over
   placements a of: 1 if the placement makes a c-five, else the maximum over
   the eight single-quadrant turns b of -v_cbar(b).  (h_c(b) = -v_cbar(b)
   covers the both-fives case, since a board with both fives is terminal with
   value 0.) */
static int value_rec(memo_t *m, const uint8_t *b)
{
    int nb, nw;
    count_stones(b, &nb, &nw);
    int c = (nb == nw) ? BLACK : WHITE;
    int cb = 3 - c;
    int fc = po_five(b, c), fo = po_five(b, cb);
    if (fc || fo || nb + nw == 36) return fc - fo;
    uint64_t key = board_key(b);
    int8_t memo;
    if (memo_get(m, key, &memo)) return memo;
    int best = -1;
    for (int p = 0; p < 36 && best < 1; p++) {
        if (b[p] != EMPTY) continue;
        uint8_t a[36];
        memcpy(a, b, 36);
        a[p] = (uint8_t)c;
        if (po_five(a, c)) { best = 1; break; }
        for (int q = 0; q < 4 && best < 1; q++)
            for (int dir = 1; dir <= 3 && best < 1; dir += 2) { /* +90 and -90 */
                uint8_t u[36];
                memcpy(u, a, 36);
                po_turn(u, q, dir);
                int v = -value_rec(m, u);
                if (v > best) best = v;
            }
    }
    memo_put(m, key, (int8_t)best);
    return best;
}

int po_value(const uint8_t *b)
{
    if (!po_mover(b)) return -2;
    memo_t m;
    memo_init(&m, 1 << 12);
    int v = value_rec(&m, b);
    memo_free(&m);
    return v;
}

static void set_bits(uint64_t *t, int g, int v)
{
    uint64_t bit = 1ull << (g & 63);
    if (v == 1) t[g >> 6] |= bit;       /* win */
    if (v >= 0) t[4 + (g >> 6)] |= bit; /* not lose */
}

/* The rotation-abstracted table of one board: for every g in L, the value of
   g.s (Section III), one bit for win and one for not-lose. */
static void minimax_table(const uint8_t *s, uint64_t *out)
{
    memo_t m;
    memo_init(&m, 1 << 14);
    memset(out, 0, 8 * sizeof(uint64_t));
    for (int g = 0; g < 256; g++) {
        uint8_t gs[36];
        po_apply(s, g, gs);
        set_bits(out, g, value_rec(&m, gs));
    }
    memo_free(&m);
}

/* ------------------------------------------------------------------------ */
/* Simple thread pool over independent items                                  */
/* ------------------------------------------------------------------------ */

typedef void (*item_fn)(void *ctx, long i);
typedef struct {
    item_fn fn;
    void *ctx;
    long n;
    long next;
} pool_t;

static void *pool_worker(void *arg)
{
    pool_t *p = (pool_t *)arg;
    for (;;) {
        long i = __sync_fetch_and_add(&p->next, 1);
        if (i >= p->n) break;
        p->fn(p->ctx, i);
    }
    return NULL;
}

static void run_pool(item_fn fn, void *ctx, long n, int nthreads)
{
    pool_t p = {fn, ctx, n, 0};
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, pool_worker, &p);
    pool_worker(&p);
    for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
}

typedef struct {
    const uint8_t *boards;
    uint64_t *out;
} mm_ctx;

static void mm_item(void *vctx, long i)
{
    mm_ctx *c = (mm_ctx *)vctx;
    minimax_table(c->boards + 36 * i, c->out + 8 * i);
}

/* Tables of n boards by minimax; returns -1 if any board is invalid. */
int po_minimax_tables(const uint8_t *boards, long n, uint64_t *out, int nthreads)
{
    for (long i = 0; i < n; i++)
        if (!po_mover(boards + 36 * i)) return -1;
    mm_ctx c = {boards, out};
    run_pool(mm_item, &c, n, nthreads);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Quadrant orbits and sections (Section IV, Fig. 4)                          */
/* ------------------------------------------------------------------------ */

#define NCODES 19683
static int CODE_TURN[NCODES];      /* code after one counter-clockwise turn */
static int CODE_MIN[NCODES];       /* least code over the four turns */
static int CODE_K[NCODES];         /* least k with turn^k(code) == CODE_MIN */
static int CODE_INDEX[NCODES];     /* index of a minimal code within its class */
static int CLASS_START[10][10];
static int CLASS_SIZE[10][10];
static int CLASS_CODES[NCODES];
static int POW3[10];

static int digit(int code, int l) { return (code / POW3[l]) % 3; }

static void build_quadrants(void)
{
    POW3[0] = 1;
    for (int i = 1; i < 10; i++) POW3[i] = 3 * POW3[i - 1];
    for (int code = 0; code < NCODES; code++) {
        int t = 0;
        for (int lr = 0; lr < 3; lr++)
            for (int lc = 0; lc < 3; lc++)
                t += digit(code, 3 * lr + lc) * POW3[3 * (2 - lc) + lr];
        CODE_TURN[code] = t;
    }
    for (int code = 0; code < NCODES; code++) {
        int best = code, bestk = 0, cur = code;
        for (int k = 1; k < 4; k++) {
            cur = CODE_TURN[cur];
            if (cur < best) { best = cur; bestk = k; }
        }
        CODE_MIN[code] = best;
        CODE_K[code] = bestk;
    }
    memset(CLASS_SIZE, 0, sizeof(CLASS_SIZE));
    int n = 0;
    for (int b = 0; b <= 9; b++)
        for (int w = 0; b + w <= 9; w++) {
            CLASS_START[b][w] = n;
            for (int code = 0; code < NCODES; code++) {
                if (CODE_MIN[code] != code) continue;
                int nb = 0, nw = 0;
                for (int l = 0; l < 9; l++) {
                    int d = digit(code, l);
                    nb += d == 1;
                    nw += d == 2;
                }
                if (nb == b && nw == w) {
                    CODE_INDEX[code] = n - CLASS_START[b][w];
                    CLASS_CODES[n++] = code;
                }
            }
            CLASS_SIZE[b][w] = n - CLASS_START[b][w];
        }
}

int po_class_size(int b, int w)
{
    if (b < 0 || w < 0 || b + w > 9) return 0;
    return CLASS_SIZE[b][w];
}

int po_class_code(int b, int w, int i)
{
    if (i < 0 || i >= po_class_size(b, w)) return -1;
    return CLASS_CODES[CLASS_START[b][w] + i];
}

int po_code_turn(int code, int turns)
{
    for (int t = 0; t < (turns & 3); t++) code = CODE_TURN[code];
    return code;
}

int po_canon(int code, int *k)
{
    if (k) *k = CODE_K[code];
    return CODE_MIN[code];
}

/* counts = {black0..black3, white0..white3} */
static int section_valid(const int *counts)
{
    int sb = 0, sw = 0;
    for (int j = 0; j < 4; j++) {
        if (counts[j] < 0 || counts[4 + j] < 0 || counts[j] + counts[4 + j] > 9) return 0;
        sb += counts[j];
        sw += counts[4 + j];
    }
    return sb == sw || sb == sw + 1;
}

static void section_shape(const int *counts, long *m)
{
    for (int j = 0; j < 4; j++) m[j] = CLASS_SIZE[counts[j]][counts[4 + j]];
}

long po_section_entries(const int *counts)
{
    if (!section_valid(counts)) return -1;
    long m[4];
    section_shape(counts, m);
    return m[0] * m[1] * m[2] * m[3];
}

/* Offset of entry idx in the 8x8x8x8-blocked layout (Section IV: blocks of
   8^4 entries, smaller at the section boundary).  Blocks are in row-major
   order of block coordinates (dimension 3 fastest); inside a block the
   entries are row-major over the block's own extents.  Written out as the
   count of entries that precede idx. */
static long block_extent(long m, long B) { return (m - 8 * B < 8) ? (m - 8 * B) : 8; }

long po_section_offset(const int *counts, const int *idx)
{
    if (!section_valid(counts)) return -1;
    long m[4];
    section_shape(counts, m);
    long B[4], r[4], s[4];
    for (int j = 0; j < 4; j++) {
        if (idx[j] < 0 || idx[j] >= m[j]) return -1;
        B[j] = idx[j] / 8;
        r[j] = idx[j] % 8;
        s[j] = block_extent(m[j], B[j]);
    }
    /* entries in earlier block slabs, slab by slab */
    long off = 0;
    off += 8 * B[0] * m[1] * m[2] * m[3];
    off += s[0] * 8 * B[1] * m[2] * m[3];
    off += s[0] * s[1] * 8 * B[2] * m[3];
    off += s[0] * s[1] * s[2] * 8 * B[3];
    /* position inside the block */
    off += ((r[0] * s[1] + r[1]) * s[2] + r[2]) * s[3] + r[3];
    return off;
}

int po_section_board(const int *counts, const int *idx, uint8_t *board)
{
    if (!section_valid(counts)) return -1;
    memset(board, 0, 36);
    for (int j = 0; j < 4; j++) {
        int code = po_class_code(counts[j], counts[4 + j], idx[j]);
        if (code < 0) return -1;
        for (int l = 0; l < 9; l++) board[cell_of(j, l)] = (uint8_t)digit(code, l);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O4: plain section retrograde (Section II recurrence on concrete boards,    */
/* children looked up in the (n+1)-stone child sections)                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int counts[8];
    int child_counts[4][8];
    const uint64_t *child[4];
    const int *idx;
    uint64_t *out;
    int mover;
    int bad;
} sec_ctx;

static int quadrant_of_cell(int p) { return 2 * ((p / 6) / 3) + (p % 6) / 3; }

/* v of a board u with n+1 stones, read from the child section table: each
   quadrant of u is turned to its rotation-minimal pattern (turns k_j), which
   names the entry; u itself is the entry's board turned by -k_j in each
   quadrant, so its value is the entry's table at g = (-k_0, ..., -k_3). */
static int child_value(sec_ctx *c, int qchild, const uint8_t *u)
{
    int mover = 3 - c->mover;
    if (!c->child[qchild]) { /* on-demand terminal board: 36 stones */
        return po_five(u, mover) - po_five(u, 3 - mover);
    }
    int idx[4], g = 0;
    for (int j = 0; j < 4; j++) {
        int code = 0;
        for (int l = 8; l >= 0; l--) code = 3 * code + u[cell_of(j, l)];
        int k;
        int mn = po_canon(code, &k);
        idx[j] = CODE_INDEX[mn];
        g |= ((4 - k) & 3) << (2 * j);
    }
    long off = po_section_offset(c->child_counts[qchild], idx);
    const uint64_t *t = c->child[qchild] + 8 * off;
    int w = (int)((t[g >> 6] >> (g & 63)) & 1);
    int nl = (int)((t[4 + (g >> 6)] >> (g & 63)) & 1);
    return w ? 1 : (nl ? 0 : -1);
}

static void sec_item(void *vctx, long i)
{
    sec_ctx *c = (sec_ctx *)vctx;
    uint8_t s[36];
    po_section_board(c->counts, c->idx + 4 * i, s);
    uint64_t *out = c->out + 8 * i;
    memset(out, 0, 8 * sizeof(uint64_t));
    int x = c->mover, xb = 3 - x;
    for (int g = 0; g < 256; g++) {
        uint8_t gs[36];
        po_apply(s, g, gs);
        int fc = po_five(gs, x), fo = po_five(gs, xb);
        int nb, nw;
        count_stones(gs, &nb, &nw);
        int v;
        if (fc || fo || nb + nw == 36) {
            v = fc - fo;
        } else {
            int best = -1;
            for (int p = 0; p < 36 && best < 1; p++) {
                if (gs[p] != EMPTY) continue;
                uint8_t t[36];
                memcpy(t, gs, 36);
                t[p] = (uint8_t)x;
                if (po_five(t, x)) { best = 1; break; }
                int qc = quadrant_of_cell(p);
                for (int q = 0; q < 4 && best < 1; q++)
                    for (int dir = 1; dir <= 3 && best < 1; dir += 2) {
                        uint8_t u[36];
                        memcpy(u, t, 36);
                        po_turn(u, q, dir);
                        int cv = -child_value(c, qc, u);
                        if (cv > best) best = cv;
                    }
            }
            v = best;
        }
        set_bits(out, g, v);
    }
}

/* Solve listed entries (idx: n x 4) of a section.  child[j] is the table of
   the section with the mover's count in quadrant j raised by one, or NULL
   when quadrant j is full (unused) or when that child is the 36-stone slice
   (computed on demand).  Returns 0, or -1 for an invalid section, -2 for a
   missing child, -3 for an index out of range. */
int po_section_solve(const int *counts, const uint64_t *const *child, const int *idx,
                     long n, uint64_t *out, int nthreads)
{
    if (!section_valid(counts)) return -1;
    sec_ctx c;
    memcpy(c.counts, counts, sizeof(c.counts));
    int sb = 0, sw = 0;
    for (int j = 0; j < 4; j++) { sb += counts[j]; sw += counts[4 + j]; }
    c.mover = (sb == sw) ? BLACK : WHITE;
    long m[4];
    section_shape(counts, m);
    for (int j = 0; j < 4; j++) {
        memcpy(c.child_counts[j], counts, sizeof(c.counts));
        c.child_counts[j][(c.mover == BLACK ? 0 : 4) + j] += 1;
        c.child[j] = child ? child[j] : NULL;
        int full = counts[j] + counts[4 + j] == 9;
        if (!full && !c.child[j] && sb + sw + 1 != 36) return -2;
    }
    for (long i = 0; i < n; i++)
        for (int j = 0; j < 4; j++)
            if (idx[4 * i + j] < 0 || idx[4 * i + j] >= m[j]) return -3;
    c.idx = idx;
    c.out = out;
    c.bad = 0;
    run_pool(sec_item, &c, n, nthreads);
    return 0;
}

/* Every entry index of a section, in blocked-layout order (n x 4). */
long po_section_all_indices(const int *counts, int *idx)
{
    long n = po_section_entries(counts);
    if (n < 0) return -1;
    long m[4];
    section_shape(counts, m);
    int t[4];
    for (t[0] = 0; t[0] < m[0]; t[0]++)
        for (t[1] = 0; t[1] < m[1]; t[1]++)
            for (t[2] = 0; t[2] < m[2]; t[2]++)
                for (t[3] = 0; t[3] < m[3]; t[3]++) {
                    long off = po_section_offset(counts, t);
                    memcpy(idx + 4 * off, t, sizeof(t));
                }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Board symmetries and section tables (Section III: the group G = L x| D4;  */
/* Section IV: only D4-minimal sections are computed)                         */
/* ------------------------------------------------------------------------ */

/* The 8 board symmetries, numbered sym = r + 4*f: mirror left-right when f
   is set ((row, col) -> (row, 5 - col)), then r quarter turns of the whole
   board counter-clockwise ((row, col) -> (5 - col, row)).  Writes the cell
   map: the stone on cell c moves to cell perm[c]. */
int po_sym_cells(int sym, int *perm)
{
    if (sym < 0 || sym > 7) return -1;
    for (int c = 0; c < 36; c++) {
        int r = c / 6, col = c % 6;
        if (sym & 4) col = 5 - col;
        for (int t = 0; t < (sym & 3); t++) {
            int nr = 5 - col, nc = r;
            r = nr;
            col = nc;
        }
        perm[c] = 6 * r + col;
    }
    return 0;
}

/* Quadrant position map of a symmetry: quadrant q moves to qmap[q] (read off
   where the centre cell of q goes). */
int po_sym_quadrants(int sym, int *qmap)
{
    int perm[36];
    if (po_sym_cells(sym, perm)) return -1;
    for (int q = 0; q < 4; q++) qmap[q] = quadrant_of_cell(perm[cell_of(q, 4)]);
    return 0;
}

/* Counts of the image section sym(s): the counts of quadrant q move to
   quadrant qmap[q]. */
int po_sym_counts(const int *counts, int sym, int *out)
{
    int qmap[4];
    if (!section_valid(counts) || po_sym_quadrants(sym, qmap)) return -1;
    for (int q = 0; q < 4; q++) {
        out[qmap[q]] = counts[q];
        out[4 + qmap[q]] = counts[4 + q];
    }
    return 0;
}

typedef struct {
    int src_counts[8], dst_counts[8];
    int perm[36];
    const uint64_t *src;
    const int *idx;
    uint64_t *out;
} sym_ctx;

/* One entry of the image table, bit by bit.  The values of a position and of
   its image under a board symmetry are equal (the rules do not distinguish
   them), so bit G of the image entry is the value of the board G.b', where b'
   is the image entry's board, and that board's preimage under the symmetry
   is a concrete board of the source section: canonicalise its quadrants and
   read the source table as child_value does. */
static void sym_item(void *vctx, long i)
{
    sym_ctx *c = (sym_ctx *)vctx;
    uint8_t dst[36];
    po_section_board(c->dst_counts, c->idx + 4 * i, dst);
    uint64_t *out = c->out + 8 * i;
    memset(out, 0, 8 * sizeof(uint64_t));
    for (int G = 0; G < 256; G++) {
        uint8_t gd[36], pre[36];
        po_apply(dst, G, gd);
        for (int cell = 0; cell < 36; cell++) pre[cell] = gd[c->perm[cell]];
        int idx[4], g = 0;
        for (int j = 0; j < 4; j++) {
            int code = 0;
            for (int l = 8; l >= 0; l--) code = 3 * code + pre[cell_of(j, l)];
            int k;
            int mn = po_canon(code, &k);
            idx[j] = CODE_INDEX[mn];
            g |= ((4 - k) & 3) << (2 * j);
        }
        const uint64_t *t = c->src + 8 * po_section_offset(c->src_counts, idx);
        int w = (int)((t[g >> 6] >> (g & 63)) & 1);
        int nl = (int)((t[4 + (g >> 6)] >> (g & 63)) & 1);
        set_bits(out, G, w ? 1 : (nl ? 0 : -1));
    }
}

/* Entries idx (n x 4, indices of the image section sym(s)) of the table of
   sym(s), from the whole table src of section s (blocked order).  Returns 0,
   or -1 for an invalid section or symmetry, -3 for an index out of range. */
int po_section_transform(const int *counts, const uint64_t *src, int sym, const int *idx, long n,
                         uint64_t *out, int nthreads)
{
    sym_ctx c;
    memcpy(c.src_counts, counts, sizeof(c.src_counts));
    if (po_sym_counts(counts, sym, c.dst_counts) || po_sym_cells(sym, c.perm)) return -1;
    long m[4];
    section_shape(c.dst_counts, m);
    for (long i = 0; i < n; i++)
        for (int j = 0; j < 4; j++)
            if (idx[4 * i + j] < 0 || idx[4 * i + j] >= m[j]) return -3;
    c.src = src;
    c.idx = idx;
    c.out = out;
    run_pool(sym_item, &c, n, nthreads);
    return 0;
}

int po_init(void)
{
    if (NLINES) return 0;
    build_lines();
    build_quadrants();
    return 0;
}
