// api.hip -- the C ABI of include/pentago.h: argument checks, per-device
// tables, job construction and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pentago.h"
#include "internal.h"
#include "kernels.h"

namespace pg {

static thread_local std::string t_last_error;

int fail(int code, const std::string &msg)
{
    t_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *where)
{
    t_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return PENTAGO_EDEVICE;
}

// ---------------------------------------------------------------------------
// Per-device tables
// ---------------------------------------------------------------------------

static std::mutex g_dev_mutex;
static std::map<int, DevTables> g_dev_tables;

int device_tables(DevTables *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    auto it = g_dev_tables.find(dev);
    if (it != g_dev_tables.end()) {
        *out = it->second;
        return 0;
    }
    const HostTables &H = host_tables();
    DevTables T;
    memset(&T, 0, sizeof(T));
    std::vector<uint32_t> nodes;
    std::vector<uint16_t> ranks, submask, subrank, edges;
    for (int k = 0; k <= 10; k++) {
        const DagLayout &L = dag_layout(k);
        T.dag_node_off[k] = (int)nodes.size();
        T.dag_rank_off[k] = (int)ranks.size();
        T.dag_sub_off[k] = (int)submask.size();
        nodes.insert(nodes.end(), L.node.begin(), L.node.end());
        ranks.insert(ranks.end(), L.rank.begin(), L.rank.end());
        submask.insert(submask.end(), L.sub_mask.begin(), L.sub_mask.end());
        subrank.insert(subrank.end(), L.sub_rank.begin(), L.sub_rank.end());
        edges.insert(edges.end(), L.edge.begin(), L.edge.end());
        for (int t = 0; t < 12; t++) {
            T.dag_layer[k][t] = t <= k + 1 ? L.layer_start[t] : 0;
            T.dag_sub_start[k][t] = t <= k + 1 ? L.sub_start[t] : 0;
        }
        T.dag_max[k] = L.max_layer;
        T.dag_sub_max[k] = L.max_subsets;
    }
    void *p;
    struct Up {
        const void *src;
        size_t bytes;
        void **dst;
    };
    void *canon, *qinfo, *lm, *dn, *dr, *sel, *cref, *uref, *smask, *srank, *symmap, *symcode, *syminv, *dedge, *plm, *psel, *pch;
    Up ups[] = {{H.canon.data(), H.canon.size() * 2, &canon},
                {H.qinfo.data(), H.qinfo.size() * sizeof(QInfo), &qinfo},
                {H.lm.data(), H.lm.size() * sizeof(LineMasks), &lm},
                {nodes.data(), nodes.size() * 4, &dn},
                {ranks.data(), ranks.size() * 2, &dr},
                {H.sel.data(), H.sel.size() * 4, &sel},
                {H.chunk_ref.data(), H.chunk_ref.size() * 2, &cref},
                {H.u_ref.data(), H.u_ref.size() * 4, &uref},
                {submask.data(), submask.size() * 2, &smask},
                {subrank.data(), subrank.size() * 2, &srank},
                {H.symmap.data(), H.symmap.size() * 2, &symmap},
                {H.symcode.data(), H.symcode.size() * 2, &symcode},
                {H.syminv.data(), H.syminv.size() * 2, &syminv},
                {H.pat_lm.data(), H.pat_lm.size() * sizeof(LineMasks), &plm},
                {H.pat_sel.data(), H.pat_sel.size() * 4, &psel},
                {H.pat_child.data(), H.pat_child.size() * sizeof(PosChild), &pch},
                {edges.data(), edges.size() * 2, &dedge}};
    for (Up &u : ups) {
        e = hipMalloc(&p, u.bytes);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(tables)");
        e = hipMemcpy(p, u.src, u.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(tables)");
        *u.dst = p;
    }
    T.canon = (const uint16_t *)canon;
    T.qinfo = (const QInfo *)qinfo;
    T.lm = (const LineMasks *)lm;
    T.dag_node = (const uint32_t *)dn;
    T.dag_rank = (const uint16_t *)dr;
    T.dag_edge = (const uint4 *)dedge;
    T.sel = (const uint4 *)sel;
    T.chunk_ref = (const uint16_t *)cref;
    T.u_ref = (const uint32_t *)uref;
    T.dag_sub_mask = (const uint16_t *)smask;
    T.dag_sub_rank = (const uint16_t *)srank;
    T.symmap = (const uint16_t *)symmap;
    T.symcode = (const uint16_t *)symcode;
    T.syminv = (const uint16_t *)syminv;
    T.pat_lm = (const LineMasks *)plm;
    T.pat_sel = (const uint4 *)psel;
    T.pat_child = (const PosChild *)pch;
    g_dev_tables[dev] = T;
    *out = T;
    return 0;
}

int device_tables_ready(DevTables *out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    auto it = g_dev_tables.find(dev);
    if (it == g_dev_tables.end()) return -1;
    *out = it->second;
    return 0;
}

// ---------------------------------------------------------------------------
// Sections
// ---------------------------------------------------------------------------

bool section_valid(const pentago_section &s)
{
    int sb = 0, sw = 0;
    for (int j = 0; j < 4; j++) {
        if (s.black[j] + s.white[j] > 9) return false;
        sb += s.black[j];
        sw += s.white[j];
    }
    return sb == sw || sb == sw + 1;
}

int section_mover(const pentago_section &s)
{
    int sb = 0, sw = 0;
    for (int j = 0; j < 4; j++) {
        sb += s.black[j];
        sw += s.white[j];
    }
    return sb == sw ? 1 : 2;
}

int section_stones(const pentago_section &s)
{
    int n = 0;
    for (int j = 0; j < 4; j++) n += s.black[j] + s.white[j];
    return n;
}

static uint64_t multinomial9(int b, int w)
{
    static const uint64_t f[10] = {1, 1, 2, 6, 24, 120, 720, 5040, 40320, 362880};
    return f[9] / (f[b] * f[w] * f[9 - b - w]);
}

pentago_section child_of(const pentago_section &s, int j)
{
    pentago_section c = s;
    if (section_mover(s) == 1) c.black[j]++;
    else c.white[j]++;
    return c;
}

uint64_t host_block_offset(const int *m, const int *idx)
{
    int B[4], r[4], s[4];
    for (int j = 0; j < 4; j++) {
        B[j] = idx[j] >> 3;
        r[j] = idx[j] & 7;
        s[j] = std::min(8, m[j] - 8 * B[j]);
    }
    uint64_t off = (uint64_t)(8 * B[0]) * m[1] * m[2] * m[3];
    off += (uint64_t)s[0] * 8 * B[1] * m[2] * m[3];
    off += (uint64_t)s[0] * s[1] * 8 * B[2] * m[3];
    off += (uint64_t)s[0] * s[1] * s[2] * 8 * B[3];
    off += (uint64_t)((r[0] * s[1] + r[1]) * s[2] + r[2]) * s[3] + r[3];
    return off;
}

void section_shape_of(const pentago_section &s, int m[4])
{
    const HostTables &H = host_tables();
    for (int j = 0; j < 4; j++) m[j] = H.class_size[s.black[j]][s.white[j]];
}

// Build the sweep job of one section.  `force_d` >= 0 picks the staged
// dimension; G > 0 the lines per tile, force_threads > 0 the workgroup
// size and force_order >= 0 the tile order (for the tile autotuner).
int make_job(const pentago_section &s, const pentago_superinfo *const child[4],
             pentago_superinfo *out, SweepJob *J, int force_d, int forceG, int force_threads,
             int force_order)
{
    if (!section_valid(s)) return fail(PENTAGO_EINVAL, "invalid section counts");
    if (!out) return fail(PENTAGO_EINVAL, "out is NULL");
    const HostTables &H = host_tables();
    memset(J, 0, sizeof(*J));
    section_shape_of(s, J->m);
    J->mover = section_mover(s);
    const int stones = section_stones(s);
    int best = -1, best_e = -1, best_cm = -1;
    for (int j = 0; j < 4; j++) {
        J->qb[j] = H.class_start[s.black[j]][s.white[j]];
        const int empt = 9 - s.black[j] - s.white[j];
        if (empt == 0) continue;
        J->emask |= 1 << j;
        const pentago_section c = child_of(s, j);
        J->cm[j] = H.class_size[c.black[j]][c.white[j]];
        J->cqb[j] = H.class_start[c.black[j]][c.white[j]];
        const pentago_superinfo *cp = child ? child[j] : nullptr;
        if (!cp) {
            if (stones + 1 == 36) J->odmask |= 1 << j;
            else return fail(PENTAGO_ENOCHILD, "child table of quadrant " + std::to_string(j) + " is NULL");
        }
        J->child[j] = (const uint4 *)cp;
        if (empt > best_e || (empt == best_e && J->cm[j] > best_cm)) {
            best = j;
            best_e = empt;
            best_cm = J->cm[j];
        }
    }
    {
        uint64_t entries = 1;
        for (int j = 0; j < 4; j++) entries *= (uint64_t)J->m[j];
        if (entries >= (1ull << 32)) return fail(PENTAGO_ERANGE, "sections of 2^32 entries or more are not supported");
        // out must not overlap a child table the sweep reads
        const uintptr_t o0 = (uintptr_t)out, o1 = o0 + 64 * entries;
        for (int j = 0; j < 4; j++) {
            if (!J->child[j]) continue;
            const uint64_t centries = entries / (uint64_t)J->m[j] * (uint64_t)J->cm[j];
            const uintptr_t c0 = (uintptr_t)J->child[j], c1 = c0 + 64 * centries;
            if (o0 < c1 && c0 < o1)
                return fail(PENTAGO_EINVAL, "out overlaps the child table of quadrant " + std::to_string(j));
        }
    }
    if (force_d >= 0 && ((J->emask >> force_d) & 1)) best = force_d;
    J->d = best >= 0 ? best : 3;
    J->e = J->d == 3 ? 2 : 3;
    // every pattern of a (black, white) class has the same empty cells count
    J->nchd = (J->emask >> J->d) & 1 ? 9 - s.black[J->d] - s.white[J->d] : 0;
    int o[2], n = 0;
    for (int j = 0; j < 4; j++)
        if (j != J->d && j != J->e) o[n++] = j;
    J->o1 = o[0];
    J->o2 = o[1];
    const int cmd = (J->emask >> J->d) & 1 ? J->cm[J->d] : 0;
    // lines per tile: at most 8 (one 8^4 block row), the child items of a
    // tile in one pass of its 256 threads when the child line allows, and the
    // tile's LDS within 64 KiB
    int G = 8;
    const TileShape tuned = tuned_tile_shape(*J);
    J->threads = force_threads > 0 ? force_threads : tuned.lines > 0 ? tuned.threads : 256;
    J->order = force_order >= 0 ? force_order : tuned.lines > 0 ? tuned.order : 0;
    if (forceG > 0) G = forceG;
    else if (tuned.lines > 0) G = tuned.lines;
    else {
        // (the kernels give every line 8 slots per position when D == 3,
        // so a smaller G only helps the child pass for D == 3)
        while (G > 1 && sweep_lds_bytes(G, J->m[J->d], cmd) > 65536) G--;
    }
    J->G = G;
    J->ngroups = (J->m[J->e] + G - 1) / G;
    J->ntiles = (long long)J->m[J->o1] * J->m[J->o2] * J->ngroups;
    J->lds_bytes = sweep_lds_bytes(G, J->m[J->d], cmd);
    J->out = (uint4 *)out;
    return 0;
}

size_t prep_bytes(const SweepJob &J, int j)
{
    size_t n = (size_t)J.cm[j];
    for (int i = 0; i < 4; i++)
        if (i != j) n *= (size_t)J.m[i];
    return 64 * n;
}

}  // namespace pg

using namespace pg;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

int pentago_section_shape(pentago_section s, uint32_t shape[4], uint64_t *entries,
                          uint64_t *positions)
{
    if (!section_valid(s)) return fail(PENTAGO_EINVAL, "invalid section counts");
    int m[4];
    section_shape_of(s, m);
    uint64_t e = 1, p = 1;
    for (int j = 0; j < 4; j++) {
        if (shape) shape[j] = (uint32_t)m[j];
        e *= (uint64_t)m[j];
        p *= multinomial9(s.black[j], s.white[j]);
    }
    if (entries) *entries = e;
    if (positions) *positions = p;
    return 0;
}

int pentago_section_offset(pentago_section s, const uint32_t idx[4], uint64_t *offset)
{
    if (!section_valid(s) || !idx || !offset) return fail(PENTAGO_EINVAL, "invalid arguments");
    int m[4], i[4];
    section_shape_of(s, m);
    for (int j = 0; j < 4; j++) {
        if (idx[j] >= (uint32_t)m[j]) return fail(PENTAGO_EINVAL, "index out of range");
        i[j] = (int)idx[j];
    }
    *offset = host_block_offset(m, i);
    return 0;
}

int pentago_section_board(pentago_section s, const uint32_t idx[4], pentago_board *board)
{
    if (!section_valid(s) || !idx || !board) return fail(PENTAGO_EINVAL, "invalid arguments");
    const HostTables &H = host_tables();
    for (int j = 0; j < 4; j++) {
        const int b = s.black[j], w = s.white[j];
        if (idx[j] >= (uint32_t)H.class_size[b][w]) return fail(PENTAGO_EINVAL, "index out of range");
        board->q[j] = H.qinfo[H.class_start[b][w] + idx[j]].code;
    }
    return 0;
}

int pentago_child_section(pentago_section s, int j, pentago_section *child)
{
    if (!section_valid(s) || j < 0 || j > 3 || !child) return fail(PENTAGO_EINVAL, "invalid arguments");
    if (s.black[j] + s.white[j] == 9) return fail(PENTAGO_EINVAL, "quadrant is full");
    *child = child_of(s, j);
    return 0;
}

int pentago_solve_section(pentago_section s, const pentago_superinfo *const child[4],
                          pentago_superinfo *out, void *hip_stream)
{
    DevTables T;
    int rc = device_tables(&T);
    if (rc) return rc;
    SweepJob J;
    rc = make_job(s, child, out, &J, -1, 0);
    if (rc) return rc;
    rc = validate_children(J, (hipStream_t)hip_stream);
    if (rc) return rc;
    return run_job(J, T, (hipStream_t)hip_stream);
}

const char *pentago_strerror(int code)
{
    switch (code) {
    case PENTAGO_OK: return "ok";
    case PENTAGO_EINVAL: return "invalid argument";
    case PENTAGO_ENOCHILD: return "missing child section table";
    case PENTAGO_ENOMEM: return "out of memory";
    case PENTAGO_ERANGE: return "size out of supported range";
    case PENTAGO_EAGAIN: return "try again";
    case PENTAGO_EDEVICE: return "HIP runtime error";
    default: return "unknown error";
    }
}

const char *pentago_last_error(void) { return t_last_error.c_str(); }

}  // extern "C"
