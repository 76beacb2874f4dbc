// serve.hip -- the query server (Section VIII: positions in the database are
// looked up, others solved on the fly): a background thread batches pending
// queries by kind (lookup, or search by number of empty cells), admits a batch
// when a stream is idle and its device scratch fits the memory budget, and
// publishes results as batches complete.  New queries keep being admitted
// while earlier batches run on other streams (continuous batching).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "internal.h"

using namespace pg;

namespace {

using Clock = std::chrono::steady_clock;
using SecKey = std::tuple<uint8_t, uint8_t, uint8_t, uint8_t, uint8_t, uint8_t, uint8_t, uint8_t>;

SecKey key_of(const pentago_section &s)
{
    return SecKey(s.black[0], s.black[1], s.black[2], s.black[3], s.white[0], s.white[1],
                  s.white[2], s.white[3]);
}

struct Query {
    uint64_t ticket;
    uint64_t board;
    Clock::time_point t_submit;
    int cls;   // 0 lookup, 1 search <= 6 empties, 2: 7, 3: 8, 4: 9..10
    int sec;   // resident section index (lookups)
};

struct Batch {
    int stream = -1;
    int cls = 0;
    std::vector<Query> qs;
    size_t scratch = 0;
    hipEvent_t done = nullptr;
};

constexpr int kClasses = 6;

// search classes by empty cells: 1 (<= 6), 2 (7), 3 (8), 4 (9-10) in batches
// on the batched endgame solver, 5 (11-20) one at a time on the deep solver
int class_of_empties(int e) { return e <= 6 ? 1 : e == 7 ? 2 : e == 8 ? 3 : e <= 10 ? 4 : 5; }

}  // namespace

struct pentago_server {
    pentago_serve_config cfg;
    int device = 0, grid = 0;
    DevTables T;
    // resident sections: section counts -> index into secs | symmetry << 24,
    // for every registered section and each of its images under the board
    // symmetries (a registered section itself always maps with symmetry 0)
    std::map<SecKey, int> resident;
    std::vector<ResidentSection> secs;
    ResidentSection *d_secs = nullptr;
    size_t d_secs_cap = 0;
    // per-stream buffers
    std::vector<hipStream_t> streams;
    std::vector<uint64_t *> h_boards, d_boards;
    std::vector<int *> h_sec, d_sec;
    std::vector<uint4 *> h_out, d_out;
    std::vector<Batch> running;   // running[i].stream == i when busy
    std::vector<bool> busy;
    size_t scratch_in_use = 0;
    // queues
    std::mutex mu;
    std::deque<Query> pending[kClasses];
    std::atomic<size_t> npending{0};  // total over the classes (read without the lock)
    int class_running[kClasses] = {};  // batches in flight per search class
    std::unordered_map<uint64_t, pentago_superinfo> results;
    std::unordered_map<uint64_t, int> live;  // ticket -> 0 pending, 1 done
    uint64_t next_ticket = 1;
    size_t inflight = 0;
    std::thread worker;
    std::atomic<bool> stop{false};
    std::condition_variable cv;
    std::condition_variable done_cv;  // notified when a batch's results are published
    int worker_error = 0;
    // statistics
    std::vector<double> lat_us, lat_lookup_us, lat_search_us;
    uint64_t nqueries = 0, nlookups = 0, nsearches = 0, nbatches = 0;
    Clock::time_point t_first;
    Clock::time_point t_last;
    bool any = false;
};

namespace {

void publish(pentago_server *S, Batch &B)
{
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> lock(S->mu);
    const uint4 *h = S->h_out[B.stream];
    for (size_t i = 0; i < B.qs.size(); i++) {
        pentago_superinfo r;
        memcpy(&r, h + 4 * i, sizeof(r));
        S->results[B.qs[i].ticket] = r;
        S->live[B.qs[i].ticket] = 1;
        const double us = std::chrono::duration<double, std::micro>(now - B.qs[i].t_submit).count();
        S->lat_us.push_back(us);
        (B.cls == 0 ? S->lat_lookup_us : S->lat_search_us).push_back(us);
        S->nqueries++;
        (B.cls == 0 ? S->nlookups : S->nsearches)++;
    }
    S->t_last = now;
    S->nbatches++;
    S->scratch_in_use -= B.scratch;
    S->class_running[B.cls]--;
    S->done_cv.notify_all();
}

// Launch a batch on stream si: boards up, lookup or search kernels, results down.
int launch_batch(pentago_server *S, int si, Batch &B)
{
    const hipStream_t st = S->streams[si];
    const size_t n = B.qs.size();
    for (size_t i = 0; i < n; i++) {
        S->h_boards[si][i] = B.qs[i].board;
        S->h_sec[si][i] = B.qs[i].sec;
    }
    hipError_t e = hipMemcpyAsync(S->d_boards[si], S->h_boards[si], n * 8, hipMemcpyHostToDevice, st);
    int rc = 0;
    if (e == hipSuccess && B.cls == 0) {
        e = hipMemcpyAsync(S->d_sec[si], S->h_sec[si], n * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = launch_lookup(S->d_boards[si], S->d_sec[si], (int)n, S->d_secs, S->d_out[si], S->T, st);
    } else if (e == hipSuccess && B.cls == 5) {
        rc = eval_deep_enqueue(B.qs[0].board, S->d_out[si], st);
    } else if (e == hipSuccess) {
        // search classes 1..4 (empties <= 6, 7, 8, 9-10) -> endgame classes 2, 1, 0, 0
        const int ecls = B.cls == 1 ? 2 : B.cls == 2 ? 1 : 0;
        rc = eval_enqueue_class(S->d_boards[si], n, S->d_out[si], ecls, B.cls == 4, S->grid, st);
    }
    if (e == hipSuccess && rc == 0)
        e = hipMemcpyAsync(S->h_out[si], S->d_out[si], n * 64, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && rc == 0) e = hipEventRecord(B.done, st);
    if (e != hipSuccess) return hip_fail(e, "serve launch");
    return rc;
}

void worker_loop(pentago_server *S)
{
    (void)hipSetDevice(S->device);
    const size_t nst = S->streams.size();
    while (!S->stop.load()) {
        bool progress = false;
        // 1. completions
        for (size_t i = 0; i < nst; i++) {
            if (!S->busy[i]) continue;
            if (hipEventQuery(S->running[i].done) == hipSuccess) {
                publish(S, S->running[i]);
                S->running[i].qs.clear();
                S->busy[i] = false;
                progress = true;
            }
        }
        // 2. admissions, while a stream is idle and memory allows: lookups
        //    first (they take microseconds), then the oldest search class.
        //    With two or more streams, stream 0 runs lookups only, so a
        //    lookup never waits behind a search batch.
        for (size_t i = 0; i < nst; i++) {
            if (S->busy[i]) continue;
            if (S->npending.load(std::memory_order_relaxed) == 0) break;
            Batch &B = S->running[i];
            {
                std::lock_guard<std::mutex> lock(S->mu);
                int best = -1;
                if (!S->pending[0].empty()) best = 0;
                else if (i > 0 || nst == 1) {
                    // one batch in flight per batched search class: under load
                    // the class's queue grows while its batch runs, so batches
                    // grow with the load instead of fragmenting; deep queries
                    // (one per batch) run on every search stream at once, so
                    // the small layers of one overlap the others' work
                    for (int c = 1; c < kClasses; c++)
                        if (!S->pending[c].empty() && (c == 5 || S->class_running[c] == 0) &&
                            (best < 0 || S->pending[c].front().t_submit < S->pending[best].front().t_submit))
                            best = c;
                }
                if (best < 0) continue;
                const size_t take = best == 5 ? 1 : std::min<size_t>(S->pending[best].size(), S->cfg.max_batch);
                const size_t need = best == 0   ? 0
                                    : best == 5 ? deep_scratch_bytes(board_empties(S->pending[5].front().board))
                                                : eval_scratch_bytes(take, S->grid, best == 4);
                // lookups hold no scratch: the budget never holds them back
                if (need > 0 && S->scratch_in_use + need > S->cfg.memory_budget && S->scratch_in_use > 0)
                    continue;
                B.cls = best;
                S->class_running[best]++;
                B.qs.assign(S->pending[best].begin(), S->pending[best].begin() + take);
                S->pending[best].erase(S->pending[best].begin(), S->pending[best].begin() + take);
                S->npending.fetch_sub(take, std::memory_order_relaxed);
                B.scratch = need;
                S->scratch_in_use += need;
            }
            B.stream = (int)i;
            if (launch_batch(S, (int)i, B) != 0) {
                std::lock_guard<std::mutex> lock(S->mu);
                S->worker_error = PENTAGO_EDEVICE;
                S->done_cv.notify_all();
                for (const Query &q : B.qs) S->live.erase(q.ticket);
                S->scratch_in_use -= B.scratch;
                S->class_running[B.cls]--;
                B.qs.clear();
                continue;
            }
            S->busy[i] = true;
            progress = true;
        }
        if (!progress) {
            std::unique_lock<std::mutex> lock(S->mu);
            bool idle = true;
            for (size_t i = 0; i < nst; i++) idle = idle && !S->busy[i];
            bool empty = true;
            for (int c = 0; c < kClasses; c++) empty = empty && S->pending[c].empty();
            if (idle && empty) S->cv.wait_for(lock, std::chrono::milliseconds(2));
            else {
                lock.unlock();
                std::this_thread::yield();
            }
        }
    }
}

void destroy_buffers(pentago_server *S)
{
    for (size_t i = 0; i < S->streams.size(); i++) {
        if (S->streams[i]) (void)hipStreamSynchronize(S->streams[i]);
        if (S->running.size() > i && S->running[i].done) (void)hipEventDestroy(S->running[i].done);
        if (S->h_boards[i]) (void)hipHostFree(S->h_boards[i]);
        if (S->h_sec[i]) (void)hipHostFree(S->h_sec[i]);
        if (S->h_out[i]) (void)hipHostFree(S->h_out[i]);
        if (S->d_boards[i]) (void)hipFree(S->d_boards[i]);
        if (S->d_sec[i]) (void)hipFree(S->d_sec[i]);
        if (S->d_out[i]) (void)hipFree(S->d_out[i]);
        if (S->streams[i]) (void)hipStreamDestroy(S->streams[i]);
    }
    if (S->d_secs) (void)hipFree(S->d_secs);
}

}  // namespace

extern "C" {

int pentago_serve_create(const pentago_serve_config *cfg, pentago_server **out)
{
    if (!cfg || !out) return fail(PENTAGO_EINVAL, "NULL argument");
    if (cfg->streams < 1 || cfg->streams > 8 || cfg->max_batch < 1 || cfg->max_inflight < 1)
        return fail(PENTAGO_EINVAL, "streams must be 1..8, max_batch and max_inflight positive");
    pentago_server *S = new pentago_server;
    S->cfg = *cfg;
    (void)hipGetDevice(&S->device);
    int rc = device_tables(&S->T);
    if (rc == 0) rc = eval_grid(&S->grid);
    if (rc) { delete S; return rc; }
    const size_t nst = cfg->streams, mb = cfg->max_batch;
    S->streams.assign(nst, nullptr);
    S->h_boards.assign(nst, nullptr); S->d_boards.assign(nst, nullptr);
    S->h_sec.assign(nst, nullptr); S->d_sec.assign(nst, nullptr);
    S->h_out.assign(nst, nullptr); S->d_out.assign(nst, nullptr);
    S->running.assign(nst, Batch());
    S->busy.assign(nst, false);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < nst && e == hipSuccess; i++) {
        e = hipStreamCreateWithFlags(&S->streams[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&S->running[i].done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void **)&S->h_boards[i], mb * 8);
        if (e == hipSuccess) e = hipHostMalloc((void **)&S->h_sec[i], mb * 4);
        if (e == hipSuccess) e = hipHostMalloc((void **)&S->h_out[i], mb * 64);
        if (e == hipSuccess) e = hipMalloc((void **)&S->d_boards[i], mb * 8);
        if (e == hipSuccess) e = hipMalloc((void **)&S->d_sec[i], mb * 4);
        if (e == hipSuccess) e = hipMalloc((void **)&S->d_out[i], mb * 64);
    }
    if (e != hipSuccess) {
        destroy_buffers(S);
        delete S;
        return hip_fail(e, "server buffers");
    }
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return 0;
}

int pentago_serve_add_section(pentago_server *srv, pentago_section s, const pentago_superinfo *table)
{
    if (!srv || !table || !section_valid(s)) return fail(PENTAGO_EINVAL, "invalid arguments");
    ResidentSection r;
    r.table = (const uint4 *)table;
    section_shape_of(s, r.m);
    std::lock_guard<std::mutex> lock(srv->mu);
    if (srv->inflight > 0) return fail(PENTAGO_EINVAL, "sections are registered before queries are submitted");
    auto it = srv->resident.find(key_of(s));
    int index;
    if (it != srv->resident.end() && (it->second >> 24) == 0) {
        index = it->second;  // registered before: replace its table
        srv->secs[index] = r;
    } else {
        if (srv->secs.size() >= (1u << 24)) return fail(PENTAGO_ERANGE, "too many resident sections");
        index = (int)srv->secs.size();
        srv->secs.push_back(r);
        srv->resident[key_of(s)] = index;
    }
    // its images under the board symmetries, unless registered themselves
    for (int d = 1; d < 8; d++) {
        const SecKey k = key_of(section_image(s, d));
        auto jt = srv->resident.find(k);
        if (jt == srv->resident.end() || (jt->second >> 24) != 0) srv->resident[k] = index | (d << 24);
    }
    if (srv->secs.size() > srv->d_secs_cap) {
        // grow the device copy after the device is idle (lookups in flight
        // read the old one)
        size_t cap = std::max<size_t>(64, 2 * srv->secs.size());
        ResidentSection *d = nullptr;
        if (srv->d_secs) (void)hipDeviceSynchronize();
        if (hipMalloc((void **)&d, cap * sizeof(ResidentSection)) != hipSuccess)
            return fail(PENTAGO_ENOMEM, "resident section table");
        if (srv->d_secs) (void)hipFree(srv->d_secs);
        srv->d_secs = d;
        srv->d_secs_cap = cap;
    }
    // entries are only appended (or replaced for a re-registered section), so
    // lookups in flight keep reading valid entries
    if (hipMemcpy(srv->d_secs, srv->secs.data(), srv->secs.size() * sizeof(ResidentSection),
                  hipMemcpyHostToDevice) != hipSuccess)
        return fail(PENTAGO_EDEVICE, "resident section table upload");
    return 0;
}

int pentago_serve_submit(pentago_server *srv, pentago_board board, uint64_t *ticket)
{
    if (!srv || !ticket) return fail(PENTAGO_EINVAL, "NULL argument");
    int nb = 0, nw = 0;
    pentago_section s;
    for (int j = 0; j < 4; j++) {
        if (board.q[j] >= 19683) return fail(PENTAGO_EINVAL, "invalid quadrant code");
        int b = 0, w = 0, x = board.q[j];
        for (int l = 0; l < 9; l++, x /= 3) {
            b += x % 3 == 1;
            w += x % 3 == 2;
        }
        s.black[j] = (uint8_t)b;
        s.white[j] = (uint8_t)w;
        nb += b;
        nw += w;
    }
    if (nb != nw && nb != nw + 1) return fail(PENTAGO_EINVAL, "invalid stone counts");
    const int e = 36 - nb - nw;
    Query q;
    q.board = (uint64_t)board.q[0] | ((uint64_t)board.q[1] << 16) | ((uint64_t)board.q[2] << 32) |
              ((uint64_t)board.q[3] << 48);
    q.t_submit = Clock::now();
    std::lock_guard<std::mutex> lock(srv->mu);
    if (srv->worker_error) return fail(srv->worker_error, "server worker failed");
    if (srv->inflight >= srv->cfg.max_inflight) return PENTAGO_EAGAIN;
    auto it = srv->resident.find(key_of(s));
    if (it != srv->resident.end()) {
        q.cls = 0;
        q.sec = it->second;
    } else {
        if (e > 20) return fail(PENTAGO_ERANGE, "more than 20 empty cells and no resident section");
        q.cls = class_of_empties(e);
        q.sec = 0;
    }
    q.ticket = srv->next_ticket++;
    srv->live[q.ticket] = 0;
    srv->inflight++;
    if (!srv->any) {
        srv->any = true;
        srv->t_first = q.t_submit;
    }
    srv->pending[q.cls].push_back(q);
    srv->npending.fetch_add(1, std::memory_order_relaxed);
    *ticket = q.ticket;
    srv->cv.notify_one();
    return 0;
}

int pentago_serve_poll(pentago_server *srv, uint64_t ticket, pentago_superinfo *out)
{
    if (!srv || !out) return fail(PENTAGO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->live.find(ticket);
    if (it == srv->live.end()) return fail(srv->worker_error ? srv->worker_error : PENTAGO_EINVAL,
                                           "unknown ticket");
    if (it->second == 0) return PENTAGO_EAGAIN;
    *out = srv->results[ticket];
    srv->results.erase(ticket);
    srv->live.erase(it);
    srv->inflight--;
    return 0;
}

int pentago_serve_stats_get(pentago_server *srv, pentago_serve_stats *st)
{
    if (!srv || !st) return fail(PENTAGO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    memset(st, 0, sizeof(*st));
    st->queries = srv->nqueries;
    st->lookups = srv->nlookups;
    st->searches = srv->nsearches;
    st->batches = srv->nbatches;
    auto pct = [](std::vector<double> v, double *p50, double *p99) {
        if (v.empty()) return;
        std::sort(v.begin(), v.end());
        *p50 = v[(v.size() - 1) / 2];
        *p99 = v[(size_t)((v.size() - 1) * 0.99)];
    };
    pct(srv->lat_lookup_us, &st->lookup_p50_us, &st->lookup_p99_us);
    pct(srv->lat_search_us, &st->search_p50_us, &st->search_p99_us);
    if (!srv->lat_us.empty()) {
        pct(srv->lat_us, &st->p50_us, &st->p99_us);
        const double span = std::chrono::duration<double>(srv->t_last - srv->t_first).count();
        st->queries_per_s = span > 0 ? srv->nqueries / span : 0;
    }
    return 0;
}

int pentago_serve_reset_stats(pentago_server *srv)
{
    if (!srv) return fail(PENTAGO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->lat_us.clear();
    srv->lat_lookup_us.clear();
    srv->lat_search_us.clear();
    srv->nqueries = srv->nlookups = srv->nsearches = srv->nbatches = 0;
    srv->any = false;
    return 0;
}

int pentago_serve_replay(pentago_server *srv, const pentago_board *boards, const double *arrival_s,
                         size_t n, pentago_superinfo *results)
{
    if (!srv || (n && (!boards || !arrival_s || !results))) return fail(PENTAGO_EINVAL, "NULL argument");
    std::vector<uint64_t> tickets(n, 0);
    std::vector<std::atomic<int>> ready(n);
    for (size_t i = 0; i < n; i++) ready[i].store(0);
    std::atomic<int> err{0};
    // results are collected in submission order; the collector sleeps on the
    // server's completion signal instead of polling
    std::thread poller([&] {
        for (size_t i = 0; i < n && !err.load(); i++) {
            while (!ready[i].load() && !err.load()) std::this_thread::yield();
            if (err.load()) break;
            std::unique_lock<std::mutex> lock(srv->mu);
            srv->done_cv.wait(lock, [&] {
                auto it = srv->live.find(tickets[i]);
                return srv->worker_error != 0 || it == srv->live.end() || it->second != 0;
            });
            auto it = srv->live.find(tickets[i]);
            if (it == srv->live.end() || it->second == 0) {
                err.store(srv->worker_error ? srv->worker_error : PENTAGO_EINVAL);
                break;
            }
            results[i] = srv->results[tickets[i]];
            srv->results.erase(tickets[i]);
            srv->live.erase(it);
            srv->inflight--;
        }
    });
    const Clock::time_point t0 = Clock::now();
    for (size_t i = 0; i < n && !err.load(); i++) {
        const Clock::time_point target =
            t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
        while (Clock::now() < target) {}
        for (;;) {
            const int rc = pentago_serve_submit(srv, boards[i], &tickets[i]);
            if (rc == 0) break;
            if (rc != PENTAGO_EAGAIN) { err.store(rc); break; }
            std::this_thread::yield();
        }
        ready[i].store(1);
    }
    poller.join();
    return err.load();
}

int pentago_serve_destroy(pentago_server *srv)
{
    if (!srv) return 0;
    srv->stop.store(true);
    srv->cv.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    destroy_buffers(srv);
    delete srv;
    return 0;
}

}  // extern "C"
