// Serving: many graph sessions share one GPU.  A server thread admits
// sessions while their sketches fit an HBM budget and packs the update batches
// queued by all admitted sessions into one fused multi-graph ingest per tick
// (continuous batching: a batch submitted while a tick runs joins the next
// one).  Connectivity queries go to a small pool of query threads, each query
// on its session's own stream, so that queries of different sessions and the
// next ticks' ingests overlap on the device.  Requests of one session are
// applied in submission order: a query is taken once the session's earlier
// batches are applied, and the session's later batches wait for the query.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "gz_internal.h"

namespace {

constexpr int kQueryThreads = 4;

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

uint32_t bitlen64(uint64_t x) {
    uint32_t n = 0;
    while (x) { ++n; x >>= 1; }
    return n;
}

// device bytes a session holds: sketches plus its query scratch
uint64_t session_bytes(uint32_t V) {
    const uint64_t n = (uint64_t)V * (V - 1) / 2;
    const uint64_t R = bitlen64(V - 1) + 1, B = bitlen64(n - 1) + 1;
    const uint64_t sketch = 12ull * B * R * GZ_COLUMNS * V;
    const uint64_t query = (uint64_t)V * (3 * B * GZ_COLUMNS * 4 + 96);
    return sketch + query;
}

}  // namespace

struct gz_ticket {
    enum Kind { UPDATES, QUERY } kind = UPDATES;
    gz_session* sess = nullptr;
    std::vector<uint32_t> src, dst;
    uint32_t* labels = nullptr;
    gz_result res{};
    bool done = false;
};

struct gz_session {
    gz_server* srv = nullptr;
    uint32_t V = 0;
    uint64_t seed = 0;
    uint64_t bytes = 0;
    gz_graph* g = nullptr;            // non-null once admitted
    std::deque<gz_ticket*> queue;     // submitted, not yet taken by a tick
    uint32_t inflight = 0;            // taken, not yet completed (batches and query)
    uint32_t upd_inflight = 0;        // batches taken, not yet completed
    bool query_busy = false;          // a query of this session is running
    bool closing = false;
    std::vector<uint32_t> scratch_labels;
};

struct gz_server {
    int device = 0;
    uint64_t budget = 0, used = 0, tick_cap = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_query;
    std::deque<gz_ticket*> qq;        // queries handed to the query threads
    std::vector<std::thread> query_threads;
    uint32_t queries_running = 0;
    bool stop_queries = false;
    std::vector<gz_session*> admitted;
    std::deque<gz_session*> waiting;
    std::thread worker;
    bool stop = false;
    hipStream_t stream = nullptr;
    // double-buffered pinned staging of a tick's updates
    uint32_t* h_stage[2] = {nullptr, nullptr};
    uint64_t stage_cap[2] = {0, 0};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    gz_server_stats stats{};
    gz_status error = GZ_OK;  // first device error seen by the worker
};

namespace {

// Take work for one tick under the lock: each admitted session contributes
// the update batches at the front of its queue (up to the tick's budget of
// updates) and, if a query then heads its queue, that query.
struct Tick {
    std::vector<gz_session*> upd_sessions;
    std::vector<std::vector<gz_ticket*>> upd;
    std::vector<gz_ticket*> queries;
    uint64_t n = 0;
};

void take_tick(gz_server* S, Tick& t) {
    for (gz_session* s : S->admitted) {
        if (s->query_busy) continue;  // later batches wait for the running query
        std::vector<gz_ticket*> mine;
        while (!s->queue.empty() && s->queue.front()->kind == gz_ticket::UPDATES) {
            gz_ticket* k = s->queue.front();
            if (t.n > 0 && t.n + k->src.size() > S->tick_cap) break;
            t.n += k->src.size();
            mine.push_back(k);
            s->queue.pop_front();
        }
        if (!mine.empty()) {
            t.upd_sessions.push_back(s);
            s->inflight += (uint32_t)mine.size();
            s->upd_inflight += (uint32_t)mine.size();
            t.upd.push_back(std::move(mine));
        }
        // a query runs once every earlier batch of its session is applied
        if (!s->queue.empty() && s->queue.front()->kind == gz_ticket::QUERY &&
            s->upd_inflight == 0) {
            t.queries.push_back(s->queue.front());
            s->queue.pop_front();
            s->inflight += 1;
            s->query_busy = true;
            S->queries_running++;
        }
    }
}

void admit(gz_server* S) {
    while (!S->waiting.empty() && S->used + S->waiting.front()->bytes <= S->budget) {
        gz_session* s = S->waiting.front();
        gz_graph* g = nullptr;
        if (gz_sketch_init(&g, s->V, s->seed, nullptr) != GZ_OK) break;  // retry later
        s->g = g;
        S->used += s->bytes;
        S->waiting.pop_front();
        S->admitted.push_back(s);
        S->stats.sessions_admitted++;
    }
}

bool has_work(gz_server* S) {
    for (gz_session* s : S->admitted)
        if (!s->query_busy && !s->queue.empty() &&
            (s->queue.front()->kind == gz_ticket::UPDATES || s->upd_inflight == 0))
            return true;
    if (!S->waiting.empty() && S->used + S->waiting.front()->bytes <= S->budget) return true;
    return false;
}

void complete(gz_server* S, gz_ticket* k, gz_status st) {
    k->res.status = st;
    k->res.done_ns = now_ns();
    std::lock_guard<std::mutex> lk(S->mu);
    k->done = true;
    k->sess->inflight -= 1;
    if (k->kind == gz_ticket::UPDATES) k->sess->upd_inflight -= 1;
    S->cv_done.notify_all();
}

// Query threads: run the queries the tick loop hands over, each on its
// session's query stream; the session's next batches are released afterwards.
void query_main(gz_server* S) {
    hipSetDevice(S->device);
    for (;;) {
        gz_ticket* k = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_query.wait(lk, [&] { return S->stop_queries || !S->qq.empty(); });
            if (S->qq.empty()) return;
            k = S->qq.front();
            S->qq.pop_front();
        }
        gz_session* s = k->sess;
        k->res.start_ns = now_ns();
        uint32_t* out = k->labels;
        if (!out) {
            s->scratch_labels.resize(s->V);
            out = s->scratch_labels.data();
        }
        uint32_t ncc = 0;
        const gz_status q = gz_connected_components(s->g, out, &ncc);
        k->res.num_cc = ncc;
        k->res.status = q;
        k->res.done_ns = now_ns();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stats.queries++;
            k->done = true;
            s->inflight -= 1;
            s->query_busy = false;
            S->queries_running--;
            S->cv_done.notify_all();
        }
        S->cv_work.notify_one();
    }
}

void worker_main(gz_server* S) {
    hipSetDevice(S->device);
    struct Pending {
        Tick tick;
        int buf = -1;
    };
    Pending prev;  // the previous tick's updates, completed when its ingest finishes
    int buf = 0;
    for (;;) {
        Tick t;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            admit(S);
            if (prev.buf < 0)
                S->cv_work.wait(lk, [&] {
                    return (S->stop && S->queries_running == 0) || has_work(S);
                });
            admit(S);
            if (S->stop && !has_work(S) && prev.buf < 0 && S->queries_running == 0) break;
            take_tick(S, t);
        }
        // 1. launch this tick's fused ingest (host staging -> device, async)
        gz_status st = GZ_OK;
        if (t.n > 0) {
            if (S->stage_cap[buf] < 2 * t.n) {
                hipEventSynchronize(S->stage_ev[buf]);
                hipHostFree(S->h_stage[buf]);
                S->h_stage[buf] = nullptr;
                S->stage_cap[buf] = 0;
                if (hipHostMalloc((void**)&S->h_stage[buf], 8 * t.n, hipHostMallocDefault) ==
                    hipSuccess)
                    S->stage_cap[buf] = 2 * t.n;
                else
                    st = GZ_ENOMEM;
            } else {
                hipEventSynchronize(S->stage_ev[buf]);  // its last upload has left the buffer
            }
            if (!st) {
                uint32_t* hs = S->h_stage[buf];
                uint32_t* hd = hs + t.n;
                std::vector<gz_graph*> gs;
                std::vector<uint64_t> offs(1, 0);
                uint64_t at = 0;
                const uint64_t start = now_ns();
                for (size_t i = 0; i < t.upd_sessions.size(); ++i) {
                    gs.push_back(t.upd_sessions[i]->g);
                    for (gz_ticket* k : t.upd[i]) {
                        std::memcpy(hs + at, k->src.data(), 4 * k->src.size());
                        std::memcpy(hd + at, k->dst.data(), 4 * k->dst.size());
                        at += k->src.size();
                        k->res.start_ns = start;
                    }
                    offs.push_back(at);
                }
                st = gz_ingest_multi(gs.data(), (uint32_t)gs.size(), offs.data(), hs, hd, GZ_ASYNC,
                                     S->stream);
                if (!st && hipEventRecord(S->stage_ev[buf], S->stream) != hipSuccess)
                    st = GZ_EDEVICE;
                if (!st) {
                    std::lock_guard<std::mutex> lk(S->mu);
                    S->stats.ticks++;
                    S->stats.updates += t.n;
                }
            }
        }
        // 2. hand the queries to the query threads
        if (!t.queries.empty()) {
            {
                std::lock_guard<std::mutex> lk(S->mu);
                for (gz_ticket* k : t.queries) S->qq.push_back(k);
            }
            S->cv_query.notify_all();
        }
        // 3. the previous tick's updates are applied once its ingest is done
        if (prev.buf >= 0) {
            gz_status pst = hipEventSynchronize(S->stage_ev[prev.buf]) == hipSuccess ? GZ_OK
                                                                                      : GZ_EDEVICE;
            // Every batch was validated when it was submitted, so the ingest
            // cannot have met an invalid update: its completion is all that is
            // left to wait for, and the graphs need no flush-time error check
            // (two synchronous device reads per session, most of a tick's time
            // when a tick holds dozens of sessions).  No query of these
            // sessions runs until their batches complete, below.
            for (size_t i = 0; i < prev.tick.upd_sessions.size(); ++i) {
                prev.tick.upd_sessions[i]->g->pending_error = false;
                for (gz_ticket* k : prev.tick.upd[i]) complete(S, k, pst);
            }
            prev = Pending{};
        }
        if (t.n > 0) {
            if (st) {
                for (size_t i = 0; i < t.upd_sessions.size(); ++i)
                    for (gz_ticket* k : t.upd[i]) complete(S, k, st);
                std::lock_guard<std::mutex> lk(S->mu);
                if (!S->error) S->error = st;
            } else {
                prev.tick = std::move(t);
                prev.buf = buf;
                buf ^= 1;
            }
        }
    }
}

}  // namespace

extern "C" {

gz_status gz_server_create(uint64_t hbm_budget, uint64_t tick_updates, gz_server** out) {
    if (!out) return gz::fail(GZ_EINVAL, "null output");
    *out = nullptr;
    gz_server* S = new gz_server();
    if (hipGetDevice(&S->device) != hipSuccess ||
        hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->stage_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&S->stage_ev[1], hipEventDisableTiming) != hipSuccess) {
        delete S;
        return gz::fail(GZ_EDEVICE, "server stream/events");
    }
    S->budget = hbm_budget;
    S->tick_cap = tick_updates ? tick_updates : (16ull << 20);
    S->stats.hbm_budget = hbm_budget;
    S->worker = std::thread(worker_main, S);
    for (int i = 0; i < kQueryThreads; ++i) S->query_threads.emplace_back(query_main, S);
    *out = S;
    return GZ_OK;
}

gz_status gz_session_open(gz_server* S, uint32_t V, uint64_t seed, gz_session** out) {
    if (!S || !out) return gz::fail(GZ_EINVAL, "null argument");
    *out = nullptr;
    if (V < 2 || V > GZ_MAX_NODES) return gz::fail(GZ_EINVAL, "V must be in [2, 65536]");
    gz_session* s = new gz_session();
    s->srv = S;
    s->V = V;
    s->seed = seed;
    s->bytes = session_bytes(V);
    if (s->bytes > S->budget) {
        delete s;
        return gz::fail(GZ_ENOMEM, "session larger than the whole HBM budget");
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->waiting.push_back(s);
    }
    S->cv_work.notify_one();
    *out = s;
    return GZ_OK;
}

static gz_status submit(gz_session* s, gz_ticket* k, gz_ticket** out) {
    gz_server* S = s->srv;
    k->sess = s;
    k->res.submit_ns = now_ns();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (s->closing) {
            delete k;
            return gz::fail(GZ_ESTATE, "session is closing");
        }
        s->queue.push_back(k);
    }
    S->cv_work.notify_one();
    *out = k;
    return GZ_OK;
}

gz_status gz_submit_updates(gz_session* s, const uint32_t* src, const uint32_t* dst, uint64_t N,
                            gz_ticket** out) {
    if (!s || !out || (N && (!src || !dst))) return gz::fail(GZ_EINVAL, "null argument");
    *out = nullptr;
    for (uint64_t i = 0; i < N; ++i)
        if (src[i] == dst[i] || src[i] >= s->V || dst[i] >= s->V)
            return gz::fail(GZ_EINVAL, "invalid update (self-loop or node id out of range)");
    gz_ticket* k = new gz_ticket();
    k->kind = gz_ticket::UPDATES;
    k->src.assign(src, src + N);
    k->dst.assign(dst, dst + N);
    k->res.updates = N;
    return submit(s, k, out);
}

gz_status gz_submit_query(gz_session* s, uint32_t* labels, gz_ticket** out) {
    if (!s || !out) return gz::fail(GZ_EINVAL, "null argument");
    *out = nullptr;
    gz_ticket* k = new gz_ticket();
    k->kind = gz_ticket::QUERY;
    k->labels = labels;
    return submit(s, k, out);
}

gz_status gz_wait(gz_ticket* k, gz_result* res) {
    if (!k) return gz::fail(GZ_EINVAL, "null ticket");
    gz_server* S = k->sess->srv;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return k->done; });
    }
    gz_result r = k->res;
    r.kind = k->kind == gz_ticket::QUERY ? 1u : 0u;
    if (res) *res = r;
    delete k;
    return r.status == GZ_ESKETCH_FAIL ? GZ_OK : r.status;
}

gz_status gz_session_close(gz_session* s) {
    if (!s) return GZ_OK;
    gz_server* S = s->srv;
    std::unique_lock<std::mutex> lk(S->mu);
    s->closing = true;
    if (!s->g) {
        // never admitted: its queued requests cannot run any more
        for (gz_ticket* k : s->queue) {
            k->res.status = GZ_ESTATE;
            k->res.done_ns = now_ns();
            k->done = true;
        }
        s->queue.clear();
        S->cv_done.notify_all();
    }
    S->cv_work.notify_one();
    S->cv_done.wait(lk, [&] { return s->queue.empty() && s->inflight == 0 && !s->query_busy; });
    auto it = std::find(S->admitted.begin(), S->admitted.end(), s);
    if (it != S->admitted.end()) {
        S->admitted.erase(it);
        S->used -= s->bytes;
    }
    auto wt = std::find(S->waiting.begin(), S->waiting.end(), s);
    if (wt != S->waiting.end()) S->waiting.erase(wt);
    gz_graph* g = s->g;
    lk.unlock();
    gz_free(g);
    delete s;
    S->cv_work.notify_one();  // memory freed: waiting sessions may be admitted
    return GZ_OK;
}

gz_status gz_server_get_stats(gz_server* S, gz_server_stats* out) {
    if (!S || !out) return gz::fail(GZ_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->hbm_used = S->used;
    out->sessions_waiting = S->waiting.size();
    out->sessions_active = S->admitted.size();
    return S->error;
}

gz_status gz_server_destroy(gz_server* S) {
    if (!S) return GZ_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_one();
    S->worker.join();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop_queries = true;
    }
    S->cv_query.notify_all();
    for (std::thread& t : S->query_threads) t.join();
    std::vector<gz_session*> left;
    for (gz_session* s : S->admitted) left.push_back(s);
    for (gz_session* s : S->waiting) left.push_back(s);
    for (gz_session* s : left) {
        for (gz_ticket* k : s->queue) delete k;
        gz_free(s->g);
        delete s;
    }
    for (int b = 0; b < 2; ++b) {
        if (S->stage_ev[b]) {
            hipEventSynchronize(S->stage_ev[b]);
            hipEventDestroy(S->stage_ev[b]);
        }
        hipHostFree(S->h_stage[b]);
    }
    hipStreamDestroy(S->stream);
    delete S;
    return GZ_OK;
}

}  // extern "C"
