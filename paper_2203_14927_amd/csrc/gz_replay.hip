// Replay of a multi-session workload through a server from native client
// threads: the load generator of the serving path.  Each client thread drives
// its share of the sessions (k = t, t + T, ...) and takes completions with
// gz_wait_any, so no thread waits on one session while another of its sessions
// could go on, and the measured rate is the server's, not the clients'.
#include <algorithm>
#include <chrono>
#include <mutex>
#include <queue>
#include <thread>
#include <vector>

#include "gz_internal.h"

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

void sleep_until_ns(uint64_t t) {
    const uint64_t n = now_ns();
    if (t > n) std::this_thread::sleep_for(std::chrono::nanoseconds(t - n));
}

struct Live {
    gz_ticket* t;
    uint32_t sess;
    uint64_t batch;     // batch index (queries: the batch they follow)
    bool query;
    uint64_t sched_ns;  // arrival (open loop) or submission (closed loop)
};

struct ReplayCtx {
    gz_server* S;
    const gz_replay_session* sess;
    const uint64_t* offs;
    const uint32_t *src, *dst;
    const uint64_t* arrival;
    uint32_t query_every;
    uint64_t start;
    uint64_t* lat;
    uint64_t* svc;
    uint64_t* qlat;
    std::mutex mu;
    gz_status err = GZ_OK;
};

void client(ReplayCtx* C, uint32_t t, uint32_t T, uint32_t n_sessions) {
    std::vector<uint32_t> mine;
    for (uint32_t k = t; k < n_sessions; k += T) mine.push_back(k);
    std::vector<gz_session*> h(n_sessions, nullptr);
    std::vector<uint64_t> next(n_sessions, 0), left(n_sessions, 0);
    std::vector<Live> live;
    std::vector<gz_ticket*> tix;
    // open loop: (time, session, kind) with kind 0 = open the session, 1 = next batch
    using Ev = std::tuple<uint64_t, uint32_t, int>;
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> evq;
    gz_status st = GZ_OK;
    auto submit_batch = [&](uint32_t k, uint64_t sched) -> gz_status {
        const gz_replay_session& s = C->sess[k];
        const uint64_t b = s.first_batch + next[k];
        gz_ticket* tk = nullptr;
        gz_status e = gz_submit_updates(h[k], C->src + C->offs[b], C->dst + C->offs[b],
                                        C->offs[b + 1] - C->offs[b], &tk);
        if (e) return e;
        live.push_back(Live{tk, k, b, false, sched});
        ++next[k];
        ++left[k];
        if ((C->query_every && next[k] % C->query_every == 0) || next[k] == s.n_batches) {
            e = gz_submit_query(h[k], nullptr, &tk);
            if (e) return e;
            live.push_back(Live{tk, k, b, true, sched});
            ++left[k];
        }
        return GZ_OK;
    };
    sleep_until_ns(C->start);
    for (uint32_t k : mine) {
        if (!C->arrival) {
            st = gz_session_open(C->S, C->sess[k].V, C->sess[k].seed, &h[k]);
            if (!st && C->sess[k].n_batches) st = submit_batch(k, now_ns());
            if (st) break;
        } else {
            evq.emplace(C->start + C->sess[k].open_ns, k, 0);
        }
    }
    while (!st && (!live.empty() || !evq.empty())) {
        uint64_t now = now_ns();
        while (!st && !evq.empty() && std::get<0>(evq.top()) <= now) {
            const auto [when, k, kind] = evq.top();
            evq.pop();
            if (kind == 0) {
                st = gz_session_open(C->S, C->sess[k].V, C->sess[k].seed, &h[k]);
                if (!st && C->sess[k].n_batches)
                    evq.emplace(C->start + C->arrival[C->sess[k].first_batch], k, 1);
            } else {
                st = submit_batch(k, when);
                if (!st && next[k] < C->sess[k].n_batches)
                    evq.emplace(C->start + C->arrival[C->sess[k].first_batch + next[k]], k, 1);
            }
        }
        if (st) break;
        if (live.empty()) {
            if (!evq.empty()) sleep_until_ns(std::get<0>(evq.top()));
            continue;
        }
        tix.resize(live.size());
        for (size_t i = 0; i < live.size(); ++i) tix[i] = live[i].t;
        now = now_ns();
        const uint64_t timeout =
            evq.empty() ? UINT64_MAX
                        : (std::get<0>(evq.top()) > now ? std::get<0>(evq.top()) - now : 0);
        uint32_t idx = 0;
        gz_result r{};
        const gz_status w = gz_wait_any(tix.data(), (uint32_t)tix.size(), timeout, &idx, &r);
        if (w == GZ_ETIMEOUT) continue;
        if (idx >= live.size()) {
            st = w ? w : GZ_EDEVICE;
            break;
        }
        const Live L = live[idx];
        live[idx] = live.back();
        live.pop_back();
        if (w) {
            st = w;
            break;
        }
        const uint64_t from = C->arrival ? L.sched_ns : r.submit_ns;
        const uint64_t lat = r.done_ns - std::min(from, r.done_ns);
        const uint64_t svc_from = std::max(from, r.admit_ns);
        const uint64_t svc = r.done_ns - std::min(svc_from, r.done_ns);
        if (L.query) {
            if (C->qlat) C->qlat[L.batch] = lat;
        } else {
            if (C->lat) C->lat[L.batch] = lat;
            if (C->svc) C->svc[L.batch] = svc;
        }
        const uint32_t k = L.sess;
        if (--left[k] == 0) {
            if (next[k] < C->sess[k].n_batches) {
                if (!C->arrival) st = submit_batch(k, now_ns());
            } else {
                st = gz_session_close(h[k]);
                h[k] = nullptr;
            }
        }
    }
    if (st) {
        // drain what this thread still holds, then close its sessions
        for (Live& L : live) gz_wait(L.t, nullptr);
        std::lock_guard<std::mutex> lk(C->mu);
        if (!C->err) C->err = st;
    }
    for (uint32_t k : mine)
        if (h[k]) gz_session_close(h[k]);
}

}  // namespace

extern "C" gz_status gz_server_replay(gz_server* S, const gz_replay_session* sessions,
                                      uint32_t n_sessions, const uint64_t* batch_offs,
                                      uint64_t n_batches, const uint32_t* src,
                                      const uint32_t* dst, const uint64_t* arrival_ns,
                                      uint32_t query_every, uint32_t client_threads,
                                      uint64_t* batch_latency_ns, uint64_t* batch_service_ns,
                                      uint64_t* query_latency_ns, uint64_t* wall_ns) {
    if (!S || !sessions || !batch_offs || !client_threads || (n_batches && (!src || !dst)))
        return gz::fail(GZ_EINVAL, "null argument");
    for (uint32_t k = 0; k < n_sessions; ++k) {
        const gz_replay_session& s = sessions[k];
        if (s.first_batch + s.n_batches > n_batches)
            return gz::fail(GZ_EINVAL, "a session's batches run past the batch table");
        if (arrival_ns && s.n_batches && arrival_ns[s.first_batch] < s.open_ns)
            return gz::fail(GZ_EINVAL, "a session's first batch arrives before it opens");
    }
    for (uint64_t b = 0; b < n_batches; ++b)
        if (batch_offs[b + 1] < batch_offs[b])
            return gz::fail(GZ_EINVAL, "batch offsets must be non-decreasing");
    for (uint64_t* a : {batch_latency_ns, batch_service_ns, query_latency_ns})
        if (a) std::fill(a, a + n_batches, 0);
    ReplayCtx C;
    C.S = S;
    C.sess = sessions;
    C.offs = batch_offs;
    C.src = src;
    C.dst = dst;
    C.arrival = arrival_ns;
    C.query_every = query_every;
    C.lat = batch_latency_ns;
    C.svc = batch_service_ns;
    C.qlat = query_latency_ns;
    C.start = now_ns() + 20000000ull;  // every client starts its clock together
    const uint32_t T = std::min(client_threads, std::max(n_sessions, 1u));
    std::vector<std::thread> th;
    for (uint32_t t = 0; t < T; ++t) th.emplace_back(client, &C, t, T, n_sessions);
    for (auto& x : th) x.join();
    if (wall_ns) *wall_ns = now_ns() - C.start;
    if (C.err) return gz::fail(C.err, "replay: a request failed");
    return GZ_OK;
}
