// Serving: many graph sessions share one GPU.  An admission thread admits
// sessions while their sketches fit an HBM budget (their sketches and gutters
// cut from an arena allocated with the server), and a worker thread takes the
// update batches queued by all admitted sessions every tick (continuous
// batching: a batch submitted while a tick runs joins the next one).  A tick
// gathers batches into their sessions' gutters and applies the gutters that
// are full or that a query needs with one fused multi-graph ingest, so that
// each node's sketch is read and written once for many updates.  Connectivity queries go to two query threads, each answering all
// the queries queued at that time with one fused Boruvka run, so that queries
// and the next ticks' ingests overlap on the device.  Requests of one session
// are applied in submission order: a query is taken once the session's earlier
// batches are applied, and the session's later batches wait for the query.
//
// A batch reaches HBM with one host copy at most: gz_submit_updates copies
// (and validates) it into a pinned buffer on the submitting thread, and
// gz_submit_updates_inplace lends the caller's own device or pinned memory.
// Per tick, one gather kernel reads every batch of the tick where it lies
// (pinned host memory over the host link, device memory in HBM) into the
// tick's device staging arrays, which the fused ingest then reads.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "gz_internal.h"

namespace {

constexpr int kQueryThreads = 2;
constexpr uint32_t kGutterPerNode = 64;      // gutter updates per node of a session
constexpr uint64_t kGutterMin = 1ull << 16;  // and at least this many
constexpr size_t kQueryBatch = 512;  // queries answered by one fused run

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

// bytes of a session's sketches (V <= 2^16: three planes)
uint64_t sketch_bytes(uint32_t V) {
    const uint64_t n = (uint64_t)V * (V - 1) / 2;
    const uint64_t R = bitlen64(V - 1) + 1, B = bitlen64(n - 1) + 1;
    return 12ull * B * R * GZ_COLUMNS * V;
}

// a session's share of the server's arena: its sketches, then its gutter
uint64_t gutter_offset(uint32_t V) { return (sketch_bytes(V) + 255) & ~255ull; }
uint64_t arena_bytes(uint32_t V, uint64_t gcap) { return gutter_offset(V) + 8 * gcap; }

// The server's sketch memory: one device allocation made when the server is
// created, from which admitted sessions take their sketches (first fit,
// 256-byte granules, neighbours merged when freed).  Device allocations made
// while sessions are served (and the driver's clearing of them) would stall
// the device for every other session.
class Arena {
  public:
    static constexpr uint64_t kAlign = 256;
    bool init(uint64_t bytes) {
        bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
        if (!bytes || hipMalloc((void**)&base_, bytes) != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
            return false;
        }
        free_[0] = bytes;
        return true;
    }
    void release() {
        hipFree(base_);
        base_ = nullptr;
        free_.clear();
    }
    bool active() const { return base_ != nullptr; }
    bool fits(uint64_t bytes) const {
        bytes = round(bytes);
        for (const auto& f : free_)
            if (f.second >= bytes) return true;
        return false;
    }
    uint8_t* take(uint64_t bytes) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                const uint64_t off = it->first, size = it->second;
                free_.erase(it);
                if (size > bytes) free_[off + bytes] = size - bytes;
                return base_ + off;
            }
        return nullptr;
    }
    void give(uint8_t* p, uint64_t bytes) {
        if (!p) return;
        bytes = round(bytes);
        uint64_t off = (uint64_t)(p - base_);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

  private:
    static uint64_t round(uint64_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }
    uint8_t* base_ = nullptr;
    std::map<uint64_t, uint64_t> free_;  // offset -> bytes
};

// Pinned host buffers for copied batches, in power-of-two size classes and
// reused (allocating pinned memory costs far more than filling it).  Up to
// kKeepBytes of returned buffers are kept; beyond that they are freed.
class PinnedPool {
  public:
    static constexpr uint32_t kMinLog = 16;  // 64 KiB
    static constexpr uint64_t kKeepBytes = 4ull << 30;

    uint32_t* take(uint64_t bytes, uint64_t* cap) {
        uint32_t lg = kMinLog;
        while ((1ull << lg) < bytes) ++lg;
        *cap = 1ull << lg;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (free_.size() > lg && !free_[lg].empty()) {
                uint32_t* p = free_[lg].back();
                free_[lg].pop_back();
                kept_ -= *cap;
                return p;
            }
        }
        uint32_t* p = nullptr;
        if (hipHostMalloc((void**)&p, *cap, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess)
            return nullptr;
        return p;
    }
    void give(uint32_t* p, uint64_t cap) {
        if (!p) return;
        uint32_t lg = 0;
        while ((1ull << lg) < cap) ++lg;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (kept_ + cap <= kKeepBytes) {
                if (free_.size() <= lg) free_.resize(lg + 1);
                free_[lg].push_back(p);
                kept_ += cap;
                return;
            }
        }
        hipHostFree(p);
    }
    void release_all() {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto& v : free_)
            for (uint32_t* p : v) hipHostFree(p);
        free_.clear();
        kept_ = 0;
    }

  private:
    std::mutex mu_;
    std::vector<std::vector<uint32_t*>> free_;
    uint64_t kept_ = 0;
};

// One piece of a tick's gather: up to kGatherPiece updates of one batch, read
// from where the batch lies (or from a session's gutter) and written to the
// tick's staging arrays or into a session's gutter.
struct GatherPiece {
    const uint32_t* src;
    const uint32_t* dst;
    uint32_t* out_src;
    uint32_t* out_dst;
    uint32_t count;
    uint32_t pad;
};
constexpr uint32_t kGatherPiece = 4096;
constexpr uint32_t kGatherThreads = 256;
constexpr uint32_t kGatherUnroll = 4;  // loads of each array in flight per lane

__global__ __launch_bounds__(kGatherThreads) void k_srv_gather(
    const GatherPiece* __restrict__ pieces) {
    const GatherPiece p = pieces[blockIdx.x];
    // system-scope loads: host memory the caller may have rewritten since an
    // earlier tick read it is never served from a stale cached line; several
    // in flight per lane, since each crosses the host link
    for (uint32_t i0 = 0; i0 < p.count; i0 += kGatherThreads * kGatherUnroll) {
        uint32_t a[kGatherUnroll], b[kGatherUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kGatherUnroll; ++u) {
            const uint32_t i = i0 + u * kGatherThreads + threadIdx.x;
            a[u] = i < p.count ? __hip_atomic_load(p.src + i, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_SYSTEM)
                               : 0u;
            b[u] = i < p.count ? __hip_atomic_load(p.dst + i, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_SYSTEM)
                               : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < kGatherUnroll; ++u) {
            const uint32_t i = i0 + u * kGatherThreads + threadIdx.x;
            if (i < p.count) {
                p.out_src[i] = a[u];
                p.out_dst[i] = b[u];
            }
        }
    }
}

// in-place batches in device memory: any self-loop or id >= V sets *bad
__global__ __launch_bounds__(256) void k_srv_validate(const uint32_t* __restrict__ src,
                                                      const uint32_t* __restrict__ dst,
                                                      uint64_t n, uint32_t V,
                                                      uint32_t* __restrict__ bad) {
    uint32_t any = 0;
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += gridDim.x * 256ull) {
        const uint32_t a = src[i], b = dst[i];
        any |= (a == b) | (a >= V) | (b >= V);
    }
    if (__any(any) && __lane_id() == 0) atomicOr(bad, 1u);
}

}  // namespace

struct gz_ticket {
    enum Kind { UPDATES, QUERY } kind = UPDATES;
    gz_session* sess = nullptr;  // valid until the ticket completes
    gz_server* srv = nullptr;
    // update batches: device-readable addresses of the batch (a pinned copy, or
    // the caller's memory for in-place batches)
    const uint32_t* src = nullptr;
    const uint32_t* dst = nullptr;
    uint64_t n = 0;
    uint32_t* pinned = nullptr;  // the pool buffer of a copied batch
    uint64_t pinned_cap = 0;
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
    uint64_t admit_ns = 0;
    uint64_t wait_since = 0;          // when the session was opened
    uint8_t* storage = nullptr;       // its sketches in the server's arena
    bool admitting = false;           // its graph is being created
    std::deque<gz_ticket*> queue;     // submitted, not yet taken by a tick
    uint32_t inflight = 0;            // taken, not yet completed (batches and query)
    uint32_t upd_inflight = 0;        // batches taken, not yet completed
    bool query_busy = false;          // a query of this session is running
    bool closing = false;
    // The session's gutter: batches are gathered into it and applied to the
    // sketches together, when it cannot hold the next batch, when a query
    // needs them or when gz_session_graph asks, so that one ingest updates
    // each node's sketch with many updates at a time.
    uint32_t* gut = nullptr;          // gcap sources, then gcap destinations (in the arena)
    uint64_t gcap = 0;                // updates it holds (0: batches are applied as taken)
    uint64_t gfill = 0;               // updates in it, those a running gather writes included
    uint32_t ingests_inflight = 0;    // ticks whose ingest updates this session, not yet done
    bool flush_req = false;           // gz_session_graph waits for the gutter to be applied
    gz_status gstatus = GZ_OK;        // a failed ingest of its gutter, reported by its queries
};

struct gz_server {
    int device = 0;
    uint64_t budget = 0, used = 0, tick_cap = 0;
    uint32_t gutter_per_node = kGutterPerNode;  // sessions opened from now on
    uint64_t tick_seq = 0;
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
    std::thread admitter;            // creates admitted sessions' graphs
    std::condition_variable cv_admit;
    bool stop_admit = false;
    hipStream_t stream = nullptr;
    PinnedPool pool;
    Arena arena;  // sessions' sketches (inactive: each graph allocates its own)
    // double-buffered per-tick device staging (src then dst) and gather lists
    uint32_t* d_stage[2] = {nullptr, nullptr};
    uint64_t stage_cap[2] = {0, 0};  // updates
    GatherPiece* h_pieces[2] = {nullptr, nullptr};
    GatherPiece* d_pieces[2] = {nullptr, nullptr};
    uint64_t pieces_cap[2] = {0, 0};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    hipEvent_t tick_t0[2] = {nullptr, nullptr};  // timing: a tick's first and last kernel
    hipEvent_t tick_t1[2] = {nullptr, nullptr};
    std::vector<gz_tick_record> timeline;
    // validation of in-place device batches
    std::mutex vmu;
    hipStream_t vstream = nullptr;
    uint32_t* vflag = nullptr;  // pinned, mapped
    gz_server_stats stats{};
    gz_status error = GZ_OK;  // first device error seen by the worker
};

namespace {

// Take work for one tick under the lock.  Each admitted session contributes
// the update batches at the front of its queue (up to the tick's budget of new
// updates): into its gutter while they fit, else to the tick's ingest behind
// the gutter's content, which the tick then applies (a flush).  A query at the
// front of the queue, or gz_session_graph, has the gutter flushed too, and the
// query is taken once every earlier batch of its session is applied.  A tick
// that writes batches into a session's gutter does not also flush it: the
// flush of the next tick reads what this tick's gather wrote (one stream).
struct Tick {
    // sessions whose sketches the tick's ingest updates, each with the gutter
    // updates it flushes and the batches staged behind them
    std::vector<gz_session*> upd_sessions;
    std::vector<uint64_t> flushed;
    std::vector<std::vector<gz_ticket*>> upd;
    // batches gathered into their session's gutter, at that gutter position
    std::vector<std::pair<gz_ticket*, uint64_t>> gut;
    std::vector<gz_ticket*> queries;
    uint64_t n = 0;         // new updates taken
    uint64_t ingested = 0;  // updates the ingest applies (flushed and staged)
    uint32_t batches = 0;
    uint64_t take_ns = 0, launched_ns = 0;
};
constexpr size_t kTimelineCap = 1 << 20;  // tick records kept per server

bool query_ready(const gz_session* s) {
    return !s->queue.empty() && s->queue.front()->kind == gz_ticket::QUERY &&
           s->upd_inflight == 0 && s->ingests_inflight == 0 && s->gfill == 0;
}

bool flush_wanted(const gz_session* s) {
    return s->gfill > 0 && (s->flush_req || (!s->queue.empty() &&
                                             s->queue.front()->kind == gz_ticket::QUERY));
}

void take_tick(gz_server* S, Tick& t) {
    // a different session first in each tick: a session whose flush did not
    // fit one tick's budget comes early in a later one
    const size_t A = S->admitted.size();
    const size_t first = A ? S->tick_seq++ % A : 0;
    for (size_t j = 0; j < A; ++j) {
        gz_session* s = S->admitted[(first + j) % A];
        if (s->query_busy) continue;  // later batches wait for the running query
        std::vector<gz_ticket*> mine;
        bool flush = false, wrote_gutter = false;
        // flushes are bounded like new updates, one always allowed
        auto may_flush = [&] { return t.ingested == 0 || t.ingested + s->gfill <= S->tick_cap; };
        while (!s->queue.empty() && s->queue.front()->kind == gz_ticket::UPDATES) {
            gz_ticket* k = s->queue.front();
            if (t.n > 0 && t.n + k->n > S->tick_cap) break;
            if (s->gcap && !flush) {
                if (s->gfill + k->n <= s->gcap) {
                    t.gut.emplace_back(k, s->gfill);
                    s->gfill += k->n;
                    wrote_gutter = true;
                } else {
                    // the gutter cannot take the batch: flush it (in the next
                    // tick if this one wrote to it) and stage the batch behind
                    if (wrote_gutter || !may_flush()) break;
                    flush = true;
                    mine.push_back(k);
                }
            } else {
                mine.push_back(k);
            }
            t.n += k->n;
            t.batches++;
            s->inflight += 1;
            s->upd_inflight += 1;
            s->queue.pop_front();
        }
        if (!flush && !wrote_gutter && flush_wanted(s) && may_flush()) flush = true;
        if (flush || !mine.empty()) {
            uint64_t staged = flush ? s->gfill : 0;
            for (gz_ticket* k : mine) staged += k->n;
            t.upd_sessions.push_back(s);
            t.flushed.push_back(flush ? s->gfill : 0);
            t.upd.push_back(std::move(mine));
            t.ingested += staged;
            if (flush) s->gfill = 0;
            s->ingests_inflight += 1;
        }
        if (query_ready(s)) {
            t.queries.push_back(s->queue.front());
            s->queue.pop_front();
            s->inflight += 1;
            s->query_busy = true;
            S->queries_running++;
        }
    }
}

// The next waiting session to admit: the oldest one whose bytes fit.  Younger
// sessions may pass a waiting one that does not fit, until the oldest has
// waited kAdmitPatience; from then on only it may go, so that memory freed by
// closing sessions gathers for it instead of being taken by smaller ones.
constexpr uint64_t kAdmitPatienceNs = 100000000;  // 100 ms

std::deque<gz_session*>::iterator admissible(gz_server* S) {
    auto it = S->waiting.begin();
    if (it == S->waiting.end()) return it;
    const bool head_only = now_ns() - (*it)->wait_since > kAdmitPatienceNs;
    for (; it != S->waiting.end(); ++it) {
        if (S->used + (*it)->bytes <= S->budget &&
            (!S->arena.active() || S->arena.fits(arena_bytes((*it)->V, (*it)->gcap))))
            return it;
        if (head_only) break;
    }
    return S->waiting.end();
}

// Admit what fits.  Creating a session's graph (allocation, zeroing) runs with
// the lock released: clients, completions and queries go on meanwhile; the
// session counts against the budget from the start.
bool admit(gz_server* S, std::unique_lock<std::mutex>& lk) {
    for (;;) {
        auto it = admissible(S);
        if (it == S->waiting.end()) break;
        gz_session* s = *it;
        S->waiting.erase(it);
        S->used += s->bytes;
        s->admitting = true;
        gz_config cfg{};
        if (S->arena.active()) {
            s->storage = S->arena.take(arena_bytes(s->V, s->gcap));
            cfg.storage = s->storage;
            cfg.storage_bytes = sketch_bytes(s->V);
            if (s->gcap) s->gut = reinterpret_cast<uint32_t*>(s->storage + gutter_offset(s->V));
        }
        lk.unlock();
        gz_graph* g = nullptr;
        const uint64_t t0 = now_ns();
        const gz_status st = gz_sketch_init(&g, s->V, s->seed, &cfg);
        const uint64_t dt = now_ns() - t0;
        lk.lock();
        S->stats.create_ns += dt;
        S->stats.create_ns_max = std::max(S->stats.create_ns_max, dt);
        s->admitting = false;
        S->cv_done.notify_all();  // a close may wait for the admission to end
        if (st != GZ_OK) {
            S->used -= s->bytes;
            S->arena.give(s->storage, arena_bytes(s->V, s->gcap));
            s->storage = nullptr;
            s->gut = nullptr;
            S->waiting.push_front(s);  // retry later
            return false;
        }
        s->g = g;
        s->admit_ns = now_ns();
        S->admitted.push_back(s);
        S->stats.sessions_admitted++;
        S->cv_work.notify_one();  // its queued requests can run
    }
    return true;
}

// Admission runs on a thread of its own: creating a graph (allocating and
// zeroing gigabytes) takes milliseconds, which would otherwise stall the tick
// loop for every session admitted while others are served.
void admit_main(gz_server* S) {
    hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    bool ok = true;
    for (;;) {
        if (ok)
            S->cv_admit.wait(lk, [&] {
                return S->stop_admit || admissible(S) != S->waiting.end();
            });
        else  // a graph could not be created: try again a little later
            S->cv_admit.wait_for(lk, std::chrono::milliseconds(5));
        if (S->stop_admit) break;
        ok = admit(S, lk);
    }
}

bool has_work(gz_server* S) {
    for (gz_session* s : S->admitted)
        if (!s->query_busy &&
            ((!s->queue.empty() && s->queue.front()->kind == gz_ticket::UPDATES) ||
             flush_wanted(s) || query_ready(s)))
            return true;
    return false;
}

void complete(gz_server* S, gz_ticket* k, gz_status st) {
    k->res.status = st;
    k->res.done_ns = now_ns();
    std::lock_guard<std::mutex> lk(S->mu);
    k->res.admit_ns = k->sess->admit_ns;
    k->done = true;
    k->sess->inflight -= 1;
    if (k->kind == gz_ticket::UPDATES) k->sess->upd_inflight -= 1;
    S->cv_done.notify_all();
}

// Query threads: each takes every query queued so far (up to kQueryBatch) and
// answers them with one fused Boruvka run over their graphs, so that queries
// that come due together (sessions reach their n-th batch at similar times)
// cost one launch sequence; a session's next batches are released afterwards.
void query_main(gz_server* S) {
    hipSetDevice(S->device);
    uint32_t* lab = nullptr;  // pinned labels of a fused run
    uint64_t lab_cap = 0;
    for (;;) {
        std::vector<gz_ticket*> batch;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_query.wait(lk, [&] { return S->stop_queries || !S->qq.empty(); });
            if (S->qq.empty()) break;
            while (!S->qq.empty() && batch.size() < kQueryBatch) {
                batch.push_back(S->qq.front());
                S->qq.pop_front();
            }
        }
        const uint64_t start = now_ns();
        const uint32_t G = (uint32_t)batch.size();
        std::vector<gz_graph*> gs(G);
        std::vector<uint64_t> off(G + 1, 0);
        for (uint32_t i = 0; i < G; ++i) {
            batch[i]->res.start_ns = start;
            gs[i] = batch[i]->sess->g;
            off[i + 1] = off[i] + batch[i]->sess->V;
        }
        std::vector<uint32_t> ncc(G, 0);
        std::vector<int32_t> gst(G, GZ_OK);
        gz_status q = GZ_OK;
        if (lab_cap < off[G]) {
            hipHostFree(lab);
            lab = nullptr;
            lab_cap = 0;
            if (hipHostMalloc((void**)&lab, 4 * off[G], hipHostMallocDefault) == hipSuccess)
                lab_cap = off[G];
            else
                q = GZ_ENOMEM;
        }
        if (!q) q = gz_connected_components_multi(gs.data(), G, lab, ncc.data(), gst.data());
        const uint64_t done = now_ns();
        for (uint32_t i = 0; i < G; ++i) {
            gz_ticket* k = batch[i];
            k->res.num_cc = ncc[i];
            // a run that ended with a component still active reports that per graph
            k->res.status = q == GZ_OK || q == GZ_ESKETCH_FAIL ? gst[i] : q;
            if (k->labels && (q == GZ_OK || q == GZ_ESKETCH_FAIL))
                std::memcpy(k->labels, lab + off[i], 4ull * k->sess->V);
            k->res.done_ns = done;
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (gz_ticket* k : batch) {
                gz_session* s = k->sess;
                S->stats.queries++;
                k->res.admit_ns = s->admit_ns;
                if (s->gstatus) k->res.status = s->gstatus;  // some of its updates failed
                k->done = true;
                s->inflight -= 1;
                s->query_busy = false;
                S->queries_running--;
            }
            S->stats.query_runs++;
            S->cv_done.notify_all();
        }
        S->cv_work.notify_one();
    }
    hipHostFree(lab);
}

// grow a tick buffer set to hold n updates in `pieces` gather pieces
gz_status ensure_tick_buffers(gz_server* S, int buf, uint64_t n, uint64_t pieces) {
    if (S->stage_cap[buf] < n) {
        hipFree(S->d_stage[buf]);
        S->d_stage[buf] = nullptr;
        S->stage_cap[buf] = 0;
        const uint64_t cap = std::max<uint64_t>(n + n / 2, 1u << 20);
        GZ_HIP(hipMalloc((void**)&S->d_stage[buf], 8 * cap));
        S->stage_cap[buf] = cap;
    }
    if (S->pieces_cap[buf] < pieces) {
        hipFree(S->d_pieces[buf]);
        hipHostFree(S->h_pieces[buf]);
        S->d_pieces[buf] = nullptr;
        S->h_pieces[buf] = nullptr;
        S->pieces_cap[buf] = 0;
        const uint64_t cap = std::max<uint64_t>(pieces + pieces / 2, 1024);
        GZ_HIP(hipMalloc((void**)&S->d_pieces[buf], cap * sizeof(GatherPiece)));
        GZ_HIP(hipHostMalloc((void**)&S->h_pieces[buf], cap * sizeof(GatherPiece),
                             hipHostMallocDefault));
        S->pieces_cap[buf] = cap;
    }
    return GZ_OK;
}

// One gather kernel moves the tick's batches into their sessions' gutters
// and, session after session, the flushed gutters' content and the batches
// staged behind it into the staging arrays of `buf`; then the fused ingest
// over the sessions whose sketches the tick updates.
gz_status launch_tick(gz_server* S, Tick& t, int buf) {
    auto npieces = [](uint64_t n) { return (n + kGatherPiece - 1) / kGatherPiece; };
    uint64_t pieces = 0;
    for (size_t i = 0; i < t.upd_sessions.size(); ++i) {
        pieces += npieces(t.flushed[i]);
        for (gz_ticket* k : t.upd[i]) pieces += npieces(k->n);
    }
    for (auto& kp : t.gut) pieces += npieces(kp.first->n);
    GZ_TRY(ensure_tick_buffers(S, buf, t.ingested, pieces));
    uint32_t* dsrc = S->d_stage[buf];
    uint32_t* ddst = dsrc + S->stage_cap[buf];
    GatherPiece* hp = S->h_pieces[buf];
    uint64_t np = 0;
    auto add = [&](const uint32_t* a, const uint32_t* b, uint32_t* oa, uint32_t* ob, uint64_t n) {
        for (uint64_t o = 0; o < n; o += kGatherPiece)
            hp[np++] = GatherPiece{a + o, b + o, oa + o, ob + o,
                                   (uint32_t)std::min<uint64_t>(kGatherPiece, n - o), 0};
    };
    std::vector<gz_graph*> gs;
    std::vector<uint64_t> offs(1, 0);
    uint64_t at = 0;
    const uint64_t start = now_ns();
    for (size_t i = 0; i < t.upd_sessions.size(); ++i) {
        gz_session* s = t.upd_sessions[i];
        gs.push_back(s->g);
        add(s->gut, s->gut + s->gcap, dsrc + at, ddst + at, t.flushed[i]);
        at += t.flushed[i];
        for (gz_ticket* k : t.upd[i]) {
            add(k->src, k->dst, dsrc + at, ddst + at, k->n);
            at += k->n;
            k->res.start_ns = start;
        }
        offs.push_back(at);
    }
    for (auto& kp : t.gut) {
        gz_ticket* k = kp.first;
        gz_session* s = k->sess;
        add(k->src, k->dst, s->gut + kp.second, s->gut + s->gcap + kp.second, k->n);
        k->res.start_ns = start;
    }
    if (np)
        GZ_HIP(hipMemcpyAsync(S->d_pieces[buf], hp, np * sizeof(GatherPiece),
                              hipMemcpyHostToDevice, S->stream));
    GZ_HIP(hipEventRecord(S->tick_t0[buf], S->stream));
    if (np) {
        k_srv_gather<<<(uint32_t)np, kGatherThreads, 0, S->stream>>>(S->d_pieces[buf]);
        GZ_HIP(hipGetLastError());
    }
    if (!gs.empty())
        GZ_TRY(gz_ingest_multi(gs.data(), (uint32_t)gs.size(), offs.data(), dsrc, ddst,
                               GZ_ASYNC | GZ_DEVICE_PTR, S->stream));
    GZ_HIP(hipEventRecord(S->tick_t1[buf], S->stream));
    GZ_HIP(hipEventRecord(S->stage_ev[buf], S->stream));
    std::lock_guard<std::mutex> lk(S->mu);
    S->stats.staged_bytes += 8 * t.n;
    return GZ_OK;
}

// the tick's requests are done: its batches complete, and its sessions' gutter
// ingests are no longer in flight (a failed one is reported by their queries)
void finish_tick(gz_server* S, Tick& t, gz_status st) {
    for (size_t i = 0; i < t.upd_sessions.size(); ++i) {
        t.upd_sessions[i]->g->pending_error = false;
        for (gz_ticket* k : t.upd[i]) {
            S->pool.give(k->pinned, k->pinned_cap);  // the gather has read it
            k->pinned = nullptr;
            complete(S, k, st);
        }
    }
    for (auto& kp : t.gut) {
        S->pool.give(kp.first->pinned, kp.first->pinned_cap);
        kp.first->pinned = nullptr;
        complete(S, kp.first, st);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t i = 0; i < t.upd_sessions.size(); ++i) {
        gz_session* s = t.upd_sessions[i];
        s->ingests_inflight -= 1;
        if (st && !s->gstatus) s->gstatus = st;
    }
    if (st) {
        for (auto& kp : t.gut)
            if (!kp.first->sess->gstatus) kp.first->sess->gstatus = st;
    }
    S->cv_done.notify_all();  // gz_session_graph may wait for a flush
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
            if (prev.buf < 0)
                S->cv_work.wait(lk, [&] {
                    return (S->stop && S->queries_running == 0) || has_work(S);
                });
            if (S->stop && !has_work(S) && prev.buf < 0 && S->queries_running == 0) break;
            take_tick(S, t);
        }
        t.take_ns = now_ns();
        // 1. launch this tick's gather and fused ingest (async)
        gz_status st = GZ_OK;
        const bool launch = !t.upd_sessions.empty() || !t.gut.empty();
        if (launch) {
            const uint64_t t0 = now_ns();
            hipEventSynchronize(S->stage_ev[buf]);  // tick t-2's ingest is done with buf
            const uint64_t t1 = now_ns();
            st = launch_tick(S, t, buf);
            const uint64_t t2 = now_ns();
            t.launched_ns = t2;
            std::lock_guard<std::mutex> lk(S->mu);
            S->stats.worker_wait_ns += t1 - t0;
            S->stats.worker_launch_ns += t2 - t1;
            if (!st) {
                S->stats.ticks++;
                S->stats.updates += t.n;
                S->stats.ingested += t.ingested;
                for (uint64_t f : t.flushed) S->stats.flushes += f > 0;
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
            {
                gz_tick_record rec{};
                rec.take_ns = prev.tick.take_ns;
                rec.launched_ns = prev.tick.launched_ns;
                rec.done_ns = now_ns();
                rec.updates = prev.tick.n;
                rec.ingested = prev.tick.ingested;
                rec.batches = prev.tick.batches;
                rec.graphs = (uint32_t)prev.tick.upd_sessions.size();
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, S->tick_t0[prev.buf], S->tick_t1[prev.buf]) ==
                    hipSuccess)
                    rec.device_ms = ms;
                std::lock_guard<std::mutex> lk(S->mu);
                if (S->timeline.size() < kTimelineCap) S->timeline.push_back(rec);
            }
            // Every batch was validated when it was submitted, so the ingest
            // cannot have met an invalid update: its completion is all that is
            // left to wait for, and the graphs need no flush-time error check
            // (two synchronous device reads per session, most of a tick's time
            // when a tick holds dozens of sessions).  No query of these
            // sessions runs until their ingests complete.
            finish_tick(S, prev.tick, pst);
            prev = Pending{};
        }
        if (launch) {
            if (st) {
                hipStreamSynchronize(S->stream);  // nothing of the tick may still read them
                finish_tick(S, t, st);
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
        hipStreamCreateWithFlags(&S->vstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->stage_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&S->stage_ev[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&S->tick_t0[0]) != hipSuccess || hipEventCreate(&S->tick_t0[1]) != hipSuccess ||
        hipEventCreate(&S->tick_t1[0]) != hipSuccess || hipEventCreate(&S->tick_t1[1]) != hipSuccess ||
        hipHostMalloc((void**)&S->vflag, 4, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess) {
        if (S->stream) hipStreamDestroy(S->stream);
        if (S->vstream) hipStreamDestroy(S->vstream);
        for (hipEvent_t e : {S->stage_ev[0], S->stage_ev[1], S->tick_t0[0], S->tick_t0[1],
                             S->tick_t1[0], S->tick_t1[1]})
            if (e) hipEventDestroy(e);
        delete S;
        return gz::fail(GZ_EDEVICE, "server streams/events");
    }
    // both staging sets start "free": their events are complete
    hipEventRecord(S->stage_ev[0], S->stream);
    hipEventRecord(S->stage_ev[1], S->stream);
    S->budget = hbm_budget;
    S->tick_cap = tick_updates ? tick_updates : (16ull << 20);
    S->arena.init(hbm_budget);  // best effort: without it each graph allocates its own
    S->stats.hbm_budget = hbm_budget;
    S->worker = std::thread(worker_main, S);
    S->admitter = std::thread(admit_main, S);
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
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->gutter_per_node && S->arena.active())
            s->gcap = std::max<uint64_t>((uint64_t)S->gutter_per_node * V, kGutterMin);
    }
    s->bytes = session_bytes(V) + 8 * s->gcap;
    if (s->bytes > S->budget) {
        delete s;
        return gz::fail(GZ_ENOMEM, "session larger than the whole HBM budget");
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        s->wait_since = now_ns();
        S->waiting.push_back(s);
    }
    S->cv_admit.notify_one();
    *out = s;
    return GZ_OK;
}

static gz_status submit(gz_session* s, gz_ticket* k, gz_ticket** out) {
    gz_server* S = s->srv;
    k->sess = s;
    k->srv = S;
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
    gz_ticket* k = new gz_ticket();
    k->kind = gz_ticket::UPDATES;
    k->n = N;
    k->res.updates = N;
    if (N) {
        // one pass: validate while copying into a pinned buffer the gather reads
        k->pinned = s->srv->pool.take(8 * N, &k->pinned_cap);
        if (!k->pinned) {
            delete k;
            return gz::fail(GZ_ENOMEM, "pinned staging of a batch");
        }
        uint32_t* ps = k->pinned;
        uint32_t* pd = k->pinned + N;
        const uint32_t V = s->V;
        uint32_t bad = 0;
        for (uint64_t i = 0; i < N; ++i) {
            const uint32_t a = src[i], b = dst[i];
            bad |= (uint32_t)(a == b) | (uint32_t)(a >= V) | (uint32_t)(b >= V);
            ps[i] = a;
            pd[i] = b;
        }
        uint32_t* dev = nullptr;
        const hipError_t e = bad ? hipSuccess : hipHostGetDevicePointer((void**)&dev, ps, 0);
        if (bad || e != hipSuccess) {
            s->srv->pool.give(k->pinned, k->pinned_cap);
            delete k;
            if (e != hipSuccess) return gz::hip_fail(e, "device address of a pinned batch");
            return gz::fail(GZ_EINVAL, "invalid update (self-loop or node id out of range)");
        }
        k->src = dev;
        k->dst = dev + N;
    }
    {
        std::lock_guard<std::mutex> lk(s->srv->mu);
        s->srv->stats.batches_copied++;
    }
    return submit(s, k, out);
}

// where an in-place array lies: its device-readable address, and whether the
// host can read it (pinned host memory) or only the device
static gz_status locate(gz_server* S, const uint32_t* p, const uint32_t** dev, bool* host) {
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return gz::fail(GZ_EINVAL, "in-place batches must be device or pinned host memory");
    }
    if (at.type == hipMemoryTypeHost && at.devicePointer) {
        // the address may point into the middle of the allocation
        *dev = static_cast<const uint32_t*>(at.devicePointer);
        *host = true;
        return GZ_OK;
    }
    if (at.type == hipMemoryTypeDevice && at.device == S->device) {
        *dev = p;
        *host = false;
        return GZ_OK;
    }
    return gz::fail(GZ_EINVAL, "in-place batches must be device memory of the server's GPU "
                               "or pinned host memory");
}

gz_status gz_submit_updates_inplace(gz_session* s, const uint32_t* src, const uint32_t* dst,
                                    uint64_t N, gz_ticket** out) {
    if (!s || !out || (N && (!src || !dst))) return gz::fail(GZ_EINVAL, "null argument");
    *out = nullptr;
    gz_server* S = s->srv;
    gz_ticket* k = new gz_ticket();
    k->kind = gz_ticket::UPDATES;
    k->n = N;
    k->res.updates = N;
    if (N) {
        const uint32_t *ds = nullptr, *dd = nullptr;
        bool hs = false, hd = false;
        gz_status st = locate(S, src, &ds, &hs);
        if (!st) st = locate(S, dst, &dd, &hd);
        if (st) {
            delete k;
            return st;
        }
        uint32_t bad = 0;
        const uint32_t V = s->V;
        if (hs && hd) {
            for (uint64_t i = 0; i < N; ++i) {
                const uint32_t a = src[i], b = dst[i];
                bad |= (uint32_t)(a == b) | (uint32_t)(a >= V) | (uint32_t)(b >= V);
            }
        } else {
            // device memory (or one array of each kind): checked by a kernel
            std::lock_guard<std::mutex> lk(S->vmu);
            uint32_t* flag_dev = nullptr;
            volatile uint32_t* flag = S->vflag;
            *flag = 0;
            hipError_t e = hipHostGetDevicePointer((void**)&flag_dev, S->vflag, 0);
            if (e == hipSuccess) {
                const uint64_t blocks = std::min<uint64_t>((N + 255) / 256, 1024);
                k_srv_validate<<<(uint32_t)blocks, 256, 0, S->vstream>>>(ds, dd, N, V, flag_dev);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipStreamSynchronize(S->vstream);
            if (e != hipSuccess) {
                delete k;
                return gz::hip_fail(e, "validation of an in-place batch");
            }
            bad = *flag;
        }
        if (bad) {
            delete k;
            return gz::fail(GZ_EINVAL, "invalid update (self-loop or node id out of range)");
        }
        k->src = ds;
        k->dst = dd;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stats.batches_inplace++;
    }
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

static gz_status take_result(gz_ticket* k, gz_result* res) {
    // (a completed ticket may outlive its session: only the server is used here)
    if (k->pinned) k->srv->pool.give(k->pinned, k->pinned_cap);  // never gathered
    gz_result r = k->res;
    r.kind = k->kind == gz_ticket::QUERY ? 1u : 0u;
    if (res) *res = r;
    delete k;
    return r.status == GZ_ESKETCH_FAIL ? GZ_OK : r.status;
}

gz_status gz_wait(gz_ticket* k, gz_result* res) {
    if (!k) return gz::fail(GZ_EINVAL, "null ticket");
    gz_server* S = k->srv;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return k->done; });
    }
    return take_result(k, res);
}

gz_status gz_wait_any(gz_ticket* const* tickets, uint32_t n, uint64_t timeout_ns,
                      uint32_t* index, gz_result* res) {
    if (!tickets || !n || !index) return gz::fail(GZ_EINVAL, "null argument");
    *index = n;
    for (uint32_t i = 0; i < n; ++i)
        if (!tickets[i]) return gz::fail(GZ_EINVAL, "null ticket");
    gz_server* S = tickets[0]->srv;
    for (uint32_t i = 1; i < n; ++i)
        if (tickets[i]->srv != S) return gz::fail(GZ_EINVAL, "tickets of several servers");
    uint32_t found = n;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        auto any_done = [&] {
            for (uint32_t i = 0; i < n; ++i)
                if (tickets[i]->done) {
                    found = i;
                    return true;
                }
            return false;
        };
        if (timeout_ns == UINT64_MAX)
            S->cv_done.wait(lk, any_done);
        else
            S->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), any_done);
    }
    if (found == n) return gz::fail(GZ_ETIMEOUT, "no ticket completed within the timeout");
    *index = found;
    return take_result(tickets[found], res);
}

gz_status gz_session_graph(gz_session* s, gz_graph** out) {
    if (!s || !out) return gz::fail(GZ_EINVAL, "null argument");
    gz_server* S = s->srv;
    std::unique_lock<std::mutex> lk(S->mu);
    *out = s->g;
    if (!s->g) return gz::fail(GZ_ESTATE, "session not admitted yet");
    if (!s->queue.empty() || s->inflight)
        return gz::fail(GZ_ESTATE, "the session has requests in flight");
    if (s->gfill || s->ingests_inflight) {
        // the sketches hold every batch once the gutter is applied
        s->flush_req = true;
        S->cv_work.notify_one();
        S->cv_done.wait(lk, [&] { return s->gfill == 0 && s->ingests_inflight == 0; });
        s->flush_req = false;
    }
    if (s->gstatus) return gz::fail(s->gstatus, "an ingest of the session's updates failed");
    return GZ_OK;
}

gz_status gz_server_set_gutter(gz_server* S, uint32_t updates_per_node) {
    if (!S) return gz::fail(GZ_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    S->gutter_per_node = updates_per_node;
    return GZ_OK;
}

gz_status gz_session_close(gz_session* s) {
    if (!s) return GZ_OK;
    gz_server* S = s->srv;
    std::unique_lock<std::mutex> lk(S->mu);
    s->closing = true;
    S->cv_done.wait(lk, [&] { return !s->admitting; });
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
    // (updates still in its gutter are dropped with the session)
    S->cv_done.wait(lk, [&] {
        return s->queue.empty() && s->inflight == 0 && !s->query_busy && s->ingests_inflight == 0;
    });
    auto it = std::find(S->admitted.begin(), S->admitted.end(), s);
    const bool held = it != S->admitted.end();
    if (held) S->admitted.erase(it);
    auto wt = std::find(S->waiting.begin(), S->waiting.end(), s);
    if (wt != S->waiting.end()) S->waiting.erase(wt);
    gz_graph* g = s->g;
    lk.unlock();
    const uint64_t t0 = now_ns();
    gz_free(g);
    const uint64_t dt = now_ns() - t0;
    lk.lock();
    S->stats.free_ns += dt;
    S->stats.free_ns_max = std::max(S->stats.free_ns_max, dt);
    S->arena.give(s->storage, arena_bytes(s->V, s->gcap));
    s->storage = nullptr;
    s->gut = nullptr;
    if (held) S->used -= s->bytes;  // the memory is free now: waiting sessions may go
    lk.unlock();
    delete s;
    S->cv_admit.notify_one();
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

gz_status gz_server_timeline(gz_server* S, gz_tick_record* out, uint64_t cap, uint64_t* n) {
    if (!S || !n || (cap && !out)) return gz::fail(GZ_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *n = S->timeline.size();
    std::copy(S->timeline.begin(), S->timeline.begin() + std::min<uint64_t>(cap, *n), out);
    return GZ_OK;
}

gz_status gz_server_destroy(gz_server* S) {
    if (!S) return GZ_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop_admit = true;
    }
    S->cv_admit.notify_one();
    S->admitter.join();
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
        for (gz_ticket* k : s->queue) {
            S->pool.give(k->pinned, k->pinned_cap);
            delete k;
        }
        gz_free(s->g);
        delete s;
    }
    for (int b = 0; b < 2; ++b) {
        if (S->stage_ev[b]) {
            hipEventSynchronize(S->stage_ev[b]);
            hipEventDestroy(S->stage_ev[b]);
        }
        hipEventDestroy(S->tick_t0[b]);
        hipEventDestroy(S->tick_t1[b]);
        hipFree(S->d_stage[b]);
        hipFree(S->d_pieces[b]);
        hipHostFree(S->h_pieces[b]);
    }
    S->pool.release_all();
    S->arena.release();
    hipHostFree(S->vflag);
    hipStreamDestroy(S->vstream);
    hipStreamDestroy(S->stream);
    delete S;
    return GZ_OK;
}

}  // extern "C"
