// C-ABI entry points: graph lifecycle, seeds, export, status reporting.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gz_device.h"
#include "gz_internal.h"

namespace gz {

namespace {
thread_local std::string g_last_error;

uint32_t bitlen64(uint64_t x) {
    uint32_t n = 0;
    while (x) { ++n; x >>= 1; }
    return n;
}

// the pair-keyed form of wide graphs: ((a*u + a2*v + b) mod 2^64) >> 32
uint32_t host_hash_pair(uint64_t a, uint64_t a2, uint64_t b, uint32_t u, uint32_t v) {
    return (uint32_t)((a * u + a2 * v + b) >> 32);
}

uint32_t host_hash(uint64_t mult, uint64_t incr, uint64_t x) {
    return (uint32_t)((mult * x + incr) >> 32);
}
}  // namespace

// Graph memory comes from the device's stream-ordered pool where the device
// has one (memory freed into it is kept for later graphs): freeing a graph then
// costs no wait for the rest of the device's work, whereas hipFree waits for
// the whole device, which stalls every other stream of a serving process each
// time a session ends.
namespace {
struct PoolState {
    std::once_flag once;
    bool ok = false;
};
bool use_pool(int dev) {
    static PoolState* states = new PoolState[64];  // never freed: used until exit
    PoolState& ps = states[(unsigned)dev % 64];
    std::call_once(ps.once, [&] {
        int v = 0;
        hipMemPool_t pool = nullptr;
        uint64_t keep = UINT64_MAX;
        ps.ok = hipDeviceGetAttribute(&v, hipDeviceAttributeMemoryPoolsSupported, dev) ==
                    hipSuccess &&
                v && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess &&
                hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) == hipSuccess;
        (void)hipGetLastError();
    });
    return ps.ok;
}

hipError_t graph_alloc(const gz_graph* g, void** p, size_t bytes, hipStream_t s) {
    return use_pool(g->device) ? hipMallocAsync(p, bytes, s) : hipMalloc(p, bytes);
}

// after every use of p is complete (the caller has waited for the graph's work)
void graph_release(const gz_graph* g, void* p, hipStream_t s) {
    if (!p) return;
    if (use_pool(g->device)) hipFreeAsync(p, s);
    else hipFree(p);
}
}  // namespace


// the graph's query stream, created on first use (many-graph sets never query
// most graphs one by one)
hipError_t query_stream(gz_graph* g, hipStream_t* out) {
    if (!g->qstream) {
        hipError_t e = hipStreamCreateWithFlags(&g->qstream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            g->qstream = nullptr;
            return e;
        }
    }
    *out = g->qstream;
    return hipSuccess;
}

// Error words of graphs live in pinned, coherent host memory that kernels write
// directly, so that gz_flush reads a graph's word without a device copy (a
// flush over thousands of graphs of one fused call then costs no transfers).
// Slabs of kErrSlab words are taken per device on demand; a slab is released
// when its last graph is freed.  The registry itself is never destroyed, so no
// HIP call runs from a static destructor at exit.
namespace {
constexpr uint32_t kErrSlab = 1024;
struct ErrSlab {
    int device;
    uint32_t* host;
    uint32_t* dev;
    std::vector<uint32_t> free_slots;
};
std::mutex& err_mutex() {
    static std::mutex* m = new std::mutex();
    return *m;
}
std::vector<ErrSlab*>& err_slabs() {
    static std::vector<ErrSlab*>* v = new std::vector<ErrSlab*>();
    return *v;
}
}  // namespace

hipError_t err_word_take(gz_graph* g) {
    std::lock_guard<std::mutex> lk(err_mutex());
    ErrSlab* slab = nullptr;
    for (ErrSlab* s : err_slabs())
        if (s->device == g->device && !s->free_slots.empty()) {
            slab = s;
            break;
        }
    if (!slab) {
        uint32_t* host = nullptr;
        hipError_t e = hipHostMalloc((void**)&host, kErrSlab * 4,
                                     hipHostMallocMapped | hipHostMallocCoherent);
        if (e != hipSuccess) return e;
        uint32_t* dev = nullptr;
        e = hipHostGetDevicePointer((void**)&dev, host, 0);
        if (e != hipSuccess) {
            hipHostFree(host);
            return e;
        }
        std::memset(host, 0, kErrSlab * 4);
        slab = new ErrSlab{g->device, host, dev, {}};
        for (uint32_t k = kErrSlab; k-- > 0;) slab->free_slots.push_back(k);
        err_slabs().push_back(slab);
    }
    const uint32_t k = slab->free_slots.back();
    slab->free_slots.pop_back();
    slab->host[k] = 0;
    g->err_slab = slab;
    g->err_host = slab->host + k;
    g->err = slab->dev + k;
    return hipSuccess;
}

void err_word_release(gz_graph* g) {
    if (!g->err_slab) return;
    std::lock_guard<std::mutex> lk(err_mutex());
    ErrSlab* slab = static_cast<ErrSlab*>(g->err_slab);
    slab->free_slots.push_back((uint32_t)(g->err_host - slab->host));
    g->err_slab = nullptr;
    g->err_host = g->err = nullptr;
    if (slab->free_slots.size() == kErrSlab) {
        auto& v = err_slabs();
        v.erase(std::find(v.begin(), v.end(), slab));
        hipHostFree(slab->host);
        delete slab;
    }
}

gz_status fail(gz_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

gz_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? GZ_ENOMEM : GZ_EDEVICE;
}

int device_cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (!cached[dev % 64]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        cached[dev % 64] = n;
    }
    return cached[dev % 64];
}

hipError_t fence_wait(hipStream_t stream, gz_graph* const* gs, uint32_t G) {
    const Fence* prev = nullptr;
    std::vector<const Fence*> seen;
    for (uint32_t k = 0; k < G; ++k) {
        const Fence* f = gs[k]->last.get();
        if (!f || f == prev) continue;
        prev = f;
        if (G > 1) {
            if (std::find(seen.begin(), seen.end(), f) != seen.end()) continue;
            if (seen.size() < 64) seen.push_back(f);
        }
        hipError_t e = hipStreamWaitEvent(stream, f->ev, 0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fence_record(hipStream_t stream, gz_graph* const* gs, uint32_t G) {
    if (G == 1 && gs[0]->last && gs[0]->last.use_count() == 1)
        return hipEventRecord(gs[0]->last->ev, stream);  // sole owner: reuse the event
    FenceRef f = std::make_shared<Fence>();
    hipError_t e = hipEventCreateWithFlags(&f->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(f->ev, stream);
    if (e != hipSuccess) return e;
    for (uint32_t k = 0; k < G; ++k) gs[k]->last = f;
    return hipSuccess;
}

// Defaults before autotuning: the whole tile in LDS when it takes at most 48 KiB,
// the workgroup (multiple of 64, 256..512 lanes) with the best lane use for P
// pairs, and as many resident workgroups per CU as 160 KiB of LDS allows.
gz_tuning default_tuning(uint32_t P, uint32_t B, bool wide) {
    gz_tuning t{};
    t.chunk = 16384;
    t.lds_rows = (B * tile_row_words(P, wide) * 4 <= 48 * 1024) ? B : std::min<uint32_t>(B, 15u);
    uint32_t best = 0;
    double best_use = -1.0;
    for (uint32_t wg = 256; wg <= 512; wg += 64) {
        if (wg < P) continue;
        const double use = (double)((wg / P) * P) / wg;
        if (use > best_use + 0.01) {
            best_use = use;
            best = wg;
        }
    }
    t.wg_size = best ? best : std::min<uint32_t>(1024, (P + 63) / 64 * 64);
    const uint32_t smem = (uint32_t)update_smem_bytes(t.lds_rows, B, P, wide);
    t.wgs_per_cu = std::max<uint32_t>(1, std::min<uint32_t>(8, (160 * 1024) / smem));
    t.group_blocks = 0;
    t.node_chunk = 0;
    return t;
}

// exact-depth rows -> nested rows (row b = XOR of rows d >= b), widened to 64 bits
// (sk holds the node blocks from node `first` on; `planes` = 4 for wide
// graphs, whose alpha has a low and a high word)
__global__ void k_export(const uint32_t* __restrict__ sk, uint32_t first, uint32_t lo, uint32_t hi,
                         uint32_t R, uint32_t B, uint32_t P, uint32_t planes,
                         uint64_t* __restrict__ alpha, uint64_t* __restrict__ gamma) {
    const uint64_t total = (uint64_t)(hi - lo) * P;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = lo + (uint32_t)(t / P);
        const uint32_t p = (uint32_t)(t % P);  // p = r * C + c
        const uint32_t* base = sk + (uint64_t)(v - first) * planes * B * P +
                               sk_word_n(planes, B, p / kC, 0, 0, p % kC);
        const uint64_t out0 = (t / P) * (uint64_t)R * kC * B + (uint64_t)p * B;
        const uint32_t pg = planes - 2;  // first gamma plane
        uint32_t a = 0, ah = 0, gl = 0, gh = 0;
        for (int b = (int)B - 1; b >= 0; --b) {
            const uint32_t* row = base + b * planes * kC;  // row b of the round, column c
            a ^= row[0];
            if (planes == kPlanesWide) ah ^= row[kC];
            gl ^= row[pg * kC];
            gh ^= row[(pg + 1) * kC];
            alpha[out0 + b] = ((uint64_t)ah << 32) | a;
            gamma[out0 + b] = ((uint64_t)gh << 32) | gl;
        }
    }
}

gz_status export_nested(gz_graph* g, uint32_t lo, uint32_t hi, uint64_t* alpha, uint64_t* gamma) {
    const uint64_t n = (uint64_t)(hi - lo) * g->R * kC * g->B;
    if (n == 0) return GZ_OK;
    uint64_t *da = nullptr, *dg = nullptr;
    GZ_HIP(hipMalloc((void**)&da, n * 8));
    if (hipMalloc((void**)&dg, n * 8) != hipSuccess) {
        hipFree(da);
        return fail(GZ_ENOMEM, "export buffer");
    }
    hipStream_t s = nullptr;
    hipError_t e = query_stream(g, &s);
    if (e == hipSuccess) e = fence_wait(s, g);
    const uint32_t* src = g->sk;
    uint32_t first = 0;
    uint32_t* fetched = nullptr;
    if (e == hipSuccess && g->tier) {  // the host tier's blocks come in through a device copy
        const gz_status fs = tier_fetch(g, lo, hi, s, &fetched);
        if (fs != GZ_OK) {
            hipFree(da);
            hipFree(dg);
            return fs;
        }
        src = fetched;
        first = lo;
    }
    if (e == hipSuccess) {
        const uint64_t total = (uint64_t)(hi - lo) * g->P;
        const uint32_t blocks = (uint32_t)std::min<uint64_t>((total + 255) / 256, 65535);
        k_export<<<blocks, 256, 0, s>>>(src, first, lo, hi, g->R, g->B, g->P, g->planes, da, dg);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(alpha, da, n * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(gamma, dg, n * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(fetched);
    hipFree(da);
    hipFree(dg);
    if (e != hipSuccess) return hip_fail(e, "export");
    return GZ_OK;
}

gz_status init_graph(gz_graph** out, uint32_t V, uint64_t seed, const gz_config* cfg) {
    if (!out) return fail(GZ_EINVAL, "null output handle");
    *out = nullptr;
    if (V < 2 || V > GZ_MAX_NODES_WIDE) return fail(GZ_EINVAL, "V must be in [2, 2^24]");
    gz_graph* g = new gz_graph();
    GZ_HIP(hipGetDevice(&g->device));
    g->V = V;
    g->n = (uint64_t)V * (V - 1) / 2;
    g->R = bitlen64((uint64_t)V - 1) + 1;
    g->C = kC;
    // B = ceil(log2 n) + 1 rows; graphs with V > 2^16 have n > 2^31 and a 64-bit row hash
    g->B = bitlen64(g->n - 1) + 1;
    g->wide = V > kMaxNarrow;
    g->planes = g->wide ? kPlanesWide : kPlanes;
    if (cfg && cfg->rounds) g->R = cfg->rounds;
    if (g->R > 64) {
        delete g;
        return fail(GZ_EINVAL, "too many rounds");
    }
    g->P = g->R * kC;
    g->seed = seed;
    // seeds: SplitMix64 stream in (round, column, hash) order; per hash a
    // multiplier then an increment, or for wide graphs a, a2 then b for four
    // hashes (row low word, checksum high, checksum low, row high word)
    const uint32_t per_pair = g->wide ? 3 * kWideHashes : 6;
    g->seeds_host.resize((size_t)g->P * per_pair);
    uint64_t st = seed;
    for (uint32_t p = 0; p < g->P; ++p)
        for (uint32_t k = 0; k < per_pair; ++k)
            g->seeds_host[(size_t)p * per_pair + k] = splitmix64_next(st);
    for (uint32_t p = 0; p < g->P; ++p) {
        const uint64_t* s = &g->seeds_host[(size_t)p * per_pair];
        // edge 0 = pair (0, 1) must keep a non-zero checksum
        const uint64_t chk0 =
            g->wide ? ((uint64_t)host_hash_pair(s[3], s[4], s[5], 0, 1) << 32) |
                          host_hash_pair(s[6], s[7], s[8], 0, 1)
                    : ((uint64_t)host_hash(s[2], s[3], 0) << 32) | host_hash(s[4], s[5], 0);
        if (chk0 == 0) {
            delete g;
            return fail(GZ_EINVAL, "seed gives a zero checksum for index 0; pick another seed");
        }
    }
    // device table: word w of pair p at [w * P + p] (the 64-bit seeds split in halves)
    const uint32_t words = 2 * per_pair;
    std::vector<uint32_t> soa((size_t)words * g->P);
    for (uint32_t p = 0; p < g->P; ++p) {
        const uint64_t* s = &g->seeds_host[(size_t)p * per_pair];
        for (uint32_t k = 0; k < per_pair; ++k) {
            soa[(size_t)(2 * k) * g->P + p] = (uint32_t)s[k];
            soa[(size_t)(2 * k + 1) * g->P + p] = (uint32_t)(s[k] >> 32);
        }
    }
    g->sk_words = (uint64_t)V * g->planes * g->B * g->P;
    const uint32_t tier = cfg ? cfg->tier : GZ_TIER_HBM;
    if (tier > GZ_TIER_HOST) {
        delete g;
        return fail(GZ_EINVAL, "unknown sketch tier");
    }
    // set-up work goes on the graph's own stream and waits for that stream only,
    // so that creating a graph does not wait for other work on the device
    hipStream_t is = nullptr;
    hipError_t e = query_stream(g, &is);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "graph stream");
    }
    if (tier == GZ_TIER_HBM && cfg && cfg->storage) {
        if (cfg->storage_bytes < g->sk_words * 4 || ((uintptr_t)cfg->storage & 255)) {
            hipStreamDestroy(is);
            delete g;
            return fail(GZ_EINVAL, "sketch storage too small or not 256-byte aligned");
        }
        g->sk = static_cast<uint32_t*>(cfg->storage);
        g->sk_owned = false;
    } else if (tier == GZ_TIER_HBM) {
        e = graph_alloc(g, (void**)&g->sk, g->sk_words * 4, is);
        if (e != hipSuccess) {
            hipStreamDestroy(is);
            delete g;
            return fail(GZ_ENOMEM, "out of device memory for the sketches");
        }
    }
    e = graph_alloc(g, (void**)&g->seeds, soa.size() * 4, is);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->seeds, soa.data(), soa.size() * 4, hipMemcpyHostToDevice, is);
    if (e == hipSuccess) e = err_word_take(g);
    if (e == hipSuccess && g->sk) e = zero_words(g->sk, g->sk_words, is);
    if (e == hipSuccess && tier == GZ_TIER_HOST) {
        const gz_status ts = tier_create(g, cfg->staging_bytes);
        if (ts != GZ_OK) {
            hipStreamSynchronize(is);
            tier_free(g);
            graph_release(g, g->seeds, is);
            err_word_release(g);
            hipStreamDestroy(is);
            delete g;
            return ts;
        }
    }
    if (e == hipSuccess) e = fence_record(is, g);
    if (e == hipSuccess) e = hipStreamSynchronize(is);
    if (e != hipSuccess) {
        gz_status s = hip_fail(e, "graph init");
        hipStreamSynchronize(is);
        tier_free(g);
        if (g->sk_owned) graph_release(g, g->sk, is);
        graph_release(g, g->seeds, is);
        err_word_release(g);
        hipStreamDestroy(is);
        delete g;
        return s;
    }
    g->tuning = default_tuning(g->P, g->B, g->wide);
    // locate this device's no-allocation scratch now, so that gz_ingest_noalloc
    // makes no set-up call of its own
    uint8_t* na = nullptr;
    size_t na_cap = 0;
    e = noalloc_scratch(&na, &na_cap);
    if (e != hipSuccess) {
        gz_status s = hip_fail(e, "no-allocation scratch address");
        gz_free(g);
        return s;
    }
    *out = g;
    return GZ_OK;
}

}  // namespace gz

using namespace gz;

extern "C" {

gz_status gz_sketch_init(gz_graph** out, uint32_t V, uint64_t seed, const gz_config* cfg) {
    return init_graph(out, V, seed, cfg);
}

gz_status gz_free(gz_graph* g) {
    if (!g) return GZ_OK;
    if (g->qstream) hipStreamSynchronize(g->qstream);
    if (g->last) hipEventSynchronize(g->last->ev);
    free_ingest_scratch(g->ing);
    free_query_scratch(g->q);
    tier_free(g);
    hipStream_t s = nullptr;
    if (!g->sk_owned) g->sk = nullptr;  // caller storage
    if (query_stream(g, &s) == hipSuccess) {
        graph_release(g, g->sk, s);
        graph_release(g, g->seeds, s);
    } else {
        hipFree(g->sk);
        hipFree(g->seeds);
    }
    err_word_release(g);
    for (hipEvent_t e : g->prof_ev)
        if (e) hipEventDestroy(e);
    if (g->qstream) hipStreamDestroy(g->qstream);
    delete g;
    return GZ_OK;
}

gz_status gz_profile_enable(gz_graph* g, int on) {
    if (!g) return fail(GZ_EINVAL, "null graph");
    if (on && !g->prof_ev[0])
        for (hipEvent_t& e : g->prof_ev) GZ_HIP(hipEventCreate(&e));
    g->profiling = on != 0;
    g->prof_calls = 0;
    return GZ_OK;
}

gz_status gz_profile_last(gz_graph* g, gz_profile* out) {
    if (!g || !out) return fail(GZ_EINVAL, "null argument");
    if (!g->prof_calls) return fail(GZ_ESTATE, "no profiled ingest yet");
    GZ_HIP(hipEventSynchronize(g->prof_ev[2]));
    float a = 0, b = 0, c = 0;
    GZ_HIP(hipEventElapsedTime(&a, g->prof_ev[0], g->prof_ev[1]));
    GZ_HIP(hipEventElapsedTime(&b, g->prof_ev[1], g->prof_ev[2]));
    GZ_HIP(hipEventElapsedTime(&c, g->prof_ev[0], g->prof_ev[2]));
    out->group_ms = a;
    out->update_ms = b;
    out->ingest_ms = c;
    out->calls = g->prof_calls;
    out->reserved = 0;
    return GZ_OK;
}

gz_status gz_shape(const gz_graph* g, uint32_t* V, uint32_t* R, uint32_t* C, uint32_t* B,
                   uint64_t* n) {
    if (!g) return fail(GZ_EINVAL, "null graph");
    if (V) *V = g->V;
    if (R) *R = g->R;
    if (C) *C = g->C;
    if (B) *B = g->B;
    if (n) *n = g->n;
    return GZ_OK;
}

gz_status gz_reset(gz_graph* g, hipStream_t stream) {
    if (!g) return fail(GZ_EINVAL, "null graph");
    if (g->tier) return tier_reset(g);
    GZ_HIP(fence_wait(stream, g));
    GZ_HIP(zero_words(g->sk, g->sk_words, stream));
    GZ_HIP(fence_record(stream, g));
    return GZ_OK;
}

gz_status gz_update_sketch_batch(gz_graph* g, uint32_t node, const uint32_t* nbrs, uint64_t count,
                                 uint32_t flags, hipStream_t stream) {
    if (!g) return fail(GZ_EINVAL, "null graph");
    return update_node_batch(g, node, nbrs, count, flags, stream);
}

gz_status gz_ingest(gz_graph* g, const uint32_t* src, const uint32_t* dst, const uint8_t* op,
                    uint64_t N, uint32_t flags, hipStream_t stream) {
    (void)op;  // Z2 toggles: an insertion and a deletion are the same update
    if (!g) return fail(GZ_EINVAL, "null graph");
    if (N == 0) return GZ_OK;
    gz_graph* gs[1] = {g};
    return ingest_fused(gs, 1, nullptr, src, dst, N, flags, stream, g->ing);
}

gz_status gz_ingest_multi(gz_graph* const* gs, uint32_t G, const uint64_t* offs,
                          const uint32_t* src, const uint32_t* dst, uint32_t flags,
                          hipStream_t stream) {
    if (!gs || !offs || G == 0) return fail(GZ_EINVAL, "null argument");
    if (bad_graph_list(gs, G)) return fail(GZ_EINVAL, "null graph handle or graph listed twice");
    const uint64_t N = offs[G];
    if (N == 0) return GZ_OK;
    std::unique_lock<std::mutex> lock;
    IngestScratch& S = shared_ingest_scratch(gs[0]->device, lock);
    return ingest_fused(gs, G, offs, src, dst, N, flags, stream, S);
}

gz_status gz_flush(gz_graph* g) {
    if (!g) return fail(GZ_EINVAL, "null graph");
    GZ_HIP(hipEventSynchronize(g->last->ev));
    if (g->pending_error) {
        // the graph's own word: set by every asynchronous call that included g
        // and met an invalid update, whichever graphs it also held
        g->pending_error = false;
        volatile uint32_t* w = g->err_host;  // written by the device, complete after the wait
        if (*w) {
            *w = 0;
            return fail(GZ_EINVAL, "an asynchronous update batch was invalid and skipped");
        }
    }
    return GZ_OK;
}

gz_status gz_query(gz_graph* g, uint32_t* labels, uint32_t* num_cc, uint32_t* edges,
                   uint64_t* num_edges) {
    if (!g) return fail(GZ_EINVAL, "null graph");
    gz_status st = gz_flush(g);
    if (st) return st;
    QueryResult res;
    gz_graph* gs[1] = {g};
    st = boruvka(gs, 1, edges != nullptr || num_edges != nullptr, res, labels, false);
    if (st) return st;
    if (num_cc) *num_cc = res.num_cc[0];
    if (edges) std::memcpy(edges, res.forest.data(), 4ull * res.forest.size());
    if (num_edges) *num_edges = res.forest.size() / 2;
    if (res.status[0] != GZ_OK)
        return fail(GZ_ESKETCH_FAIL, "a component was still active after the last round");
    return GZ_OK;
}

gz_status gz_connected_components(gz_graph* g, uint32_t* labels, uint32_t* num_cc) {
    if (!labels) return fail(GZ_EINVAL, "null labels");
    return gz_query(g, labels, num_cc, nullptr, nullptr);
}

gz_status gz_list_spanning_forest(gz_graph* g, uint32_t* edges, uint64_t* num_edges) {
    if (!edges || !num_edges) return fail(GZ_EINVAL, "null output");
    return gz_query(g, nullptr, nullptr, edges, num_edges);
}

gz_status gz_connected_components_multi(gz_graph* const* gs, uint32_t G, uint32_t* labels,
                                        uint32_t* num_cc, int32_t* status) {
    if (!gs || !labels || G == 0) return fail(GZ_EINVAL, "null argument");
    for (uint32_t k = 0; k < G; ++k) {
        gz_status st = gz_flush(gs[k]);
        if (st) return st;
    }
    QueryResult res;
    gz_status st = boruvka(gs, G, false, res, labels, true);
    if (st) return st;
    bool any_fail = false;
    for (uint32_t k = 0; k < G; ++k) {
        if (num_cc) num_cc[k] = res.num_cc[k];
        if (status) status[k] = res.status[k];
        any_fail |= res.status[k] != GZ_OK;
    }
    if (any_fail) return fail(GZ_ESKETCH_FAIL, "some graph still had an active component");
    return GZ_OK;
}

gz_status gz_export_sketches(gz_graph* g, uint32_t node_lo, uint32_t node_hi, uint64_t* alpha,
                             uint64_t* gamma) {
    if (!g || !alpha || !gamma) return fail(GZ_EINVAL, "null argument");
    if (node_lo > node_hi || node_hi > g->V) return fail(GZ_EINVAL, "bad node range");
    gz_status st = gz_flush(g);
    if (st) return st;
    return export_nested(g, node_lo, node_hi, alpha, gamma);
}

gz_status gz_sketch_storage(const gz_graph* g, void** dev_ptr, uint64_t* bytes) {
    if (!g) return fail(GZ_EINVAL, "null graph");
    if (dev_ptr) *dev_ptr = g->tier ? (void*)nullptr : (void*)g->sk;
    if (bytes) *bytes = g->sk_words * 4;
    return GZ_OK;
}

gz_status gz_get_tuning(const gz_graph* g, gz_tuning* t) {
    if (!g || !t) return fail(GZ_EINVAL, "null argument");
    *t = g->tuning;
    return GZ_OK;
}

gz_status gz_set_tuning(gz_graph* g, const gz_tuning* t) {
    if (!g || !t) return fail(GZ_EINVAL, "null argument");
    if (t->wg_size < 64 || t->wg_size > 1024 || t->wg_size % 64 || t->wg_size < g->P)
        return fail(GZ_EINVAL, "wg_size must be a multiple of 64 in [max(64, R*C), 1024]");
    if (t->lds_rows < 1) return fail(GZ_EINVAL, "lds_rows must be >= 1");
    if (t->chunk < 1 || t->chunk > (1u << 30)) return fail(GZ_EINVAL, "chunk must be in [1, 2^30]");
    if (t->wgs_per_cu < 1 || t->wgs_per_cu > 64) return fail(GZ_EINVAL, "wgs_per_cu in [1, 64]");
    if (t->node_chunk > (1u << 30)) return fail(GZ_EINVAL, "node_chunk must be in [0, 2^30]");
    size_t smem = update_smem_bytes(t->lds_rows, g->B, g->P, g->wide);
    if (smem > 160 * 1024) return fail(GZ_EINVAL, "LDS tile exceeds 160 KiB");
    g->tuning = *t;
    return GZ_OK;
}

const char* gz_status_str(gz_status s) {
    switch (s) {
        case GZ_OK: return "GZ_OK";
        case GZ_EINVAL: return "GZ_EINVAL";
        case GZ_ENOMEM: return "GZ_ENOMEM";
        case GZ_EDEVICE: return "GZ_EDEVICE";
        case GZ_ESKETCH_FAIL: return "GZ_ESKETCH_FAIL";
        case GZ_EBUSY: return "GZ_EBUSY";
        case GZ_ESTATE: return "GZ_ESTATE";
        case GZ_ETIMEOUT: return "GZ_ETIMEOUT";
        default: return "GZ_UNKNOWN";
    }
}

const char* gz_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
