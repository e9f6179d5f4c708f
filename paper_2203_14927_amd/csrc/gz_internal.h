// Internal types of the CubeSketch library (host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gz.h"

namespace gz {

constexpr uint32_t kC = GZ_COLUMNS;   // columns per CubeSketch
constexpr uint32_t kPlanes = 3;       // alpha, gamma low word, gamma high word
constexpr uint32_t kSeedWords = 12;   // per (round, column): 3 hashes x (mult, incr) x 2 words
constexpr uint32_t kNone = 0xFFFFFFFFu;

// Seeds are stored structure-of-arrays: word k of pair p at seeds[k * P + p].
enum SeedWord : uint32_t {
    S_ROW_MLO = 0, S_ROW_MHI, S_ROW_ILO, S_ROW_IHI,
    S_CHI_MLO, S_CHI_MHI, S_CHI_ILO, S_CHI_IHI,
    S_CLO_MLO, S_CLO_MHI, S_CLO_ILO, S_CLO_IHI
};

// Sketch words of a node (32-bit, "exact-depth" basis: row d holds the XOR of
// the indices whose depth is exactly d, so each update touches one row per
// column).  Node v owns the block sk[v * 3 * B * P ...], P = R * C, laid out
// round-major, then row by row, the planes of a row side by side: word
// ((r * B + d) * 3 + plane) * C + c.  One round's rows of a node are thus
// contiguous (3 * B * C words), which is what a Boruvka round reads, and so are
// its rows d < DL, which is what the update of a small item reads and writes.
// Planes: 0 = alpha (indices are < 2^31, the high word is always zero),
// 1 = gamma low word, 2 = gamma high word.  The nested rows of the paper are
// the suffix XORs over d >= b of this basis (a linear, invertible change).
__host__ __device__ __forceinline__ uint32_t sk_word(uint32_t B, uint32_t r, uint32_t plane,
                                                     uint32_t d, uint32_t c) {
    return ((r * B + d) * kPlanes + plane) * kC + c;
}

// Graphs with V > 2^16 ("wide") need 64-bit indices: four planes (alpha low,
// alpha high, gamma low, gamma high), the same order.
constexpr uint32_t kPlanesWide = 4;
constexpr uint32_t kMaxNarrow = 65536;
// pair-keyed hashes per (round, column) of a wide graph: row (low word),
// checksum high, checksum low, row (high word); the row hash has 64 bits
constexpr uint32_t kWideHashes = 4;
// rows the low word of a wide row hash reaches (0..32); deeper rows need its high word
constexpr uint32_t kLowRowLimit = 32;
__host__ __device__ __forceinline__ uint32_t sk_word_n(uint32_t planes, uint32_t B, uint32_t r,
                                                       uint32_t plane, uint32_t d, uint32_t c) {
    return ((r * B + d) * planes + plane) * kC + c;
}

// Row stride of an LDS node tile: P rounded up to a multiple of 64 words.
__host__ __device__ __forceinline__ uint32_t tile_stride(uint32_t P) { return (P + 63u) & ~63u; }

// Per-graph data a kernel needs; kept in a device table for fused launches.
struct GraphDesc {
    uint32_t* sk;        // node blocks from graph-local node sk_first on
    const uint32_t* seeds;
    uint64_t n;          // V(V-1)/2
    uint32_t V, R, B, P;
    uint32_t node_base;  // global id of the graph's node 0 in a fused launch
    uint32_t nb;         // grouping chunks of this graph's updates in the launch
    uint64_t upd_base;   // first update of this graph in the launch's stream
    uint64_t hoff;       // start of this graph's (node, chunk) count table
    uint32_t node_words; // words between consecutive node blocks in sk
    uint32_t round_view; // query only: sk holds one round's slab per node (stride planes*B*C)
    uint32_t wide;       // V > 2^16: pair-keyed hashes, four planes
    uint32_t planes;     // 3, or 4 when wide
    uint32_t sk_first;   // graph-local node of the first block in sk (a host-tier slab's first
                         // node; 0 when sk holds the whole graph)
    uint32_t* err;       // the graph's own error word: set when an asynchronous call that
                         // included the graph met an invalid update (read by gz_flush)
};

// One unit of work of the persistent sketch-update kernel: up to `chunk`
// endpoint entries of one node, stored contiguously in the grouped array.
struct WorkItem {
    uint32_t begin;   // first entry in the grouped index array
    uint32_t count;
    uint32_t gnode;   // global node id
    uint32_t graph;   // index into the descriptor table
    uint32_t shared;  // 1 if other items of this launch update the same node
    uint32_t split;   // wide graphs: entries [begin, begin+split) are neighbours below the
                      // node, the rest above it (set by k_split_items)
};

// One block of the grouping pass: chunk `c` of graph `g`'s updates, counted or
// scattered for the node range [q * kGroupRange, (q+1) * kGroupRange).
struct GroupUnit {
    uint32_t g, c, q, pad;
};
constexpr uint32_t kGroupRange = 32768;  // node counters per block (128 KiB of LDS)

// Arguments of a fused ingest launch sequence, read by the kernels from device
// memory so that a captured graph can be replayed on new inputs.
struct IngestArgs {
    const uint32_t* src;
    const uint32_t* dst;
    const uint64_t* offs;     // G+1 update offsets (device)
    uint64_t N;
    uint32_t G;
    uint32_t T;               // total nodes over all graphs
    uint32_t chunk;
    uint32_t lds_rows;
    uint32_t group_chunk;     // updates per grouping block
    uint32_t n_units;
    uint64_t H_size;          // entries of the (node, chunk) count table
};

// Device scratch of the ingest path, grown on demand.
struct IngestScratch {
    int device = -1;
    uint64_t cap_updates = 0;   // capacity of the grouped array (entries = 2N)
    uint32_t cap_nodes = 0;
    uint32_t cap_graphs = 0;
    uint64_t cap_items = 0;
    uint32_t* H = nullptr;          // chunk-major (chunk, node) counts, then run starts
    uint64_t cap_H = 0;
    GroupUnit* units = nullptr;
    GroupUnit* h_units = nullptr;   // pinned
    uint32_t cap_units = 0;
    uint32_t* counts = nullptr;     // T: entries per node (u32)
    uint64_t* packed = nullptr;     // T+1: scanned (entries | items << 40)
    uint64_t* block_sums = nullptr; // scan partials
    uint32_t* cursor = nullptr;     // T: first grouped slot of every node
    uint32_t* grouped = nullptr;    // 2N edge indices grouped by endpoint
    uint32_t* buckets = nullptr;    // 2N bucket entries of the two-pass placement
    uint64_t cap_buckets = 0;
    uint32_t* bbase = nullptr;      // (chunks + 1) x buckets region starts
    uint64_t cap_bbase = 0;
    WorkItem* items = nullptr;
    uint32_t* ctl = nullptr;        // [0] ticket, [1] n_items, [2] call error, [3..7] always zero
    IngestArgs* args = nullptr;
    uint64_t* offs = nullptr;       // G+1
    GraphDesc* descs = nullptr;     // G
    uint32_t* staging = nullptr;    // host-pointer inputs copied here
    uint64_t cap_staging = 0;
    // pinned host copies of the per-call tables; reused once the previous
    // call's uploads have completed (copied_ev)
    IngestArgs* h_args = nullptr;
    GraphDesc* h_descs = nullptr;
    uint64_t* h_offs = nullptr;
    uint32_t cap_h_graphs = 0;
    hipEvent_t copied_ev = nullptr;
    hipEvent_t done_ev = nullptr;   // end of the last call's kernels that used this scratch
    uint32_t* h_err = nullptr;
};

struct QueryScratch;
struct HostTier;

// sketch update kernels (gz_update.hip)
__global__ void k_update(const WorkItem* __restrict__ items, uint32_t* __restrict__ ctl,
                         const uint32_t* __restrict__ grouped, const GraphDesc* __restrict__ gd,
                         uint32_t lds_rows);
__global__ void k_update_node(const uint32_t* __restrict__ nbrs, uint32_t count, uint32_t node,
                              GraphDesc g, uint32_t lds_rows, uint32_t chunk,
                              const uint32_t* __restrict__ err);
// the same for wide graphs (grouped entries are neighbour ids, four planes)
__global__ void k_update_wide(const WorkItem* __restrict__ items, uint32_t* __restrict__ ctl,
                              const uint32_t* __restrict__ grouped,
                              const GraphDesc* __restrict__ gd, uint32_t lds_rows);
__global__ void k_update_node_wide(const uint32_t* __restrict__ nbrs, uint32_t count,
                                   uint32_t node, GraphDesc g, uint32_t lds_rows, uint32_t chunk,
                                   const uint32_t* __restrict__ err);
// orders each wide-graph work item's entries by side of the node (sets split)
__global__ void k_split_items(const uint32_t* __restrict__ ctl, WorkItem* __restrict__ items,
                              const uint32_t* __restrict__ grouped, uint32_t* __restrict__ out,
                              const GraphDesc* __restrict__ gd);
// the entries the update kernel reads after grouping: wide graphs take the
// side-ordered copy
inline const uint32_t* update_entries(const IngestScratch& S, bool wide) {
    return wide ? S.buckets : S.grouped;
}
// LDS words of one tile row of P pairs (three planes, or four in blocks of 64
// pairs)
__host__ __device__ __forceinline__ uint32_t tile_row_words(uint32_t P, bool wide) {
    const uint32_t S = tile_stride(P);
    return (wide ? kPlanesWide : kPlanes) * S;
}

// Completion marker of the last device work submitted on a graph.  One call
// over many graphs records a single marker that all of them share, so a fused
// launch over thousands of graphs records, and later waits on, one event.
struct Fence {
    hipEvent_t ev = nullptr;
    ~Fence() {
        if (ev) hipEventDestroy(ev);
    }
};
using FenceRef = std::shared_ptr<Fence>;

}  // namespace gz

struct gz_graph {
    int device = 0;
    uint32_t V = 0, R = 0, C = 0, B = 0, P = 0;
    bool wide = false;                 // V > 2^16: pair-keyed hashes, 64-bit indices
    uint32_t planes = 3;               // sketch planes per bucket (4 when wide)
    uint64_t n = 0;
    uint64_t seed = 0;
    uint32_t* sk = nullptr;            // device sketch words
    bool sk_owned = true;              // false: caller storage (gz_config.storage)
    uint64_t sk_words = 0;
    uint32_t* seeds = nullptr;         // device seeds [12][P] (18 words per pair when wide)
    // error word: set by the device when an asynchronous call that included this
    // graph met an invalid update; pinned coherent host memory (err is its device
    // address, err_host its host address), one word of a shared slab
    uint32_t* err = nullptr;
    uint32_t* err_host = nullptr;
    void* err_slab = nullptr;
    std::vector<uint64_t> seeds_host;  // [R][C][3][2]
    gz_tuning tuning{};
    hipStream_t qstream = nullptr;     // query stream
    gz::FenceRef last;                 // last submitted work on this graph
    gz::IngestScratch ing;
    gz::QueryScratch* q = nullptr;
    gz::HostTier* tier = nullptr;      // non-null: sketches live in host DRAM
    bool pending_error = false;
    // optional per-phase timing of the last ingest (gz_profile_enable)
    bool profiling = false;
    hipEvent_t prof_ev[3] = {nullptr, nullptr, nullptr};
    uint32_t prof_calls = 0;
};

namespace gz {

// zero n words of device memory with a kernel on `stream`
hipError_t zero_words(uint32_t* p, uint64_t n, hipStream_t stream);

// error reporting
gz_status fail(gz_status s, const std::string& msg);
gz_status hip_fail(hipError_t e, const char* what);
#define GZ_HIP(call)                                              \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::gz::hip_fail(e_, #call);   \
    } while (0)
// the status of a HIP call as an expression (GZ_OK on success)
#define GZ_HIP_STATUS(call) \
    ([&]() -> gz_status { hipError_t e_ = (call); \
        return e_ == hipSuccess ? GZ_OK : ::gz::hip_fail(e_, #call); }())

int device_cu_count();
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the next output of the stream
inline uint64_t splitmix64_next(uint64_t& st) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
// true if a handle is null or listed twice
inline bool bad_graph_list(gz_graph* const* gs, uint32_t G) {
    std::vector<gz_graph*> v(gs, gs + G);
    std::sort(v.begin(), v.end());
    return (!v.empty() && v[0] == nullptr) || std::adjacent_find(v.begin(), v.end()) != v.end();
}
// make `stream` wait for the last work of every listed graph (one wait per
// distinct marker), and mark the work enqueued next on `stream` as theirs
hipError_t fence_wait(hipStream_t stream, gz_graph* const* gs, uint32_t G);
hipError_t fence_record(hipStream_t stream, gz_graph* const* gs, uint32_t G);
inline hipError_t fence_wait(hipStream_t stream, gz_graph* g) { return fence_wait(stream, &g, 1); }
inline hipError_t fence_record(hipStream_t stream, gz_graph* g) {
    return fence_record(stream, &g, 1);
}
hipError_t query_stream(gz_graph* g, hipStream_t* out);
hipError_t err_word_take(gz_graph* g);
void err_word_release(gz_graph* g);
gz_tuning default_tuning(uint32_t P, uint32_t B, bool wide);

// ingest path (gz_ingest.hip)
gz_status ingest_fused(gz_graph* const* gs, uint32_t G, const uint64_t* offs_host,
                       const uint32_t* src, const uint32_t* dst, uint64_t N, uint32_t flags,
                       hipStream_t stream, IngestScratch& S);
gz_status update_node_batch(gz_graph* g, uint32_t node, const uint32_t* nbrs, uint64_t count,
                            uint32_t flags, hipStream_t stream);
// after an asynchronous call: if its error word is set, set the error word of
// every graph of the call (descs: G device descriptors)
__global__ void k_note_error(const GraphDesc* __restrict__ descs, uint32_t G,
                             const uint32_t* __restrict__ call_err);
void free_ingest_scratch(IngestScratch& S);
// gz_ingest of device arrays with every device buffer carved from `scratch`
// (cap bytes) instead of allocated; asynchronous (errors reported at flush)
gz_status ingest_noalloc(gz_graph* g, const uint32_t* src, const uint32_t* dst, uint64_t N,
                         uint32_t flags, hipStream_t stream, uint8_t* scratch, size_t cap);
// the no-allocation scratch of the current device, located once per device
hipError_t noalloc_scratch(uint8_t** ptr, size_t* cap);

// dynamic LDS of an update launch, and raising a kernel's LDS limit above 64 KiB
// LDS rows of a tile for launches that keep up to lds_rows rows of graphs with
// up to Bmax rows: every row when they fit, else lds_rows plus one sink row
// that collects entries deeper than an item's rows (applied to HBM instead)
// LDS words at the start of an update kernel's dynamic shared memory that
// stage a small work item's entries (the tile follows them)
constexpr uint32_t kItemStageWords = 512;
__host__ __device__ __forceinline__ uint32_t tile_rows(uint32_t lds_rows, uint32_t Bmax) {
    return lds_rows >= Bmax ? Bmax : lds_rows + 1;
}
size_t update_smem_bytes(uint32_t lds_rows, uint32_t Bmax, uint32_t Pmax, bool wide);
gz_status set_smem_limit(const void* fn, size_t bytes);
#define GZ_TRY(call)                  \
    do {                              \
        gz_status s_ = (call);        \
        if (s_ != GZ_OK) return s_;   \
    } while (0)

// host-DRAM sketch tier (gz_tier.hip).  The grouping of a call runs as usual;
// group_only leaves the grouped entries and the node-sorted work items of one
// graph in g->ing and reports the launch shape of the update kernel.
struct UpdateLaunch {
    uint32_t wg, grid, lds_rows;
    size_t smem;
    bool wide;
};
gz_status group_only(gz_graph* g, const uint32_t* src, const uint32_t* dst, uint64_t N,
                     uint32_t flags, hipStream_t stream, UpdateLaunch* out);
gz_status tier_create(gz_graph* g, uint64_t staging_bytes);
void tier_free(gz_graph* g);
gz_status tier_ingest(gz_graph* g, const uint32_t* src, const uint32_t* dst, uint64_t N,
                      uint32_t flags, hipStream_t stream);
gz_status tier_update_node(gz_graph* g, uint32_t node, const uint32_t* nbrs, uint32_t count,
                           const uint32_t* errp, hipStream_t stream);
gz_status tier_reset(gz_graph* g);
// device copy of the node blocks [lo, hi) of a host-tier graph (caller frees)
gz_status tier_fetch(gz_graph* g, uint32_t lo, uint32_t hi, hipStream_t stream, uint32_t** out);
// round r's slab of every node into the device round buffer (query, on `stream`)
gz_status tier_round(gz_graph* g, uint32_t r, hipStream_t stream, uint32_t** round_buf);
IngestScratch& shared_ingest_scratch(int device, std::unique_lock<std::mutex>& lock);

// query path (gz_query.hip)
struct QueryResult {
    std::vector<uint32_t> num_cc;    // per graph
    std::vector<int32_t> status;     // per graph: GZ_OK / GZ_ESKETCH_FAIL
    std::vector<uint32_t> forest;    // per graph pairs, concatenated
    std::vector<uint64_t> forest_off;  // G+1 offsets into forest pairs
    uint32_t rounds = 0;
};
// labels_out (host, may be null): sum of V labels, local ids, graph after graph;
// shared_scratch: a per-device scratch set (fused calls) instead of the graph's own
gz_status boruvka(gz_graph* const* gs, uint32_t G, bool want_forest, QueryResult& out,
                  uint32_t* labels_out, bool shared_scratch);
void free_query_scratch(QueryScratch* q);

// sketch export (gz_api.hip)
gz_status export_nested(gz_graph* g, uint32_t lo, uint32_t hi, uint64_t* alpha, uint64_t* gamma);

}  // namespace gz
