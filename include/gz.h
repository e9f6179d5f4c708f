/*
 * gz.h -- C ABI of the MI355X CubeSketch connectivity library.
 *
 * The library keeps, for every node of a graph, one CubeSketch per Boruvka
 * round (GraphZeppelin, Tench et al. SIGMOD 2022: Sec. 2.2 for the node
 * sketches, Sec. 3.1 / Fig. "cube_code" for CubeSketch), resident in HBM, and
 * answers the streaming connected-components problem of Sec. 2.1: given an
 * insert/delete edge stream, return a spanning forest (and the component of
 * every node).
 *
 * Conventions shared by every call:
 *   - every call returns a gz_status; GZ_OK (0) on success;
 *   - a call that fails with GZ_EINVAL changes nothing;
 *   - gz_last_error() returns a message for the last failure on this thread;
 *   - a gz_graph handle may not be used from two host threads at once;
 *   - node ids are uint32 in [0, V); an update (u, v) needs u != v;
 *   - the sketch of a stream depends only on the set of pairs that occur an
 *     odd number of times (vectors over Z2, Sec. 3.1), so insertions and
 *     deletions are the same operation and their order does not matter;
 *   - stream arguments are hipStream_t values (0 = the null stream);
 *   - flags: GZ_DEVICE_PTR says that the array arguments point to device
 *     memory (else host memory); GZ_ASYNC skips the synchronous validation
 *     check, so an invalid update is reported by the next gz_flush instead
 *     (the offending call still applies nothing).
 *
 * Hash contract (identical for every implementation that must agree bit for
 * bit; the paper leaves the family open beyond 2-wise independence):
 *   shape   C = 8 columns, R = bitlen(V-1)+1 rounds, B = bitlen(n-1)+1 rows,
 *           n = V(V-1)/2, 2 <= V <= 65536;
 *   index   idx(u, v) = v(v-1)/2 + u for u < v (position in the
 *           characteristic vector, Sec. 2.2);
 *   seeds   a SplitMix64 stream (Steele, Lea, Flood 2014) started at the graph
 *           seed gives, for r = 0..R-1, c = 0..C-1, k in (row hash, checksum
 *           high, checksum low), a multiplier then an increment (uint64);
 *   hash    h(x) = ((mult * x + incr) mod 2^64) >> 32 (multiply-add-shift,
 *           strongly universal on 32-bit keys);
 *   depth   d = min(ctz(h_row(idx)), B-1), ctz(0) = 32: the update goes into
 *           rows 0..d of column c (row k+1 takes it while bit k of the row
 *           hash is zero, Fig. "cube_code");
 *   bucket  alpha ^= idx, gamma ^= checksum(idx) = h_hi(idx) << 32 | h_lo(idx);
 *   query   a bucket is EMPTY if alpha = gamma = 0, GOOD if not EMPTY, alpha < n
 *           and gamma = checksum(alpha), else BAD; a sketch is queried column by
 *           column, rows ascending, and yields the first GOOD alpha, else ZERO
 *           when every bucket is EMPTY, else FAIL (Sec. 3.1, result rule after
 *           Eq. (1)-(2)).
 *
 * Wide graphs (65536 < V <= 2^24): n reaches 2^47, so indices are 64-bit and a
 * hash keyed by a 32-bit index no longer covers them.  The hashes are keyed by
 * the pair instead:
 *   shape   as above (B = bitlen(n-1)+1, up to 48 rows);
 *   seeds   the same stream gives, for r = 0..R-1, c = 0..C-1 and k in (row
 *           hash low word, checksum high, checksum low, row hash high word),
 *           three words a, a2, b;
 *   hash    h(u, v) = ((a*u + a2*v + b) mod 2^64) >> 32 for u < v (strongly
 *           universal on pairs of 32-bit words);
 *   depth   d = min(ctz(h_row_hi(u, v) * 2^32 + h_row_lo(u, v)), B-1), ctz(0) = 64
 *           (a 64-bit row hash, so that rows up to log n exist for every cut
 *           size, Lemma "goodset");
 *   bucket  alpha ^= idx(u, v) (64-bit), gamma ^= h_hi(u, v) << 32 | h_lo(u, v);
 *   query   GOOD if not EMPTY, alpha < n and gamma equals the checksum of the
 *           pair alpha encodes; otherwise as above.
 */
#ifndef GZ_H
#define GZ_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gz_status;

enum {
    GZ_OK = 0,
    GZ_EINVAL = 1,        /* bad argument or invalid update; nothing applied */
    GZ_ENOMEM = 2,        /* device or host allocation failed / over budget */
    GZ_EDEVICE = 3,       /* a HIP runtime call failed */
    GZ_ESKETCH_FAIL = 4,  /* Boruvka ran out of rounds with a component still active */
    GZ_EBUSY = 5,         /* server: queue full or session not admitted yet */
    GZ_ESTATE = 6,        /* call not valid in the object's current state */
    GZ_ETIMEOUT = 7       /* server: no ticket completed within the timeout */
};

#define GZ_DEVICE_PTR 0x1u
#define GZ_ASYNC 0x2u
#define GZ_UNCHECKED 0x4u  /* caller guarantees valid ids: skip the validation launch of
                              gz_update_sketch_batch (invalid ids then corrupt only that
                              node's own sketch, never other memory) */

#define GZ_COLUMNS 8u
#define GZ_MAX_NODES 65536u         /* largest V under the index-keyed contract */
#define GZ_MAX_NODES_WIDE 16777216u /* largest V at all (2^24): pair-keyed contract */

typedef struct gz_graph gz_graph;

/* Optional overrides; zero fields keep the shape rule / library defaults. */
typedef struct gz_config {
    uint32_t rounds;        /* R override (tests force failures with a small R); 0 = rule */
    uint32_t tier;          /* GZ_TIER_HBM (0) or GZ_TIER_HOST (1) */
    uint64_t staging_bytes; /* host tier: device bytes of the two slab buffers (0 = 128 MiB) */
    void* storage;          /* HBM tier, nullable: device memory (256-byte aligned) that
                               holds the sketches instead of an allocation of the graph's
                               own; the caller keeps ownership and frees it after gz_free */
    uint64_t storage_bytes; /* its size: at least the graph's sketch bytes (gz_shape:
                               V * R * C * B * 12, or * 16 for V > 65536), else GZ_EINVAL */
} gz_config;

/* Sketch residency.  GZ_TIER_HOST keeps a graph's sketches in pinned host
 * memory (capacity beyond HBM; the paper keeps sketches on disk when they
 * outgrow RAM, Sec. 4): an ingest call is grouped on the device, then the node
 * blocks that received entries stream through two device slab buffers (copy in,
 * update, copy out, overlapped); a query copies one round of every node into
 * HBM per Boruvka round.  Results are bit-identical to GZ_TIER_HBM.  Host-tier
 * graphs take single-graph calls only (gz_ingest_multi, plans and fused
 * queries over several graphs return GZ_EINVAL for them). */
#define GZ_TIER_HBM 0u
#define GZ_TIER_HOST 1u

/* Kernel launch parameters of the ingest path; gz_autotune picks them. */
typedef struct gz_tuning {
    uint32_t wg_size;     /* threads per sketch-update workgroup (multiple of 64, <= 1024) */
    uint32_t lds_rows;    /* rows kept in the LDS tile (1..B); deeper rows go to HBM atomics */
    uint32_t chunk;       /* max updates of one node per work item (gutter split threshold) */
    uint32_t wgs_per_cu;  /* persistent grid = wgs_per_cu * CUs */
    uint32_t group_blocks;/* workgroups of the grouping passes per call (0 = one per CU) */
    uint32_t node_chunk;  /* gz_update_sketch_batch: entries per workgroup, the batch spread
                             over ceil(count / node_chunk) workgroups whose partial tiles
                             merge by XOR (0 = max(64, ceil(count / CUs)): the batch fills
                             the chip) */
} gz_tuning;

/* ------------------------------------------------------------------------
 * gz_sketch_init -- create a graph on V nodes with all-zero sketches.
 *   Paper: node sketches of O(log V) CubeSketches, one per Boruvka round
 *   (Sec. 2.2); CubeSketch layout of Sec. 3.1; all-zero start = empty graph.
 *   out   receives the handle (library-owned until gz_free);
 *   V     2 .. 2^24 (up to 65536 the index-keyed contract, above it the
 *         pair-keyed one); else GZ_EINVAL;
 *   seed  graph seed of the hash contract above;
 *   cfg   NULL or overrides.
 *   Allocates 12*B*R*C bytes per node (16*B*R*C for V > 65536) of HBM on the
 *   current device
 *   (GZ_ENOMEM if that fails).  GZ_EINVAL also if the seed yields a zero
 *   checksum for index 0 (probability 2^-64): edge (0,1) would be unsampleable.
 * ---------------------------------------------------------------------- */
gz_status gz_sketch_init(gz_graph** out, uint32_t V, uint64_t seed, const gz_config* cfg);

/* Release the graph and all its device memory.  NULL is accepted. */
gz_status gz_free(gz_graph* g);

/* Shape of the graph's sketches (any output pointer may be NULL). */
gz_status gz_shape(const gz_graph* g, uint32_t* V, uint32_t* R, uint32_t* C, uint32_t* B,
                   uint64_t* n);

/* Zero every sketch (the graph becomes empty again).  Stream-ordered on `stream`. */
gz_status gz_reset(gz_graph* g, hipStream_t stream);

/* ------------------------------------------------------------------------
 * gz_update_sketch_batch -- apply one node's batch of updates to that node's
 *   sketch only, in one kernel launch.  This is the per-node batch application
 *   of Sec. 5.1 (a Graph Worker applies a gutter of updates bound for one node
 *   to that node's CubeSketches); the mirror update of every edge must be
 *   submitted to the other endpoint by the caller.  The batch is cut into
 *   pieces of gz_tuning.node_chunk entries, one workgroup each (by default
 *   enough pieces to occupy every CU); pieces XOR their partial tiles into the
 *   node's sketch (linearity, Sec. 3.1).
 *   node   the node whose sketch changes (< V);
 *   nbrs   count neighbour ids: edge {node, nbrs[k]} is toggled in node's
 *          sketch; host or device memory (GZ_DEVICE_PTR), borrowed for the
 *          call (host memory is copied before the call returns);
 *   Errors: GZ_EINVAL if any nbrs[k] == node or >= V (nothing applied).
 *   Stream-ordered on `stream`.
 * ---------------------------------------------------------------------- */
gz_status gz_update_sketch_batch(gz_graph* g, uint32_t node, const uint32_t* nbrs, uint64_t count,
                                 uint32_t flags, hipStream_t stream);

/* ------------------------------------------------------------------------
 * gz_ingest -- apply a chunk of the edge stream: update k toggles edge
 *   {src[k], dst[k]} in the sketches of both endpoints (Sec. 2.2: each
 *   update changes both endpoints' characteristic vectors).  The updates are
 *   grouped by endpoint on the device and applied in one persistent launch
 *   (the role of the gutters of Sec. 4-5).
 *   src, dst  N node ids each, host or device memory (GZ_DEVICE_PTR);
 *             device inputs must stay valid until the stream reaches the call;
 *   op        nullable, never read: the insert/delete flag of each update
 *             (Delta = +1 / -1 of Sec. 2.1).  Over Z2 an insertion and a
 *             deletion are the same toggle (Sec. 3.1), so the sketches do not
 *             depend on it; the argument keeps the stream record's shape;
 *   N         < 2^31 per call.
 *   Errors: GZ_EINVAL if any src[k] == dst[k] or an id >= V (nothing applied).
 *   Returns after enqueueing (GZ_ASYNC) or after the validation check.
 * ---------------------------------------------------------------------- */
gz_status gz_ingest(gz_graph* g, const uint32_t* src, const uint32_t* dst, const uint8_t* op,
                    uint64_t N, uint32_t flags, hipStream_t stream);

/* ------------------------------------------------------------------------
 * gz_ingest_noalloc -- gz_ingest for callers that cannot allocate device
 *   memory: code under stream capture, tight serving loops, harnesses that
 *   forbid hipMalloc.  Same result as gz_ingest(g, src, dst, NULL, N,
 *   flags | GZ_ASYNC, stream), from the same kernels, but every device buffer
 *   of the call (grouping tables, grouped entries, work items, per-call
 *   tables) is carved from one fixed 64 MiB array that the library holds on
 *   each GPU it runs on until the process ends; the call itself allocates no
 *   device memory.
 *   src, dst  device arrays of N node ids (flags must hold GZ_DEVICE_PTR),
 *             read when the stream reaches the call;
 *   Always asynchronous: an invalid update applies nothing and is reported by
 *   g's next gz_flush.  GZ_EINVAL, applying nothing, for a host-tier graph,
 *   host arrays, or a call whose buffers exceed the 64 MiB: about 16 B per
 *   update plus 4 B per node per grouping chunk of max(8192, N / grouping
 *   blocks) updates (for V = 2^14, calls of up to about 2.5 M updates fit);
 *   split larger streams into several calls.
 *   Every call on one GPU uses that GPU's one array, which keeps the last
 *   call's contents: calls that overlap on one GPU (on different streams, or
 *   from different host threads) race and corrupt each other's results, so
 *   issue them one after another on one stream.
 * ---------------------------------------------------------------------- */
gz_status gz_ingest_noalloc(gz_graph* g, const uint32_t* src, const uint32_t* dst, uint64_t N,
                            uint32_t flags, hipStream_t stream);

/* ------------------------------------------------------------------------
 * gz_ingest_multi -- gz_ingest over G independent graphs in one fused
 *   launch sequence.  Updates offs[k] .. offs[k+1]-1 of src/dst belong to gs[k]
 *   (ids local to that graph).  offs is host memory (G+1 entries, offs[0]=0,
 *   non-decreasing); src/dst as in gz_ingest.  The result equals G separate
 *   gz_ingest calls.  The graphs must be distinct and on the current device,
 *   and all of one contract (all V <= 65536 or all V > 65536; else GZ_EINVAL).
 *   Calls share one scratch area per device; a call on one stream waits on
 *   the device for the previous call's kernels, whatever stream those ran on.
 * ---------------------------------------------------------------------- */
gz_status gz_ingest_multi(gz_graph* const* gs, uint32_t G, const uint64_t* offs,
                          const uint32_t* src, const uint32_t* dst, uint32_t flags,
                          hipStream_t stream);

/* ------------------------------------------------------------------------
 * Captured ingest plans: the fused launch sequence of gz_ingest_multi over a
 *   fixed set of graphs, recorded once into a HIP graph and replayed per call.
 *   Every per-call value (inputs, offsets, N) is read by the kernels from
 *   device memory, so one plan serves any call within its capacities.
 * gz_plan_create -- gs: G distinct graphs; caps[k]: the most updates graph k
 *   may receive in one call (sum < 2^31).  Allocates the plan's scratch;
 *   `stream` is used for the one-time uploads.  The graphs must outlive it.
 * gz_plan_ingest -- one call: offs (host, G+1 entries, offs[0] = 0,
 *   non-decreasing, offs[k+1]-offs[k] <= caps[k]); src/dst device arrays
 *   (flags must hold GZ_DEVICE_PTR; GZ_ASYNC as for gz_ingest).  Same result as
 *   gz_ingest_multi on the same arguments.  GZ_EINVAL on an invalid update
 *   (nothing applied) or an offset table outside the capacities.
 * gz_plan_free -- waits for the plan's work and releases it.
 * ---------------------------------------------------------------------- */
typedef struct gz_plan gz_plan;
gz_status gz_plan_create(gz_graph* const* gs, uint32_t G, const uint64_t* caps, hipStream_t stream,
                         gz_plan** out);
gz_status gz_plan_ingest(gz_plan* p, const uint64_t* offs, const uint32_t* src, const uint32_t* dst,
                         uint32_t flags, hipStream_t stream);
gz_status gz_plan_free(gz_plan* p);

/* ------------------------------------------------------------------------
 * gz_flush -- the paper's cleanup() step (Sec. 5.2): wait until every update
 *   submitted to g has been applied.  Returns GZ_EINVAL if an asynchronous
 *   call that included g (alone, in a gz_ingest_multi call or in a plan
 *   replay) carried an invalid update since g's last flush; such a call
 *   applies nothing to any of its graphs, and each of them reports it at its
 *   own next flush.
 * ---------------------------------------------------------------------- */
gz_status gz_flush(gz_graph* g);

/* ------------------------------------------------------------------------
 * gz_connected_components -- flush, then run Boruvka over XOR-merged
 *   sketches (Sec. 2.2; the three phases of Sec. 4.2: sample one edge per
 *   component, merge, sum sketches).  Round r uses every node's round-r
 *   sketch; a component whose sketch is ZERO is complete; a GOOD sample whose
 *   edge does not leave the component counts as FAIL; the sampled edges form a
 *   functional graph whose every cycle loses the edge of its smallest
 *   component.  Works on scratch copies: the sketches are not modified, so
 *   queries may be interleaved with ingestion.
 *   labels  host array of V entries: smallest node id of each node's component;
 *   num_cc  (nullable) number of components.
 *   Returns GZ_ESKETCH_FAIL (outputs still written) if a component was still
 *   active after R rounds.
 * ---------------------------------------------------------------------- */
gz_status gz_connected_components(gz_graph* g, uint32_t* labels, uint32_t* num_cc);

/* ------------------------------------------------------------------------
 * gz_list_spanning_forest -- the problem's output (Sec. 2.1): a spanning
 *   forest of the current graph, from the same Boruvka run as
 *   gz_connected_components.
 *   edges      host array of 2*(V-1) entries: pairs (u, v), u < v, sorted by
 *              idx(u, v);
 *   num_edges  number of pairs written.
 *   Status rules as gz_connected_components.
 * ---------------------------------------------------------------------- */
gz_status gz_list_spanning_forest(gz_graph* g, uint32_t* edges, uint64_t* num_edges);

/* Labels, component count, forest and status of one Boruvka run in one call
 * (any output pointer may be NULL; status per gz_connected_components). */
gz_status gz_query(gz_graph* g, uint32_t* labels, uint32_t* num_cc, uint32_t* edges,
                   uint64_t* num_edges);

/* ------------------------------------------------------------------------
 * gz_connected_components_multi -- Boruvka over G graphs at once (the
 *   many-graph form of gz_connected_components).  labels: host array of
 *   sum(V_k) entries, graph k's labels at offset sum_{j<k} V_j, local ids
 *   (caller-owned; pinned memory reused across calls takes the copy fastest);
 *   num_cc, status: host arrays of G entries (nullable).  Returns GZ_OK if
 *   every graph finished, GZ_ESKETCH_FAIL if any did not.  Graphs with
 *   V > 65536 are queried one at a time (GZ_EINVAL here when G > 1).  Runs
 *   (G = 1 included) take one of a few scratch sets the library keeps per
 *   device, so the graphs hold no query memory of their own; the call
 *   returns once its work is done with the set.
 * ---------------------------------------------------------------------- */
gz_status gz_connected_components_multi(gz_graph* const* gs, uint32_t G, uint32_t* labels,
                                        uint32_t* num_cc, int32_t* status);

/* ------------------------------------------------------------------------
 * gz_export_sketches -- copy the sketches of nodes [node_lo, node_hi) to the
 *   host in the canonical layout alpha/gamma[node][r][c][b] (uint64, rows in
 *   the nested form of Eq. (1)-(2): row b holds every index with depth >= b),
 *   whatever the internal layout.  alpha and gamma hold
 *   (node_hi - node_lo) * R * C * B entries each.  Flushes first.
 * ---------------------------------------------------------------------- */
gz_status gz_export_sketches(gz_graph* g, uint32_t node_lo, uint32_t node_hi, uint64_t* alpha,
                             uint64_t* gamma);

/* Device address and byte size of the internal sketch array (for tools that
 * measure traffic); the layout is private.  A host-tier graph has no device
 * sketch array: *dev_ptr receives NULL, *bytes the size of its host copy. */
gz_status gz_sketch_storage(const gz_graph* g, void** dev_ptr, uint64_t* bytes);

/* ------------------------------------------------------------------------
 * gz_autotune -- pick the ingest launch parameters for g's shape: time a set
 *   of candidate (workgroup size, LDS rows, chunk, workgroups per CU)
 *   configurations on the sample stream src/dst (N updates, device memory:
 *   flags must hold GZ_DEVICE_PTR), with HIP events on `stream`, using a
 *   scratch graph of the same shape (g's sketches are not touched).  The
 *   fastest configuration is set on g and returned in *best (nullable) with
 *   its ingest time in *best_ms (nullable).  Synchronous.
 * ---------------------------------------------------------------------- */
gz_status gz_autotune(gz_graph* g, const uint32_t* src, const uint32_t* dst, uint64_t N,
                      uint32_t flags, hipStream_t stream, gz_tuning* best, float* best_ms);

/* Launch parameters of the ingest path for this graph (get / set). */
gz_status gz_get_tuning(const gz_graph* g, gz_tuning* t);
gz_status gz_set_tuning(gz_graph* g, const gz_tuning* t);

/* Per-phase device timings of the most recent gz_ingest / gz_ingest_multi on a
 * graph (the first graph of a fused call), taken with HIP events on the stream
 * the kernels ran on.  Profiling is off by default; gz_profile_last waits for
 * the profiled call to finish. */
typedef struct gz_profile {
    float group_ms;    /* count + scan + scatter (grouping by endpoint) */
    float update_ms;   /* persistent sketch-update kernel */
    float ingest_ms;   /* whole ingest launch sequence */
    uint32_t calls;    /* profiled ingest calls since enabling */
    uint32_t reserved;
} gz_profile;
gz_status gz_profile_enable(gz_graph* g, int on);
gz_status gz_profile_last(gz_graph* g, gz_profile* out);

/* ------------------------------------------------------------------------
 * gz_measure_peaks -- measure, on the current device, the figures the
 *   roofline of the sketch kernels is read against: a plain 1 GiB device copy
 *   (read + write bytes per second) and the issue rates, in lane operations
 *   per second, of the integer VALU instructions the hashes and bucket XORs
 *   are made of (eight independent chains per lane, enough workgroups to fill
 *   every CU).  Synchronous on `stream`; allocates and frees 2 GiB.
 * ---------------------------------------------------------------------- */
typedef struct gz_peaks {
    double copy_gbs;          /* device copy, read + write GB/s */
    double mul_lo_u32_tops;   /* v_mul_lo_u32, T lane-ops/s */
    double mad_u64_u32_tops;  /* v_mad_u64_u32 */
    double xor_b32_tops;      /* v_xor_b32 */
    double mad_u32_u24_tops;  /* v_mad_u32_u24 */
    double add_u32_tops;      /* v_add_u32 */
    double ctz_b32_tops;      /* v_ffbl_b32 with the v_min, v_add, v_xor of its chain */
    uint32_t cus;
    uint32_t reserved;
} gz_peaks;
gz_status gz_measure_peaks(gz_peaks* out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Serving: many graph sessions on one GPU.
 *   A server thread admits sessions while the device bytes of their sketches
 *   (plus query scratch) fit `hbm_budget`; a session opened beyond the budget
 *   waits, with its requests queued, until closed sessions free memory.  Each
 *   tick takes the update batches queued by every admitted session (up to
 *   `tick_updates` new updates, 0 = 16 Mi; continuous batching: batches
 *   submitted while a tick runs join the next).  Like the gutters of Sec. 4.1 and 5.1,
 *   each session buffers its batches in a gutter in HBM and applies them to
 *   its sketches many at a time: a tick gathers batches into their sessions'
 *   gutters, and applies a session's gutter (its content and the batches
 *   taken behind it) when it cannot hold the next batch, when a query of the
 *   session comes due, or when gz_session_graph needs the sketches; the
 *   gutters a tick applies (up to `tick_updates` updates, one always) go
 *   through one fused multi-graph ingest.  gz_server_set_gutter sets the
 *   gutter size of sessions opened afterwards: updates_per_node * V updates,
 *   at least 65536 (default 64 per node; 0: no gutters, every batch applied by
 *   the tick that takes it); its 8 B per update count against the budget.
 *   An update batch's ticket completes once the batch is in its session's
 *   gutter, or applied.  A query is answered once every batch submitted
 *   before it in its session has been applied, and the session's later
 *   batches wait for it; the
 *   queries queued at that time are answered together by one fused Boruvka
 *   run over their graphs (gz_connected_components_multi), on one of two
 *   query threads, overlapping the next ticks' ingests on the device.  A session's requests
 *   take effect in submission order, so every result is the one the session
 *   would get alone.  All calls are thread-safe.
 * gz_submit_updates copies the batch (host memory, validated while copied:
 *   GZ_EINVAL applies nothing) into a pinned buffer, the only host copy it
 *   makes; the caller's arrays are free again when the call returns.
 * gz_submit_updates_inplace takes src/dst in device memory of the server's GPU
 *   or in pinned host memory (hipHostMalloc), and reads them where they are:
 *   they must hold the batch when the call is made (device memory: its
 *   producing work complete) and stay unchanged until the ticket completes.
 *   Validated at submission (device memory by a kernel, with a synchronous
 *   wait); other memory is rejected with GZ_EINVAL.
 *   Per tick, one kernel gathers the tick's batches from their pinned or
 *   device buffers into HBM staging, and one fused ingest applies them.
 * gz_submit_query writes V labels into `labels` (host, nullable) before its
 *   ticket completes.  gz_wait blocks until the ticket completes, fills *res
 *   (nullable) and releases the ticket; it returns the request's status (a
 *   query whose sketches ran out of rounds reports GZ_ESKETCH_FAIL in
 *   res->status only).  gz_wait_any waits for the first of n tickets (one
 *   server) to complete, up to timeout_ns (UINT64_MAX: no limit), sets *index
 *   and releases that ticket as gz_wait does; GZ_ETIMEOUT (index = n) if none
 *   completed in time, the tickets staying valid.  A client that drives
 *   several sessions waits with gz_wait_any: waiting on one session's ticket
 *   while another of its sessions holds HBM that a waiting session needs
 *   would never end.  Timestamps are steady-clock nanoseconds: submit, start
 *   of processing, completion.
 * gz_session_open takes 2 <= V <= 65536 (sessions share fused calls); else
 *   GZ_EINVAL.
 * gz_session_graph gives the session's graph handle (export, query), for use
 *   while none of the session's requests is queued or running; GZ_ESTATE
 *   before admission or with requests in flight.  It first waits for the
 *   session's gutter to be applied, so that the sketches hold every batch;
 *   a failed ingest of the gutter is returned.  The server keeps ownership.
 * gz_session_close waits for the session's requests and frees its sketches;
 *   gz_server_destroy stops the server and frees every session.
 * Statistics: ticks, updates taken, queries, sessions; batches submitted by
 *   copy and in place; bytes the gather kernels staged; worker time blocked on
 *   a staging set and spent building and launching ticks; fused query runs;
 *   time spent creating and releasing sessions' graphs (sum and maximum);
 *   updates applied to sketches and gutters flushed.  A query reports a
 *   failed ingest of its session's gutter in its status.
 * ---------------------------------------------------------------------- */
typedef struct gz_server gz_server;
typedef struct gz_session gz_session;
typedef struct gz_ticket gz_ticket;
typedef struct gz_result {
    int32_t status;
    uint32_t num_cc;      /* queries: number of components */
    uint32_t kind;        /* 0 = update batch, 1 = query */
    uint32_t reserved;
    uint64_t updates;     /* update batches: number of updates */
    uint64_t submit_ns, start_ns, done_ns;
    uint64_t admit_ns;    /* when the session was admitted (its sketches allocated) */
} gz_result;
typedef struct gz_server_stats {
    uint64_t ticks, updates, queries;
    uint64_t sessions_admitted, sessions_active, sessions_waiting;
    uint64_t hbm_used, hbm_budget;
    uint64_t batches_copied, batches_inplace, staged_bytes;
    uint64_t worker_wait_ns, worker_launch_ns;
    uint64_t query_runs;  /* fused Boruvka runs that answered the queries */
    uint64_t create_ns, create_ns_max;  /* admitted sessions' graph creation time */
    uint64_t free_ns, free_ns_max;      /* closed sessions' graph release time */
    uint64_t ingested;  /* updates applied to sketches (gutters flushed, batches staged) */
    uint64_t flushes;   /* gutters flushed */
} gz_server_stats;
gz_status gz_server_create(uint64_t hbm_budget, uint64_t tick_updates, gz_server** out);
gz_status gz_session_open(gz_server* srv, uint32_t V, uint64_t seed, gz_session** out);
gz_status gz_submit_updates(gz_session* s, const uint32_t* src, const uint32_t* dst, uint64_t N,
                            gz_ticket** out);
gz_status gz_submit_updates_inplace(gz_session* s, const uint32_t* src, const uint32_t* dst,
                                    uint64_t N, gz_ticket** out);
gz_status gz_submit_query(gz_session* s, uint32_t* labels, gz_ticket** out);
gz_status gz_wait(gz_ticket* t, gz_result* res);
gz_status gz_wait_any(gz_ticket* const* tickets, uint32_t n, uint64_t timeout_ns,
                      uint32_t* index, gz_result* res);
gz_status gz_session_graph(gz_session* s, gz_graph** out);
gz_status gz_session_close(gz_session* s);
gz_status gz_server_set_gutter(gz_server* srv, uint32_t updates_per_node);
gz_status gz_server_get_stats(gz_server* srv, gz_server_stats* out);
/* gz_server_timeline -- the first min(cap, *n) tick records (of the first 2^20
 *   ticks), *n = ticks recorded: when the worker took the tick, when its
 *   gather and ingest were enqueued, when the worker saw them complete
 *   (steady-clock ns), its new updates, the updates its ingest applied,
 *   its batches and the graphs it updated, and the device time from its
 *   first to its last kernel. */
typedef struct gz_tick_record {
    uint64_t take_ns, launched_ns, done_ns;
    uint64_t updates;   /* new updates the tick took */
    uint64_t ingested;  /* updates its ingest applied to sketches */
    uint32_t batches, graphs;
    float device_ms;
    uint32_t reserved;
} gz_tick_record;
gz_status gz_server_timeline(gz_server* srv, gz_tick_record* out, uint64_t cap, uint64_t* n);
gz_status gz_server_destroy(gz_server* srv);

/* gz_server_replay -- drive a multi-session workload through `srv` from
 *   client_threads native threads (the serving path's load generator), and
 *   time every request.  Session k (V, seed) owns batches first_batch ..
 *   first_batch + n_batches - 1 of the batch table: batch b is updates
 *   batch_offs[b] .. batch_offs[b+1]-1 of src/dst (host memory, n_batches+1
 *   offsets).  A query follows every query_every-th batch of a session (0:
 *   none) and its last batch.
 *   Closed loop (arrival_ns NULL): every session opens at the start and keeps
 *   one request outstanding, its next batch submitted when all its earlier
 *   requests completed.  Open loop: session k opens at open_ns after the
 *   start and batch b is submitted at arrival_ns[b] after the start (host
 *   arrays, arrival of a session's first batch >= its open_ns), whatever has
 *   completed.  A session closes after its last request completes; sessions
 *   are admitted by the server's HBM budget as usual.
 *   Outputs (host arrays of n_batches entries, nullable): per batch its
 *   latency (completion - arrival; closed loop: - submission), its service
 *   latency (completion - the later of arrival and the session's admission),
 *   and the latency of the query that follows it (0 where none); *wall_ns the
 *   time from the start to the last completion.  Client thread t drives the
 *   sessions k = t, t + T, ...; each waits with gz_wait_any. */
typedef struct gz_replay_session {
    uint32_t V;
    uint32_t n_batches;
    uint64_t seed;
    uint64_t first_batch;
    uint64_t open_ns;
} gz_replay_session;
gz_status gz_server_replay(gz_server* srv, const gz_replay_session* sessions, uint32_t n_sessions,
                           const uint64_t* batch_offs, uint64_t n_batches, const uint32_t* src,
                           const uint32_t* dst, const uint64_t* arrival_ns, uint32_t query_every,
                           uint32_t client_threads, uint64_t* batch_latency_ns,
                           uint64_t* batch_service_ns, uint64_t* query_latency_ns,
                           uint64_t* wall_ns);

/* ------------------------------------------------------------------------
 * The standard l0-sampler (Sec. 3, Fig. "agm_code"): the sketch CubeSketch
 *   replaces, built on the device so that the two update costs can be compared
 *   on the same hardware (Fig. "l0speedup" makes the comparison on a CPU).
 *   Node sketches of a graph with 2 <= V <= 65536 nodes: one sampler per
 *   Boruvka round per node, C = 8 columns, B rows, the shape of CubeSketch.
 *   A bucket holds a = sum of index * Delta, b = sum of Delta and a checksum
 *   c = sum of Delta * z^index mod p, p = 2^61 - 1.  Node vectors are signed:
 *   edge {u, v}, u < v, at index v(v-1)/2 + u, carries +Delta in u's vector and
 *   -Delta in v's (Delta = +1 inserts, -1 deletes), so a node set's sketches
 *   sum to the sketch of its cut.  Row k+1 of a column takes an update while
 *   bit k of the column's hash of the index is zero, with the row hash of the
 *   CubeSketch contract above (same seeds); the column's base z is
 *   1 + (m mod (p - 1)) for its checksum-high multiplier m.  Sums stay exact
 *   while a node's buckets take fewer than 2^32 terms.
 * gz_l0_init    -- zeroed sketches on the current device (GZ_EINVAL outside
 *                  the V range, GZ_ENOMEM); the library owns *out until gz_l0_free.
 * gz_l0_ingest  -- apply N updates: {src[k], dst[k]} with Delta = +1 when
 *                  op[k] != 0 (or op is NULL), -1 when op[k] == 0; arrays in host
 *                  or device memory (GZ_DEVICE_PTR, op then in device memory too).
 *                  Updates are grouped by endpoint on the device, then one
 *                  persistent kernel evaluates z^index by one modular multiply
 *                  per set bit of the index from a table of z^(2^k).
 *                  Synchronous; GZ_EINVAL on a self-loop or an id >= V (nothing
 *                  applied).
 * gz_l0_last_update_ms -- device time of the last ingest's update kernel (HIP
 *                  events on the ingest stream).
 * gz_l0_export  -- nodes [lo, hi) in the layout a/b/c[node][r][c][row] (row b
 *                  holds every index whose column hash has at least b trailing
 *                  zeros, as in the figure), c reduced modulo p.
 * gz_l0_sample  -- the figure's query of every node's round-r sampler: the
 *                  first bucket, columns in order and rows ascending, with b != 0,
 *                  b dividing a, v = a / b a valid index and c = b * z^v mod p.
 *                  kind[v] = 0 (all buckets zero), 1 (sample: idx[v], mult[v] = b),
 *                  2 (no bucket passes).  Host arrays of V entries.
 * gz_l0_reset, gz_l0_shape, gz_l0_free as for CubeSketch graphs.
 * ---------------------------------------------------------------------- */
typedef struct gz_l0 gz_l0;
gz_status gz_l0_init(gz_l0** out, uint32_t V, uint64_t seed);
gz_status gz_l0_free(gz_l0* s);
gz_status gz_l0_reset(gz_l0* s, hipStream_t stream);
gz_status gz_l0_shape(const gz_l0* s, uint32_t* V, uint32_t* R, uint32_t* C, uint32_t* B,
                      uint64_t* n);
gz_status gz_l0_ingest(gz_l0* s, const uint32_t* src, const uint32_t* dst, const uint8_t* op,
                       uint64_t N, uint32_t flags, hipStream_t stream);
gz_status gz_l0_last_update_ms(gz_l0* s, float* ms);
gz_status gz_l0_export(gz_l0* s, uint32_t node_lo, uint32_t node_hi, int64_t* a, int64_t* b,
                       uint64_t* c);
gz_status gz_l0_sample(gz_l0* s, uint32_t round, int32_t* kind, uint64_t* idx, int64_t* mult);

/* Human-readable name of a status code, and the last error message of this thread. */
const char* gz_status_str(gz_status s);
const char* gz_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GZ_H */
