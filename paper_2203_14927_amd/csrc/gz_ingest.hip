// Ingest path: group the stream by endpoint on the device, then apply each
// node's batch to its CubeSketches with the node tile staged in LDS.
//
// Paper: CubeSketch update (Sec. 3.1, Fig. "cube_code"); per-node batching of
// updates so that one node's sketch is touched once per batch (Sec. 4.1, 5.1);
// batch- and sketch-level parallelism (Sec. 5.1) become workgroups over node
// batches and lanes over (round, column) pairs.
//
// Grouping is a counting sort keyed by global node id: every block counts one
// chunk of one graph's updates in an LDS histogram, the (node, chunk) table of
// counts is scanned, and a second pass scatters each entry through LDS cursors
// seeded from the scanned table.  No global atomics touch the hot counters.
#include <algorithm>
#include <cstring>

#include "gz_device.h"
#include "gz_internal.h"

namespace gz {

// ---------------------------------------------------------------- kernels --

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// zero n words (16-byte stores; p from hipMalloc/hipMallocAsync, so 256-byte aligned)
__global__ __launch_bounds__(256) void k_zero_words(uint32_t* __restrict__ p, uint64_t n) {
    uint4* q = reinterpret_cast<uint4*>(p);
    const uint64_t n4 = n / 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        q[i] = make_uint4(0, 0, 0, 0);
    for (uint64_t i = n4 * 4 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = 0;
}

// Clearing with a kernel rather than hipMemsetAsync keeps large clears (a
// new graph's sketches) off the copy engines, which every call's small
// host-to-device copies need, and can be captured into a HIP graph.
hipError_t zero_words(uint32_t* p, uint64_t n, hipStream_t stream) {
    if (!n) return hipSuccess;
    const uint64_t blocks =
        std::min<uint64_t>((n / 4 + 255) / 256 + 1, (uint64_t)device_cu_count() * 8);
    k_zero_words<<<(uint32_t)blocks, 256, 0, stream>>>(p, n);
    return hipGetLastError();
}

__global__ void k_note_error(const GraphDesc* __restrict__ descs, uint32_t G,
                             const uint32_t* __restrict__ call_err) {
    if (*call_err == 0) return;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < G; k += gridDim.x * blockDim.x)
        *descs[k].err = 1u;
}

// the same for the one graph of a per-node call
__global__ void k_note_error_one(uint32_t* __restrict__ graph_err,
                                 const uint32_t* __restrict__ call_err) {
    if (threadIdx.x == 0 && *call_err) *graph_err = 1u;
}

// last graph g with node_base <= node
__device__ __forceinline__ uint32_t graph_of_node(const GraphDesc* __restrict__ gd, uint32_t G,
                                                  uint32_t node) {
    uint32_t lo = 0, hi = G - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (gd[mid].node_base <= node) lo = mid; else hi = mid - 1;
    }
    return lo;
}

constexpr uint32_t kGroupThreads = 1024;

struct UnitRange {
    uint64_t i0, i1;    // updates [i0, i1)
    uint32_t lo, size;  // local node range [lo, lo + size)
};

// Updates of graph g: from the per-call offset table when the launch has one
// (captured plans), else from the descriptor table.
__device__ __forceinline__ UnitRange unit_range(const IngestArgs* __restrict__ a,
                                                const GraphDesc* __restrict__ gd,
                                                const GroupUnit& u, const GraphDesc& g) {
    uint64_t b, e;
    if (a->offs) {
        b = a->offs[u.g];
        e = a->offs[u.g + 1];
    } else {
        b = g.upd_base;
        e = u.g + 1 < a->G ? gd[u.g + 1].upd_base : a->N;
    }
    UnitRange r;
    r.i0 = b + (uint64_t)u.c * a->group_chunk;
    r.i1 = min(e, r.i0 + a->group_chunk);  // below i0 for chunks past the graph's end
    r.lo = u.q * kGroupRange;
    r.size = min(g.V - r.lo, kGroupRange);
    return r;
}

constexpr uint32_t kCountBatch = 4;  // updates loaded per thread before counting any

// pass 1: LDS histogram of one chunk's endpoints; validation of the updates
// (ctl[2]: this call saw an invalid update)
__global__ __launch_bounds__(kGroupThreads) void k_group_count(
    const IngestArgs* __restrict__ a, const GroupUnit* __restrict__ units,
    const GraphDesc* __restrict__ gd, uint32_t* __restrict__ H, uint32_t* __restrict__ ctl) {
    extern __shared__ uint32_t hist[];
    const GroupUnit u = units[blockIdx.x];
    const GraphDesc g = gd[u.g];
    const UnitRange r = unit_range(a, gd, u, g);
    const uint32_t* __restrict__ src = a->src;
    const uint32_t* __restrict__ dst = a->dst;
    for (uint32_t k = threadIdx.x; k < r.size; k += blockDim.x) hist[k] = 0;
    __syncthreads();
    bool bad = false;
    // loads issued kCountBatch at a time, so that they are in flight together
    for (uint64_t i0 = r.i0; i0 < r.i1; i0 += (uint64_t)kCountBatch * blockDim.x) {
        uint32_t x[kCountBatch], y[kCountBatch], in = 0;
#pragma unroll
        for (uint32_t k = 0; k < kCountBatch; ++k) {
            const uint64_t i = i0 + threadIdx.x + (uint64_t)k * blockDim.x;
            if (i < r.i1) in |= 1u << k;
            x[k] = i < r.i1 ? src[i] : 0u;
            y[k] = i < r.i1 ? dst[i] : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < kCountBatch; ++k) {
            if (!((in >> k) & 1u)) continue;
            if (x[k] == y[k] || x[k] >= g.V || y[k] >= g.V) {
                bad = true;
                continue;
            }
            const uint32_t xo = x[k] - r.lo, yo = y[k] - r.lo;
            if (xo < r.size) atomicAdd(&hist[xo], 1u);
            if (yo < r.size) atomicAdd(&hist[yo], 1u);
        }
    }
    if (bad && u.q == 0) atomicOr(&ctl[2], 1u);
    __syncthreads();
    uint32_t* out = H + g.hoff + (uint64_t)u.c * g.V + r.lo;
    for (uint32_t k = threadIdx.x; k < r.size; k += blockDim.x) out[k] = hist[k];
}

// The count table of a graph is chunk-major: H[hoff + c * V + v].  A node's
// entries total the column sum over its chunks ...  kColLanes adjacent lanes
// share a node, each taking a contiguous quarter of its chunks, so that more
// loads are in flight than one lane per node would issue.
constexpr uint32_t kColLanes = 4;

__global__ void k_group_colsum(const GraphDesc* __restrict__ gd, uint32_t G, uint32_t T,
                               const uint32_t* __restrict__ H, uint32_t* __restrict__ counts) {
    const uint32_t sub = threadIdx.x % kColLanes;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < T * kColLanes;
         t += gridDim.x * blockDim.x) {
        const uint32_t v = t / kColLanes;
        const uint32_t gi = G == 1 ? 0u : graph_of_node(gd, G, v);
        const GraphDesc& g = gd[gi];
        const uint32_t* col = H + g.hoff + (v - g.node_base);
        const uint32_t c0 = g.nb * sub / kColLanes, c1 = g.nb * (sub + 1) / kColLanes;
        uint32_t sum = 0;
        for (uint32_t c = c0; c < c1; ++c) sum += col[(uint64_t)c * g.V];
        for (uint32_t off = 1; off < kColLanes; off <<= 1) sum += __shfl_xor(sum, off, kColLanes);
        if (sub == 0) counts[v] = sum;
    }
}

// ... and, once the node's first slot is known, each chunk's run starts after
// the runs of the earlier chunks (in-place exclusive scan down the column:
// each lane sums its quarter, the lanes scan those sums, then each rewrites
// its quarter)
__global__ void k_group_colscan(const GraphDesc* __restrict__ gd, uint32_t G, uint32_t T,
                                const uint32_t* __restrict__ nodeoff, uint32_t* __restrict__ H) {
    const uint32_t sub = threadIdx.x % kColLanes;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < T * kColLanes;
         t += gridDim.x * blockDim.x) {
        const uint32_t v = t / kColLanes;
        const uint32_t gi = G == 1 ? 0u : graph_of_node(gd, G, v);
        const GraphDesc& g = gd[gi];
        uint32_t* col = H + g.hoff + (v - g.node_base);
        const uint32_t c0 = g.nb * sub / kColLanes, c1 = g.nb * (sub + 1) / kColLanes;
        uint32_t part = 0;
        for (uint32_t c = c0; c < c1; ++c) part += col[(uint64_t)c * g.V];
        uint32_t incl = part;  // inclusive scan over the node's lanes
        for (uint32_t off = 1; off < kColLanes; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, kColLanes);
            if (sub >= off) incl += y;
        }
        uint32_t run = nodeoff[v] + incl - part;
        for (uint32_t c = c0; c < c1; ++c) {
            const uint32_t x = col[(uint64_t)c * g.V];
            col[(uint64_t)c * g.V] = run;
            run += x;
        }
    }
}

constexpr uint32_t kScatterBatch = 4;  // updates loaded per thread before placing any

// pass 2: scatter every endpoint entry to its slot; LDS cursors start at the
// scanned (node, chunk) prefix, so each chunk fills its own contiguous run
__global__ __launch_bounds__(kGroupThreads) void k_group_scatter(
    const IngestArgs* __restrict__ a, const GroupUnit* __restrict__ units,
    const GraphDesc* __restrict__ gd, const uint32_t* __restrict__ Hs,
    uint32_t* __restrict__ grouped, const uint32_t* __restrict__ ctl) {
    extern __shared__ uint32_t cur[];
    if (ctl[2]) return;
    const GroupUnit u = units[blockIdx.x];
    const GraphDesc g = gd[u.g];
    const UnitRange r = unit_range(a, gd, u, g);
    const uint32_t* __restrict__ src = a->src;
    const uint32_t* __restrict__ dst = a->dst;
    const uint32_t* hs = Hs + g.hoff + (uint64_t)u.c * g.V + r.lo;
    for (uint32_t k = threadIdx.x; k < r.size; k += blockDim.x) cur[k] = hs[k];
    __syncthreads();
    for (uint64_t i0 = r.i0; i0 < r.i1; i0 += (uint64_t)kScatterBatch * blockDim.x) {
        uint32_t x[kScatterBatch], y[kScatterBatch];
#pragma unroll
        for (uint32_t k = 0; k < kScatterBatch; ++k) {
            const uint64_t i = i0 + threadIdx.x + (uint64_t)k * blockDim.x;
            x[k] = i < r.i1 ? src[i] : kNone;
            y[k] = i < r.i1 ? dst[i] : kNone;
        }
#pragma unroll
        for (uint32_t k = 0; k < kScatterBatch; ++k) {
            if (x[k] == kNone) continue;
            // an entry is the edge index, or for wide graphs the other endpoint
            const uint32_t idx = g.wide ? 0u : edge_index(x[k], y[k]);
            const uint32_t xo = x[k] - r.lo, yo = y[k] - r.lo;
            if (xo < r.size) grouped[atomicAdd(&cur[xo], 1u)] = g.wide ? y[k] : idx;
            if (yo < r.size) grouped[atomicAdd(&cur[yo], 1u)] = g.wide ? x[k] : idx;
        }
    }
}

// Sorted placement for calls whose graphs all have at most kSortNodes nodes
// (a unit then covers every node of its graph).  The one-pass scatter above
// stores each entry alone into one of V open runs: on 4096 graphs at once
// those partly written lines left L2 and reached HBM as about six times the
// bytes placed.  Here a unit takes its chunk in batches of `batch` updates:
// counts per node in LDS, an exclusive scan, the batch's entries placed in
// node order in LDS, then stored run after run, so that consecutive lanes
// write consecutive words of a node's run.
constexpr uint32_t kSortNodes = 4096;
constexpr uint32_t kSortPer = 4;  // updates per thread and batch, at most
constexpr uint32_t kSortSmemTarget = 80 * 1024 - 256;  // two workgroups per CU

// exclusive scan of c[0..n) in place, n <= 4 * blockDim.x (1024 threads)
__device__ __forceinline__ void block_scan4(uint32_t* __restrict__ c, uint32_t n,
                                            uint32_t* __restrict__ wsum) {
    const uint32_t base = threadIdx.x * 4u, lane = __lane_id(), wave = threadIdx.x >> 6;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        v[k] = base + k < n ? c[base + k] : 0u;
        sum += v[k];
    }
    uint32_t incl = sum;
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) {
            const uint32_t t = wsum[w];
            wsum[w] = run;
            run += t;
        }
    }
    __syncthreads();
    uint32_t at = wsum[wave] + incl - sum;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        if (base + k < n) c[base + k] = at;
        at += v[k];
    }
}

__global__ __launch_bounds__(kGroupThreads) void k_group_scatter_sorted(
    const IngestArgs* __restrict__ a, const GroupUnit* __restrict__ units,
    const GraphDesc* __restrict__ gd, const uint32_t* __restrict__ Hs,
    uint32_t* __restrict__ grouped, const uint32_t* __restrict__ ctl, uint32_t range,
    uint32_t batch) {
    extern __shared__ uint32_t sm[];
    __shared__ uint32_t wsum[kGroupThreads / 64];
    uint32_t* gcur = sm;             // [range] next slot of each node's run in `grouped`
    uint32_t* cnt = sm + range;      // [range] batch counts, then run starts/ends in ent
    uint32_t* ent = sm + 2 * range;  // [2 * batch] the batch's entries in node order
    uint16_t* nod = reinterpret_cast<uint16_t*>(ent + 2 * batch);  // [2 * batch] their nodes
    if (ctl[2]) return;  // an invalid update: nothing is applied
    const GroupUnit u = units[blockIdx.x];
    const GraphDesc g = gd[u.g];
    const UnitRange r = unit_range(a, gd, u, g);  // lo = 0, size = V
    const uint32_t V = r.size;
    const uint32_t* __restrict__ src = a->src;
    const uint32_t* __restrict__ dst = a->dst;
    const uint32_t* hs = Hs + g.hoff + (uint64_t)u.c * g.V;
    for (uint32_t k = threadIdx.x; k < V; k += blockDim.x) gcur[k] = hs[k];
    for (uint64_t b0 = r.i0; b0 < r.i1; b0 += batch) {
        const uint32_t n = r.i1 - b0 < batch ? (uint32_t)(r.i1 - b0) : batch;
        for (uint32_t k = threadIdx.x; k < V; k += blockDim.x) cnt[k] = 0;
        __syncthreads();
        // the batch's updates stay in registers between the two passes, both
        // endpoints (< 2^16) packed in one word
        uint32_t xy[kSortPer];
#pragma unroll
        for (uint32_t j = 0; j < kSortPer; ++j) {
            const uint32_t i = j * blockDim.x + threadIdx.x;
            xy[j] = i < n ? src[b0 + i] | (dst[b0 + i] << 16) : kNone;
        }
#pragma unroll
        for (uint32_t j = 0; j < kSortPer; ++j)
            if (xy[j] != kNone) {
                atomicAdd(&cnt[xy[j] & 0xFFFFu], 1u);
                atomicAdd(&cnt[xy[j] >> 16], 1u);
            }
        __syncthreads();
        block_scan4(cnt, V, wsum);
        __syncthreads();
#pragma unroll
        for (uint32_t j = 0; j < kSortPer; ++j)
            if (xy[j] != kNone) {
                const uint32_t x = xy[j] & 0xFFFFu, y = xy[j] >> 16;
                const uint32_t idx = edge_index(x, y);
                const uint32_t p = atomicAdd(&cnt[x], 1u);
                ent[p] = idx;
                nod[p] = (uint16_t)x;
                const uint32_t q = atomicAdd(&cnt[y], 1u);
                ent[q] = idx;
                nod[q] = (uint16_t)y;
            }
        __syncthreads();
        // cnt[v] is now the end of v's run in ent, which is where v + 1's starts
        for (uint32_t i = threadIdx.x; i < 2 * n; i += blockDim.x) {
            const uint32_t v = nod[i];
            const uint32_t start = v ? cnt[v - 1] : 0u;
            grouped[gcur[v] + (i - start)] = ent[i];
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < V; k += blockDim.x)
            gcur[k] += cnt[k] - (k ? cnt[k - 1] : 0u);
        __syncthreads();
    }
}

uint32_t sort_batch(uint32_t range) {
    const uint32_t fit = (kSortSmemTarget - 8u * range) / 12u;  // 4 B entry + 2 B node, twice
    return std::min(kSortPer * kGroupThreads, fit / 256u * 256u);
}

size_t sort_smem(uint32_t range) {
    const uint32_t b = sort_batch(range);
    return (size_t)2 * range * 4 + (size_t)2 * b * 4 + (size_t)2 * b * 2;
}

// Two-pass placement for large single-graph calls.  The one-pass scatter
// above writes every chunk's entries into V node runs, far more open lines
// than L2 holds, so each 4-byte store becomes a partial-line HBM write.  Here
// pass A moves each chunk's entries into at most kMaxBuckets buckets of 2^S
// consecutive nodes (a bucket's region is the range its nodes take in the
// final array, and every chunk fills its own sub-range of it), then pass B
// places each bucket's entries into the runs of its nodes.  Both passes sort
// a batch of entries by destination run in LDS first and then write each run's
// share of the batch with consecutive stores, so HBM sees whole lines.  A
// bucket entry packs the node's offset in its bucket above the other
// endpoint: (fine << 16) | neighbour for graphs up to 2^16 nodes, and
// (fine << nbits) | neighbour, nbits = bitlen(V-1), for wider graphs up to
// 2^20 nodes (S = nbits - 8 with 256 buckets, so 32 bits suffice).
constexpr uint32_t kMaxBuckets = 256;          // runs per block (keys of a batch)
constexpr uint32_t kMaxBucketNodes = 256;      // 2^S: V <= 2^16 spread over <= 256 buckets
constexpr uint32_t kMaxBucketNodesWide = 4096; // 2^S: V <= 2^20
constexpr uint32_t kMaxTwoPassWide = 1u << 20;
constexpr uint32_t kSortPerThread = 8;     // entries per thread and batch
constexpr uint32_t kSortBatch = kSortPerThread * kGroupThreads;

struct SortSmem {
    uint32_t val[kSortBatch];
    uint8_t key[kSortBatch];
    uint32_t cnt[kMaxBuckets];   // batch counts, then local cursors
    uint32_t loff[kMaxBuckets];  // first local slot of each key
    uint32_t gpos[kMaxBuckets];  // first global slot of each key's share
    uint32_t total;
};

// Keys and values of a batch computed into registers here, before the next
// batch's loads are issued (so that the sort never waits on those loads).
__device__ __forceinline__ void materialise(uint32_t (&key)[kSortPerThread],
                                            uint32_t (&val)[kSortPerThread]) {
#pragma unroll
    for (uint32_t k = 0; k < kSortPerThread; ++k) asm volatile("" : "+v"(key[k]), "+v"(val[k]) :: "memory");
}

// Workgroup barrier for LDS traffic only: this wave's LDS operations complete
// first, its global loads may stay in flight across it (the next batch's
// loads overlap this batch's sort).
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Append one batch of (key, value) pairs, kSortPerThread per thread, to the
// runs of `out` whose next free slots are cur[key] (block-private LDS
// cursors, advanced here): the batch is counted per key and staged in LDS in
// key order, then each key's share is stored with consecutive lanes.  Order
// within a key is whatever the LDS atomics give (the sketch update is a sum
// over Z2, so the sketches do not depend on it).  Every thread of the block
// must call it.
__device__ __forceinline__ void batch_append(const uint32_t (&key)[kSortPerThread],
                                             const uint32_t (&val)[kSortPerThread],
                                             uint32_t valid_mask, uint32_t nkeys,
                                             uint32_t* __restrict__ cur, SortSmem& sm,
                                             uint32_t* __restrict__ out) {
    const uint32_t tid = threadIdx.x;
    for (uint32_t k = tid; k < nkeys; k += blockDim.x) sm.cnt[k] = 0;
    lds_barrier();
#pragma unroll
    for (uint32_t j = 0; j < kSortPerThread; ++j)
        if ((valid_mask >> j) & 1u) atomicAdd(&sm.cnt[key[j]], 1u);
    lds_barrier();
    if (tid < 64) {  // one wave scans the (at most 256) counts, four per lane
        uint32_t c[4], run = 0;
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
            const uint32_t k = tid * 4 + i;
            c[i] = k < nkeys ? sm.cnt[k] : 0u;
            run += c[i];
        }
        uint32_t incl = run;
        for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint32_t t = __shfl_up(incl, off);
            if (tid >= off) incl += t;
        }
        uint32_t at = incl - run;
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
            const uint32_t k = tid * 4 + i;
            if (k < nkeys) {
                sm.loff[k] = at;
                sm.cnt[k] = at;  // local cursor
                sm.gpos[k] = cur[k];
                cur[k] += c[i];
            }
            at += c[i];
        }
        if (tid == 63) sm.total = incl;
    }
    lds_barrier();
#pragma unroll
    for (uint32_t j = 0; j < kSortPerThread; ++j) {
        if (!((valid_mask >> j) & 1u)) continue;
        const uint32_t p = atomicAdd(&sm.cnt[key[j]], 1u);
        sm.val[p] = val[j];
        sm.key[p] = (uint8_t)key[j];
    }
    lds_barrier();
    const uint32_t total = sm.total;
    for (uint32_t p = tid; p < total; p += blockDim.x) {
        const uint32_t k = sm.key[p];
        out[sm.gpos[k] + (p - sm.loff[k])] = sm.val[p];
    }
    lds_barrier();
}

// base[c * nbk + b], c <= nb: first slot of chunk c's entries of bucket b
// (c = nb: the end of the bucket's region)
__global__ void k_group_bucket_base(const uint32_t* __restrict__ H,
                                    const uint32_t* __restrict__ nodeoff,
                                    const uint32_t* __restrict__ counts, uint32_t V, uint32_t S,
                                    uint32_t nbk, uint32_t nb, uint32_t* __restrict__ base) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (nb + 1) * nbk) return;
    const uint32_t c = t / nbk, b = t - c * nbk;
    const uint32_t v0 = b << S, v1 = min(V, (b + 1) << S);
    uint32_t sum = nodeoff[v0];
    if (c < nb) {
        const uint32_t* row = H + (uint64_t)c * V;
        for (uint32_t v = v0; v < v1; ++v) sum += row[v] - nodeoff[v];  // earlier chunks' entries
    } else {
        for (uint32_t v = v0; v < v1; ++v) sum += counts[v];
    }
    base[t] = sum;
}

// pass A: one block per chunk of the single graph's updates
__global__ __launch_bounds__(kGroupThreads) void k_group_partition(
    const IngestArgs* __restrict__ a, const GraphDesc* __restrict__ gd,
    const uint32_t* __restrict__ base, uint32_t S, uint32_t nbk, uint32_t* __restrict__ tmp,
    const uint32_t* __restrict__ ctl) {
    __shared__ uint32_t cur[kMaxBuckets];
    __shared__ SortSmem sm;
    if (ctl[2]) return;
    const GraphDesc g = gd[0];
    const UnitRange r = unit_range(a, gd, GroupUnit{0, blockIdx.x, 0, 0}, g);
    // global-memory views of the stream (pointers read from memory would load
    // through flat instructions, which also count against the LDS wait)
    typedef const __attribute__((address_space(1))) uint32_t* gsrc_t;
    const gsrc_t src = (gsrc_t)a->src;
    const gsrc_t dst = (gsrc_t)a->dst;
    for (uint32_t k = threadIdx.x; k < nbk; k += blockDim.x) cur[k] = base[blockIdx.x * nbk + k];
    __syncthreads();
    const uint32_t mask = (1u << S) - 1u;
    const uint32_t nbits = g.wide ? 32u - __builtin_clz((g.V - 1u) | 1u) : 16u;
    constexpr uint32_t kUpd = kSortPerThread / 2;                  // two entries per update
    const uint64_t step = (uint64_t)kUpd * blockDim.x;
    // the next batch's updates are loaded while this batch is sorted
    uint32_t xs[kUpd], ys[kUpd];
#pragma unroll
    for (uint32_t k = 0; k < kUpd; ++k) {
        const uint64_t i = r.i0 + threadIdx.x + (uint64_t)k * blockDim.x;
        xs[k] = i < r.i1 ? src[i] : 0u;
        ys[k] = i < r.i1 ? dst[i] : 0u;
    }
    for (uint64_t i0 = r.i0; i0 < r.i1; i0 += step) {
        uint32_t key[kSortPerThread], val[kSortPerThread], ok = 0;
#pragma unroll
        for (uint32_t k = 0; k < kUpd; ++k) {
            const uint64_t i = i0 + threadIdx.x + (uint64_t)k * blockDim.x;
            const uint32_t x = xs[k], y = ys[k];
            if (i < r.i1) ok |= 3u << (2 * k);
            key[2 * k] = x >> S;
            val[2 * k] = ((x & mask) << nbits) | y;
            key[2 * k + 1] = y >> S;
            val[2 * k + 1] = ((y & mask) << nbits) | x;
        }
        materialise(key, val);
#pragma unroll
        for (uint32_t k = 0; k < kUpd; ++k) {
            const uint64_t in = i0 + step + threadIdx.x + (uint64_t)k * blockDim.x;
            xs[k] = in < r.i1 ? src[in] : 0u;
            ys[k] = in < r.i1 ? dst[in] : 0u;
        }
        batch_append(key, val, ok, nbk, cur, sm, tmp);
    }
}

// pass B: one block per (bucket, range of cr chunks); node cursors start at the
// runs of the range's first chunk, so blocks of one bucket fill disjoint slots
__global__ __launch_bounds__(kGroupThreads) void k_group_place(
    const uint32_t* __restrict__ base, const uint32_t* __restrict__ H, uint32_t V, uint32_t S,
    uint32_t nbk, uint32_t nb, uint32_t cr, const uint32_t* __restrict__ tmp,
    uint32_t* __restrict__ grouped, const uint32_t* __restrict__ ctl) {
    __shared__ uint32_t cur[kMaxBucketNodes];
    __shared__ SortSmem sm;
    if (ctl[2]) return;
    // the workgroups of one bucket are consecutive (a hub bucket's start
    // together; dense grouping 0.91 -> 0.85 ms)
    const uint32_t per = gridDim.x / nbk;
    const uint32_t b = blockIdx.x / per;
    const uint32_t c0 = (blockIdx.x % per) * cr;
    const uint32_t c1 = min(nb, c0 + cr);
    const uint32_t v0 = b << S, n = min(V, (b + 1) << S) - v0;
    const uint32_t* row = H + (uint64_t)c0 * V + v0;
    for (uint32_t f = threadIdx.x; f < n; f += blockDim.x) cur[f] = row[f];
    __syncthreads();
    const uint32_t e1 = base[c1 * nbk + b];
    const uint32_t step = kSortPerThread * blockDim.x;
    // the next batch's entries are loaded while this batch is sorted
    uint32_t ws[kSortPerThread];
    const uint32_t e_first = base[c0 * nbk + b];
#pragma unroll
    for (uint32_t k = 0; k < kSortPerThread; ++k) {
        const uint32_t e = e_first + threadIdx.x + k * blockDim.x;
        ws[k] = e < e1 ? tmp[e] : 0u;
    }
    for (uint32_t e0 = e_first; e0 < e1; e0 += step) {
        uint32_t key[kSortPerThread], val[kSortPerThread], ok = 0;
#pragma unroll
        for (uint32_t k = 0; k < kSortPerThread; ++k) {
            const uint32_t e = e0 + threadIdx.x + k * blockDim.x;
            const uint32_t w = ws[k];
            if (e < e1) ok |= 1u << k;
            key[k] = w >> 16;
            val[k] = edge_index(v0 + (w >> 16), w & 0xFFFFu);
        }
        materialise(key, val);
#pragma unroll
        for (uint32_t k = 0; k < kSortPerThread; ++k) {
            const uint32_t en = e0 + step + threadIdx.x + k * blockDim.x;
            ws[k] = en < e1 ? tmp[en] : 0u;
        }
        batch_append(key, val, ok, n, cur, sm, grouped);
    }
}

constexpr uint32_t kLoadBatch = 8;  // loads per thread issued before their use

// Wide graphs count per bucket first (one read of the stream; validation as in
// k_group_count), take the bucket regions from those counts, and count per
// node from the bucket entries after pass A (one read of them), instead of
// reading the stream once per 32768-node range.  Hb[c * nbk + b] = entries of
// chunk c in bucket b (kept at the start of the node count table, which the
// node counts overwrite later).
__global__ __launch_bounds__(kGroupThreads) void k_group_bcount(
    const IngestArgs* __restrict__ a, const GraphDesc* __restrict__ gd, uint32_t S, uint32_t nbk,
    uint32_t* __restrict__ Hb, uint32_t* __restrict__ ctl) {
    __shared__ uint32_t hist[kMaxBuckets];
    const GraphDesc g = gd[0];
    const UnitRange r = unit_range(a, gd, GroupUnit{0, blockIdx.x, 0, 0}, g);
    typedef const __attribute__((address_space(1))) uint32_t* gsrc_t;
    const gsrc_t src = (gsrc_t)a->src;
    const gsrc_t dst = (gsrc_t)a->dst;
    for (uint32_t k = threadIdx.x; k < kMaxBuckets; k += blockDim.x) hist[k] = 0;
    __syncthreads();
    bool bad = false;
    for (uint64_t i0 = r.i0; i0 < r.i1; i0 += (uint64_t)kLoadBatch * blockDim.x) {
        uint32_t x[kLoadBatch], y[kLoadBatch], in = 0;
#pragma unroll
        for (uint32_t k = 0; k < kLoadBatch; ++k) {
            const uint64_t i = i0 + threadIdx.x + (uint64_t)k * blockDim.x;
            if (i < r.i1) in |= 1u << k;
            x[k] = i < r.i1 ? src[i] : 0u;
            y[k] = i < r.i1 ? dst[i] : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < kLoadBatch; ++k) {
            if (!((in >> k) & 1u)) continue;  // past the chunk
            if (x[k] == y[k] || x[k] >= g.V || y[k] >= g.V) {
                bad = true;
                continue;
            }
            atomicAdd(&hist[x[k] >> S], 1u);
            atomicAdd(&hist[y[k] >> S], 1u);
        }
    }
    if (bad) atomicOr(&ctl[2], 1u);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < nbk; k += blockDim.x) Hb[blockIdx.x * nbk + k] = hist[k];
}

// base[c * nbk + b] (c <= nb) from the bucket counts: bucket regions in node
// order, chunk c's share of a region after the shares of earlier chunks
__global__ __launch_bounds__(kMaxBuckets) void k_group_bbase_wide(const uint32_t* __restrict__ Hb,
                                                                  uint32_t nbk, uint32_t nb,
                                                                  uint32_t* __restrict__ base) {
    __shared__ uint32_t s_t[kMaxBuckets];
    const uint32_t b = threadIdx.x;
    uint32_t tot = 0;
    if (b < nbk)
        for (uint32_t c = 0; c < nb; ++c) tot += Hb[(uint64_t)c * nbk + b];
    s_t[b] = tot;
    __syncthreads();
    for (uint32_t off = 1; off < kMaxBuckets; off <<= 1) {
        const uint32_t t = b >= off ? s_t[b - off] : 0u;
        __syncthreads();
        s_t[b] += t;
        __syncthreads();
    }
    if (b >= nbk) return;
    uint32_t at = s_t[b] - tot;
    for (uint32_t c = 0; c < nb; ++c) {
        base[(uint64_t)c * nbk + b] = at;
        at += Hb[(uint64_t)c * nbk + b];
    }
    base[(uint64_t)nb * nbk + b] = at;
}

// node counts of chunk c from its share of bucket b: H[c * V + v] for the
// bucket's nodes v (one block per (bucket, chunk); every row word is written)
__global__ __launch_bounds__(256) void k_group_ncount(const uint32_t* __restrict__ base,
                                                      uint32_t nbk, uint32_t S, uint32_t V,
                                                      const uint32_t* __restrict__ tmp,
                                                      uint32_t* __restrict__ H,
                                                      const uint32_t* __restrict__ ctl) {
    __shared__ uint32_t hist[kMaxBucketNodesWide];
    if (ctl[2]) return;
    // workgroups of one bucket are consecutive, so that a hub bucket's (each
    // many times the average) start together at the front of the grid instead
    // of one per wave of workgroups (2.3 -> 0.5 ms on 2^18 nodes)
    const uint32_t nc = gridDim.x / nbk;
    const uint32_t b = blockIdx.x / nc, c = blockIdx.x % nc;
    const uint32_t nbits = 32u - __builtin_clz((V - 1u) | 1u);
    const uint32_t v0 = b << S, n = min(V, (b + 1) << S) - v0;
    for (uint32_t f = threadIdx.x; f < n; f += blockDim.x) hist[f] = 0;
    __syncthreads();
    const uint32_t e1 = base[(uint64_t)(c + 1) * nbk + b];
    // loads issued kLoadBatch at a time, so that they are in flight together
    for (uint32_t e0 = base[(uint64_t)c * nbk + b]; e0 < e1; e0 += kLoadBatch * blockDim.x) {
        uint32_t w[kLoadBatch];
#pragma unroll
        for (uint32_t k = 0; k < kLoadBatch; ++k) {
            const uint32_t e = e0 + threadIdx.x + k * blockDim.x;
            w[k] = e < e1 ? tmp[e] : kNone;
        }
#pragma unroll
        for (uint32_t k = 0; k < kLoadBatch; ++k)
            if (w[k] != kNone) atomicAdd(&hist[w[k] >> nbits], 1u);
    }
    __syncthreads();
    uint32_t* row = H + (uint64_t)c * V + v0;
    for (uint32_t f = threadIdx.x; f < n; f += blockDim.x) row[f] = hist[f];
}

// Wide graphs, pass B.  A typical node of a raw R-MAT stream at V = 2^18 has
// less than one entry per grouping chunk, so per-chunk runs are a few bytes;
// instead a block places whole pieces of a bucket (runs of consecutive chunks,
// all of them for most buckets) through LDS cursors, so each node's entries of
// a piece land in one contiguous run.  Pieces hold about `target` entries: hub
// buckets are cut into many (k_group_pieces), the rest take one block each.
// pieces[0] = number of pieces, then (bucket, first chunk, end chunk) triples.
__global__ __launch_bounds__(kMaxBuckets) void k_group_pieces(const uint32_t* __restrict__ base,
                                                              uint32_t nbk, uint32_t nb,
                                                              uint32_t target, uint32_t cap,
                                                              uint32_t* __restrict__ pieces,
                                                              const uint32_t* __restrict__ ctl) {
    __shared__ uint32_t s_p[kMaxBuckets];
    if (ctl[2]) return;
    const uint32_t b = threadIdx.x;
    uint32_t p = 0, lo = 0, tot = 0;
    if (b < nbk) {
        lo = base[b];
        tot = base[(uint64_t)nb * nbk + b] - lo;
        p = tot ? min(nb, (tot + target - 1) / target) : 0u;
    }
    s_p[b] = p;
    __syncthreads();
    for (uint32_t off = 1; off < kMaxBuckets; off <<= 1) {
        const uint32_t t = b >= off ? s_p[b - off] : 0u;
        __syncthreads();
        s_p[b] += t;
        __syncthreads();
    }
    const uint32_t first = s_p[b] - p;
    if (b == kMaxBuckets - 1) pieces[0] = min(s_p[b], cap);
    uint32_t c_prev = 0;
    for (uint32_t k = 0; k < p && first + k < cap; ++k) {
        uint32_t c_end = nb;
        if (k + 1 < p) {
            // first chunk whose run start reaches the piece's share of the bucket
            const uint32_t goal = lo + (uint32_t)(((uint64_t)tot * (k + 1)) / p);
            uint32_t l = c_prev, h = nb;
            while (l < h) {
                const uint32_t m = (l + h) >> 1;
                if (base[(uint64_t)m * nbk + b] >= goal) h = m;
                else l = m + 1;
            }
            c_end = l;
        }
        uint32_t* q = pieces + 1 + 3 * (first + k);
        q[0] = b;
        q[1] = c_prev;
        q[2] = c_end;
        c_prev = c_end;
    }
}

__global__ __launch_bounds__(kGroupThreads) void k_group_place_wide(
    const uint32_t* __restrict__ base, const uint32_t* __restrict__ H, uint32_t V, uint32_t S,
    uint32_t nbk, const uint32_t* __restrict__ pieces, const uint32_t* __restrict__ tmp,
    uint32_t* __restrict__ grouped, const uint32_t* __restrict__ ctl) {
    __shared__ uint32_t cur[kMaxBucketNodesWide];
    if (ctl[2]) return;
    const uint32_t nbits = 32u - __builtin_clz((V - 1u) | 1u);
    const uint32_t nmask = (1u << nbits) - 1u;
    const uint32_t np = pieces[0];
    for (uint32_t i = blockIdx.x; i < np; i += gridDim.x) {
        const uint32_t b = pieces[1 + 3 * i], c0 = pieces[2 + 3 * i], c1 = pieces[3 + 3 * i];
        if (c0 >= c1) continue;  // uniform over the block
        const uint32_t v0 = b << S, n = min(V, (b + 1) << S) - v0;
        const uint32_t* row = H + (uint64_t)c0 * V + v0;
        __syncthreads();  // the previous piece is done with the cursors
        for (uint32_t f = threadIdx.x; f < n; f += blockDim.x) cur[f] = row[f];
        __syncthreads();
        const uint32_t e1 = base[(uint64_t)c1 * nbk + b];
        for (uint32_t e0 = base[(uint64_t)c0 * nbk + b]; e0 < e1;
             e0 += kLoadBatch * blockDim.x) {
            uint32_t w[kLoadBatch];
#pragma unroll
            for (uint32_t k = 0; k < kLoadBatch; ++k) {
                const uint32_t e = e0 + threadIdx.x + k * blockDim.x;
                w[k] = e < e1 ? tmp[e] : kNone;
            }
#pragma unroll
            for (uint32_t k = 0; k < kLoadBatch; ++k)
                if (w[k] != kNone) grouped[atomicAdd(&cur[w[k] >> nbits], 1u)] = w[k] & nmask;
        }
    }
}

// Pass B for buckets of at most kStageNodes nodes, with whole-line writes: each
// node gathers its entries in a kStageWords-word LDS slot that is written out
// when full, ending at a 128-byte boundary of its run, so almost every line of
// the grouped array is written once and whole.  (Per-entry stores left partly
// written lines that L2 evicted early: about 3x the entry bytes written.)
// Entries beyond a slot's room within one batch (hub nodes) are stored at once,
// at consecutive positions taken from the node's cursor.  A node's run
// receives the same entries as from k_group_place_wide, in another order.
constexpr uint32_t kStageNodes = 1024;
constexpr uint32_t kStageWords = 32;  // one 128-byte line

__global__ __launch_bounds__(kGroupThreads) void k_group_place_staged(
    const uint32_t* __restrict__ base, const uint32_t* __restrict__ H, uint32_t V, uint32_t S,
    uint32_t nbk, const uint32_t* __restrict__ pieces, const uint32_t* __restrict__ tmp,
    uint32_t* __restrict__ grouped, const uint32_t* __restrict__ ctl) {
    __shared__ uint32_t cur[kStageNodes];   // next slot of each node's run
    __shared__ uint32_t fill[kStageNodes];  // entries claimed since the slot was last written
    __shared__ uint32_t room[kStageNodes];  // slot entries that end the run at a line boundary
    __shared__ uint32_t stage[kStageNodes * kStageWords];
    __shared__ uint32_t flist[kStageNodes], fpos[kStageNodes], fcnt[kStageNodes];
    __shared__ uint32_t s_nf;
    if (ctl[2]) return;
    const uint32_t tid = threadIdx.x, bd = blockDim.x;
    const uint32_t nbits = 32u - __builtin_clz((V - 1u) | 1u);
    const uint32_t nmask = (1u << nbits) - 1u;
    const uint32_t np = pieces[0];
    // write out the slots of the nodes whose fill reaches `need` (1: every
    // non-empty slot, at the end of a piece; else: full slots)
    auto flush = [&](uint32_t n, bool all) {
        if (tid == 0) s_nf = 0;
        lds_barrier();
        for (uint32_t f = tid; f < n; f += bd) {
            const uint32_t cnt = min(fill[f], room[f]);
            if (all ? cnt > 0 : cnt == room[f]) {
                const uint32_t k = atomicAdd(&s_nf, 1u);
                flist[k] = f;
                fpos[k] = cur[f];
                fcnt[k] = cnt;
                const uint32_t c = cur[f] + cnt;
                cur[f] = c;
                room[f] = kStageWords - c % kStageWords;
                fill[f] = 0;
            }
        }
        lds_barrier();
        const uint32_t nf = s_nf;
        for (uint32_t t = tid; t < nf * kStageWords; t += bd) {
            const uint32_t k = t / kStageWords, j = t % kStageWords;
            if (j < fcnt[k]) grouped[fpos[k] + j] = stage[flist[k] * kStageWords + j];
        }
        lds_barrier();  // the slots are refilled next
    };
    for (uint32_t i = blockIdx.x; i < np; i += gridDim.x) {
        const uint32_t b = pieces[1 + 3 * i], c0 = pieces[2 + 3 * i], c1 = pieces[3 + 3 * i];
        if (c0 >= c1) continue;  // uniform over the block
        const uint32_t v0 = b << S, n = min(V, (b + 1) << S) - v0;
        const uint32_t* row = H + (uint64_t)c0 * V + v0;
        for (uint32_t f = tid; f < n; f += bd) {
            const uint32_t c = row[f];
            cur[f] = c;
            fill[f] = 0;
            room[f] = kStageWords - c % kStageWords;
        }
        lds_barrier();
        const uint32_t e1 = base[(uint64_t)c1 * nbk + b];
        const uint32_t e_first = base[(uint64_t)c0 * nbk + b];
        uint32_t w[kLoadBatch];
#pragma unroll
        for (uint32_t k = 0; k < kLoadBatch; ++k) {
            const uint32_t e = e_first + tid + k * bd;
            w[k] = e < e1 ? tmp[e] : kNone;
        }
        for (uint32_t e0 = e_first; e0 < e1; e0 += kLoadBatch * bd) {
#pragma unroll
            for (uint32_t k = 0; k < kLoadBatch; ++k) {
                if (w[k] == kNone) continue;
                const uint32_t f = w[k] >> nbits, val = w[k] & nmask;
                const uint32_t s = atomicAdd(&fill[f], 1u);
                if (s < room[f]) stage[f * kStageWords + s] = val;
                else grouped[atomicAdd(&cur[f], 1u)] = val;
            }
            // the next batch's loads stay in flight through the slot writes
#pragma unroll
            for (uint32_t k = 0; k < kLoadBatch; ++k) {
                const uint32_t e = e0 + kLoadBatch * bd + tid + k * bd;
                w[k] = e < e1 ? tmp[e] : kNone;
            }
            lds_barrier();
            flush(n, false);
        }
        flush(n, true);
    }
}

// ------------------------------------------------------- scans (exclusive) --

constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kScanPerThread = 8;
constexpr uint32_t kScanTile = kScanThreads * kScanPerThread;
constexpr uint64_t kCountMask = (1ull << 40) - 1;

__device__ __forceinline__ uint64_t packed_of(uint32_t c, uint32_t chunk) {
    uint64_t items = (c + chunk - 1) / chunk;
    return (uint64_t)c | (items << 40);
}

// exclusive scan of 256 values in LDS (Hillis-Steele), returns this thread's prefix
template <typename T>
__device__ T block_exclusive_scan(T v, T* sh, T* total) {
    const uint32_t t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (uint32_t off = 1; off < kScanThreads; off <<= 1) {
        T add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    T incl = sh[t];
    *total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

// work items: exclusive scan of (entries | items << 40) per node, then every
// node emits ceil(entries / chunk) items
__global__ __launch_bounds__(kScanThreads) void k_scan_partial(const uint32_t* __restrict__ counts,
                                                                uint32_t T, uint32_t chunk,
                                                                uint64_t* __restrict__ block_sums) {
    __shared__ uint64_t sh[kScanThreads];
    uint64_t base = (uint64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPerThread;
    uint64_t s = 0;
    for (uint32_t k = 0; k < kScanPerThread; ++k) {
        uint64_t i = base + k;
        if (i < T) s += packed_of(counts[i], chunk);
    }
    uint64_t total;
    block_exclusive_scan<uint64_t>(s, sh, &total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// one workgroup: exclusive scan of the tile sums; publishes the item count and
// resets the work ticket
__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint64_t* __restrict__ block_sums,
                                                            uint32_t nblocks,
                                                            uint32_t* __restrict__ ctl) {
    __shared__ uint64_t sh[kScanThreads];
    uint64_t carry = 0;
    for (uint32_t b0 = 0; b0 < nblocks; b0 += kScanThreads) {
        uint32_t i = b0 + threadIdx.x;
        uint64_t v = i < nblocks ? block_sums[i] : 0;
        uint64_t total;
        uint64_t ex = block_exclusive_scan<uint64_t>(v, sh, &total);
        if (i < nblocks) block_sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        ctl[0] = 0;                           // ticket
        ctl[1] = (uint32_t)(carry >> 40);     // number of work items
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_items(
    const uint32_t* __restrict__ counts, uint32_t T, uint32_t chunk,
    const uint64_t* __restrict__ block_sums, WorkItem* __restrict__ items,
    uint32_t* __restrict__ nodeoff, const GraphDesc* __restrict__ gd, uint32_t G,
    const uint32_t* __restrict__ ctl) {
    __shared__ uint64_t sh[kScanThreads];
    uint64_t base = (uint64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPerThread;
    uint64_t vals[kScanPerThread];
    uint64_t s = 0;
    for (uint32_t k = 0; k < kScanPerThread; ++k) {
        uint64_t i = base + k;
        vals[k] = i < T ? packed_of(counts[i], chunk) : 0;
        s += vals[k];
    }
    uint64_t total;
    uint64_t pre = block_exclusive_scan<uint64_t>(s, sh, &total) + block_sums[blockIdx.x];
    const bool skip = ctl[2] != 0;
    for (uint32_t k = 0; k < kScanPerThread; ++k) {
        uint64_t i = base + k;
        if (i < T) nodeoff[i] = (uint32_t)(pre & kCountMask);
        if (i < T && !skip) {
            const uint32_t begin = (uint32_t)(pre & kCountMask);
            const uint32_t item0 = (uint32_t)(pre >> 40);
            const uint32_t c = (uint32_t)(vals[k] & kCountMask);
            const uint32_t ni = (uint32_t)(vals[k] >> 40);
            if (ni) {
                const uint32_t g = G == 1 ? 0u : graph_of_node(gd, G, (uint32_t)i);
                for (uint32_t j = 0; j < ni; ++j) {
                    WorkItem w;
                    w.begin = begin + j * chunk;
                    w.count = min(chunk, c - j * chunk);
                    w.gnode = (uint32_t)i;
                    w.graph = g;
                    w.shared = ni > 1 ? 1u : 0u;
                    w.split = 0;
                    items[item0 + j] = w;
                }
            }
        }
        pre += vals[k];
    }
}

__global__ void k_validate_nbrs(const uint32_t* __restrict__ nbrs, uint64_t count, uint32_t node,
                                uint32_t V, uint32_t* __restrict__ err) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) {
        uint32_t x = nbrs[i];
        if (x == node || x >= V) {
            atomicOr(&err[0], 1u);
            atomicOr(&err[1], 1u);
        }
    }
}

// ------------------------------------------------------------------- host --

namespace {

template <typename T>
gz_status grow(T** p, uint64_t need, const char* what) {
    if (*p) {
        // kernels of earlier calls may still read the old buffer
        GZ_HIP(hipDeviceSynchronize());
        GZ_HIP(hipFree(*p));
    }
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, std::max<uint64_t>(need, 1) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(GZ_ENOMEM, std::string("out of device memory for ") + what);
    }
    return GZ_OK;
}

template <typename T>
gz_status grow_host(T** p, uint64_t need) {
    if (*p) {
        GZ_HIP(hipDeviceSynchronize());
        GZ_HIP(hipHostFree(*p));
    }
    *p = nullptr;
    GZ_HIP(hipHostMalloc((void**)p, std::max<uint64_t>(need, 1) * sizeof(T), hipHostMallocDefault));
    return GZ_OK;
}

uint32_t grid_for(uint64_t n, uint32_t threads, uint32_t cap) {
    uint64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (uint32_t)b;
}


gz_status ensure_scratch(IngestScratch& S, uint64_t N, uint32_t T, uint32_t G, uint32_t chunk,
                         uint64_t H_size, uint32_t n_units, bool need_staging,
                         uint64_t bucket_entries = 0, uint64_t bbase_words = 0) {
    int dev = 0;
    GZ_HIP(hipGetDevice(&dev));
    if (S.device != -1 && S.device != dev) return fail(GZ_EINVAL, "graph used on another device");
    S.device = dev;
    if (!S.ctl) {
        GZ_HIP(hipMalloc((void**)&S.ctl, 8 * sizeof(uint32_t)));
        GZ_HIP(hipMemset(S.ctl, 0, 8 * sizeof(uint32_t)));
        GZ_HIP(hipMalloc((void**)&S.args, sizeof(IngestArgs)));
        GZ_HIP(hipEventCreateWithFlags(&S.copied_ev, hipEventDisableTiming));
        GZ_HIP(hipEventRecord(S.copied_ev, 0));
        GZ_HIP(hipEventCreateWithFlags(&S.done_ev, hipEventDisableTiming));
        GZ_HIP(hipEventRecord(S.done_ev, 0));
        GZ_TRY(grow_host(&S.h_args, 1));
        GZ_TRY(grow_host(&S.h_err, 4));
    }
    if (T > S.cap_nodes || !S.counts) {
        GZ_TRY(grow(&S.counts, T, "node counts"));
        GZ_TRY(grow(&S.cursor, T, "node offsets"));
        GZ_TRY(grow(&S.block_sums, (uint64_t)T / kScanTile + 2, "scan partials"));
        S.cap_nodes = T;
    }
    if (G > S.cap_graphs || !S.descs) {
        GZ_TRY(grow(&S.descs, G, "graph table"));
        GZ_TRY(grow_host(&S.h_descs, G));
        S.cap_graphs = G;
    }
    if (n_units > S.cap_units || !S.units) {
        GZ_TRY(grow(&S.units, n_units, "grouping units"));
        GZ_TRY(grow_host(&S.h_units, n_units));
        S.cap_units = n_units;
    }
    if (H_size + 1 > S.cap_H || !S.H) {
        GZ_TRY(grow(&S.H, H_size + 1, "grouping table"));
        S.cap_H = H_size + 1;
    }
    const uint64_t entries = 2 * N;
    if (entries > S.cap_updates || !S.grouped) {
        GZ_TRY(grow(&S.grouped, entries, "grouped updates"));
        S.cap_updates = entries;
    }
    const uint64_t items = (uint64_t)T + entries / chunk + 1;
    if (items > S.cap_items || !S.items) {
        GZ_TRY(grow(&S.items, items, "work items"));
        S.cap_items = items;
    }
    if (bucket_entries && (bucket_entries > S.cap_buckets || !S.buckets)) {
        GZ_TRY(grow(&S.buckets, bucket_entries, "bucket entries"));
        S.cap_buckets = bucket_entries;
    }
    if (bbase_words && (bbase_words > S.cap_bbase || !S.bbase)) {
        GZ_TRY(grow(&S.bbase, bbase_words, "bucket table"));
        S.cap_bbase = bbase_words;
    }
    if (need_staging && (2 * N > S.cap_staging || !S.staging)) {
        GZ_TRY(grow(&S.staging, 2 * N, "input staging"));
        S.cap_staging = 2 * N;
    }
    return GZ_OK;
}

}  // namespace

size_t update_smem_bytes(uint32_t lds_rows, uint32_t Bmax, uint32_t Pmax, bool wide) {
    // narrow graphs' update kernels stage small items' entries ahead of the tile
    const size_t stage = wide ? 0 : kItemStageWords;
    return (stage + (size_t)tile_rows(lds_rows, Bmax) * tile_row_words(Pmax, wide)) * 4;
}

gz_status set_smem_limit(const void* fn, size_t bytes) {
    if (bytes > 65536) GZ_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)bytes));
    return GZ_OK;
}

void free_ingest_scratch(IngestScratch& S) {
    hipFree(S.H); hipFree(S.units); hipFree(S.counts);
    hipFree(S.packed); hipFree(S.block_sums); hipFree(S.cursor);
    hipFree(S.grouped); hipFree(S.items); hipFree(S.ctl); hipFree(S.args); hipFree(S.offs);
    hipFree(S.descs); hipFree(S.staging); hipFree(S.buckets); hipFree(S.bbase);
    for (hipEvent_t ev : {S.copied_ev, S.done_ev})
        if (ev) {
            hipEventSynchronize(ev);
            hipEventDestroy(ev);
        }
    hipHostFree(S.h_args); hipHostFree(S.h_descs); hipHostFree(S.h_offs); hipHostFree(S.h_err);
    hipHostFree(S.h_units);
    S = IngestScratch{};
}

IngestScratch& shared_ingest_scratch(int device, std::unique_lock<std::mutex>& lock) {
    // never destroyed: nothing of the library is torn down by static destructors
    // at process exit (device memory still held then goes with the process)
    static std::mutex* mu = new std::mutex();
    static std::vector<IngestScratch>* per_dev = new std::vector<IngestScratch>(64);
    lock = std::unique_lock<std::mutex>(*mu);
    return (*per_dev)[(size_t)device % per_dev->size()];
}

// Static shape of a fused launch sequence: descriptor table, grouping units
// and launch parameters.  `ranges` gives each graph's update range [b, e) (the
// actual call, or the capacities of a captured plan).
struct LaunchShape {
    uint32_t G = 0, T = 0, n_units = 0, nblocks = 0, range_max = 1, pgrid = 0;
    uint32_t wg = 0, DLmax = 1, Pmax = 0, Bmax = 0, chunk = 0, lds_rows = 0, group_chunk = 0;
    uint64_t H_size = 0, N = 0;
    bool all_rows = true;
    // two-pass placement (single large graph): bucket shift, buckets, chunks,
    // chunks per pass-B block, pass-B blocks
    bool two_pass = false;
    // sorted one-pass placement (every graph of at most kSortNodes nodes):
    // updates per batch, dynamic LDS bytes
    bool sorted = false;
    uint32_t sbatch = 0;
    size_t ssmem = 0;
    bool wide = false;  // graphs with V > 2^16 (pair-keyed hashes, four planes)
    uint32_t bS = 0, nbk = 0, nbc = 0, bcr = 1, bblocks = 0;
    uint32_t ptarget = 0, pcap = 0;  // wide pass B: entries per piece, piece capacity
    size_t gsmem = 0, smem = 0;
    std::vector<GraphDesc> descs;
    std::vector<GroupUnit> units;
};

constexpr uint64_t kTableWords = 1ull << 28;

gz_status build_shape(gz_graph* const* gs, uint32_t G, const uint64_t* ranges, uint64_t N,
                      LaunchShape& L) {
    const gz_tuning tune = gs[0]->tuning;
    L = LaunchShape{};
    L.G = G;
    L.N = N;
    L.chunk = tune.chunk;
    L.lds_rows = tune.lds_rows;
    L.wg = tune.wg_size;
    // grouping blocks: about one per CU over the whole call (at least 8192 updates
    // each) unless tuned otherwise
    const uint32_t cus = (uint32_t)device_cu_count();
    const uint32_t gblocks = tune.group_blocks ? tune.group_blocks : cus;
    uint64_t gchunk = std::max<uint64_t>(8192, (N + gblocks - 1) / gblocks);
    if (gs[0] && gs[0]->wide) {
        // the (chunk, node) count table holds V words per chunk: graphs with
        // millions of nodes take fewer, longer chunks so that it stays within
        // 2^28 words
        uint64_t vsum = 0;
        for (uint32_t k = 0; k < G; ++k) vsum += gs[k] ? gs[k]->V : 0;
        gchunk = std::max<uint64_t>(gchunk, (N * vsum + kTableWords - 1) / kTableWords);
    }
    L.group_chunk = (uint32_t)gchunk;
    L.descs.resize(G);
    uint64_t T = 0;
    for (uint32_t k = 0; k < G; ++k) {
        const gz_graph* g = gs[k];
        if (!g) return fail(GZ_EINVAL, "null graph handle");
        const uint64_t b = ranges[k], e = ranges[k + 1];
        GraphDesc& d = L.descs[k];
        d = GraphDesc{};
        d.sk = g->sk;
        d.seeds = g->seeds;
        d.n = g->n;
        d.V = g->V;
        d.R = g->R;
        d.B = g->B;
        d.P = g->P;
        d.node_base = (uint32_t)T;
        d.node_words = g->planes * g->B * g->P;
        d.wide = g->wide;
        d.planes = g->planes;
        d.err = g->err;
        d.upd_base = b;
        d.nb = (uint32_t)((e - b + L.group_chunk - 1) / L.group_chunk);
        d.hoff = L.H_size;
        const uint32_t nq = (g->V + kGroupRange - 1) / kGroupRange;
        for (uint32_t c = 0; c < d.nb; ++c)
            for (uint32_t q = 0; q < nq; ++q) L.units.push_back(GroupUnit{k, c, q, 0});
        L.H_size += (uint64_t)g->V * d.nb;
        T += g->V;
        L.Pmax = std::max(L.Pmax, g->P);
        L.Bmax = std::max(L.Bmax, g->B);
        L.DLmax = std::max(L.DLmax, std::min(tune.lds_rows, g->B));
        L.all_rows = L.all_rows && tune.lds_rows >= g->B;
        L.range_max = std::max(L.range_max, std::min(g->V, kGroupRange));
    }
    if (T >= (1ull << 32)) return fail(GZ_EINVAL, "too many nodes in one call");
    if (L.H_size >= (1ull << 32)) return fail(GZ_EINVAL, "call too large: split the stream");
    if (L.wg < L.Pmax || L.wg % 64 || L.wg > 1024)
        return fail(GZ_EINVAL, "workgroup smaller than pairs");
    L.wide = gs[0]->wide;
    for (uint32_t k = 1; k < G; ++k)
        if (gs[k]->wide != L.wide)
            return fail(GZ_EINVAL, "one call takes graphs of one kind (V <= 65536, or larger)");
    L.T = (uint32_t)T;
    L.n_units = (uint32_t)L.units.size();
    // single graphs large enough that one-pass placement would keep too many
    // runs open per block take the two-pass placement
    if (G == 1 && gs[0]->V > 4096 && gs[0]->V <= kMaxTwoPassWide && L.descs[0].nb > 0) {
        L.two_pass = true;
        while (((gs[0]->V + (1u << L.bS) - 1) >> L.bS) > kMaxBuckets) ++L.bS;
        L.nbk = (gs[0]->V + (1u << L.bS) - 1) >> L.bS;
        L.nbc = L.descs[0].nb;
        const uint32_t per_bucket = std::max(1u, 4 * cus / L.nbk);
        L.bcr = (L.nbc + per_bucket - 1) / per_bucket;
        L.bblocks = L.nbk * ((L.nbc + L.bcr - 1) / L.bcr);
        if (L.wide) {
            L.ptarget = (uint32_t)std::max<uint64_t>(65536, (2 * N + 2 * cus - 1) / (2 * cus));
            L.pcap = L.nbk + (uint32_t)((2 * N + L.ptarget - 1) / L.ptarget) + 1;
        }
    }
    if (!L.two_pass && !L.wide && L.n_units && L.range_max <= kSortNodes &&
        sort_batch(L.range_max) > 0) {
        L.sorted = true;
        L.sbatch = sort_batch(L.range_max);
        L.ssmem = sort_smem(L.range_max);
        GZ_TRY(set_smem_limit((const void*)k_group_scatter_sorted, L.ssmem));
    }
    L.nblocks = (uint32_t)((T + kScanTile - 1) / kScanTile);
    L.gsmem = (size_t)L.range_max * 4;
    L.smem = update_smem_bytes(tune.lds_rows, L.Bmax, L.Pmax, L.wide);
    L.pgrid = std::max(1u, tune.wgs_per_cu) * cus;
    GZ_TRY(set_smem_limit((const void*)k_group_count, L.gsmem));
    GZ_TRY(set_smem_limit((const void*)k_group_scatter, L.gsmem));
    GZ_TRY(set_smem_limit(L.wide ? (const void*)k_update_wide : (const void*)k_update, L.smem));
    return GZ_OK;
}

// upload the shape's static tables (descriptors, grouping units)
gz_status upload_shape(IngestScratch& S, const LaunchShape& L, hipStream_t stream) {
    std::memcpy(S.h_descs, L.descs.data(), sizeof(GraphDesc) * L.G);
    if (L.n_units) std::memcpy(S.h_units, L.units.data(), sizeof(GroupUnit) * L.n_units);
    GZ_HIP(hipMemcpyAsync(S.descs, S.h_descs, sizeof(GraphDesc) * L.G, hipMemcpyHostToDevice,
                          stream));
    if (L.n_units)
        GZ_HIP(hipMemcpyAsync(S.units, S.h_units, sizeof(GroupUnit) * L.n_units,
                              hipMemcpyHostToDevice, stream));
    return GZ_OK;
}

// The device-side sequence of one fused ingest: every argument it reads per
// call (inputs, N, offsets) comes from S.args, so the sequence can be captured
// once and replayed.  The profiling events mark the start of grouping and the
// start and end of the sketch update when `prof` is given.
gz_status launch_sequence(IngestScratch& S, const LaunchShape& L, hipStream_t stream,
                          gz_graph* prof, bool with_update = true) {
    const uint32_t Tn = L.T;
    if (prof) GZ_HIP(hipEventRecord(prof->prof_ev[0], stream));
    k_fill_u32<<<1, 64, 0, stream>>>(S.ctl, 3, 0);  // ticket, items, call error (sticky kept)
    const bool wide2 = L.two_pass && L.wide;
    if (wide2) {
        // buckets first: counts, regions, pass A, then node counts from its output
        k_group_bcount<<<L.nbc, kGroupThreads, 0, stream>>>(S.args, S.descs, L.bS, L.nbk, S.H,
                                                            S.ctl);
        k_group_bbase_wide<<<1, kMaxBuckets, 0, stream>>>(S.H, L.nbk, L.nbc, S.bbase);
        k_group_partition<<<L.nbc, kGroupThreads, 0, stream>>>(S.args, S.descs, S.bbase, L.bS,
                                                               L.nbk, S.buckets, S.ctl);
        k_group_ncount<<<L.nbk * L.nbc, 256, 0, stream>>>(S.bbase, L.nbk, L.bS, Tn, S.buckets,
                                                          S.H, S.ctl);
    } else if (L.n_units) {
        k_group_count<<<L.n_units, kGroupThreads, L.gsmem, stream>>>(S.args, S.units, S.descs,
                                                                     S.H, S.ctl);
    }
    k_group_colsum<<<grid_for((uint64_t)Tn * kColLanes, 256, 16384), 256, 0, stream>>>(
        S.descs, L.G, Tn, S.H, S.counts);
    k_scan_partial<<<L.nblocks, kScanThreads, 0, stream>>>(S.counts, Tn, L.chunk, S.block_sums);
    k_scan_top<<<1, kScanThreads, 0, stream>>>(S.block_sums, L.nblocks, S.ctl);
    k_scan_items<<<L.nblocks, kScanThreads, 0, stream>>>(S.counts, Tn, L.chunk, S.block_sums,
                                                         S.items, S.cursor, S.descs, L.G, S.ctl);
    k_group_colscan<<<grid_for((uint64_t)Tn * kColLanes, 256, 16384), 256, 0, stream>>>(
        S.descs, L.G, Tn, S.cursor, S.H);
    if (wide2) {
        uint32_t* pieces = S.bbase + (uint64_t)(L.nbc + 1) * L.nbk;
        k_group_pieces<<<1, kMaxBuckets, 0, stream>>>(S.bbase, L.nbk, L.nbc, L.ptarget, L.pcap,
                                                      pieces, S.ctl);
        // one workgroup per CU: each keeps a bucket's node runs open, and two
        // per CU overflowed L2 with partly written lines (11.6 -> 11.1 ms of
        // grouping on 2^18 nodes)
        if ((1u << L.bS) <= kStageNodes)
            k_group_place_staged<<<device_cu_count(), kGroupThreads, 0, stream>>>(
                S.bbase, S.H, Tn, L.bS, L.nbk, pieces, S.buckets, S.grouped, S.ctl);
        else
            k_group_place_wide<<<device_cu_count(), kGroupThreads, 0, stream>>>(
                S.bbase, S.H, Tn, L.bS, L.nbk, pieces, S.buckets, S.grouped, S.ctl);
    } else if (L.two_pass) {
        const uint32_t nbase = (L.nbc + 1) * L.nbk;
        k_group_bucket_base<<<(nbase + 255) / 256, 256, 0, stream>>>(
            S.H, S.cursor, S.counts, Tn, L.bS, L.nbk, L.nbc, S.bbase);
        k_group_partition<<<L.nbc, kGroupThreads, 0, stream>>>(S.args, S.descs, S.bbase, L.bS,
                                                               L.nbk, S.buckets, S.ctl);
        k_group_place<<<L.bblocks, kGroupThreads, 0, stream>>>(
            S.bbase, S.H, Tn, L.bS, L.nbk, L.nbc, L.bcr, S.buckets, S.grouped, S.ctl);
    } else if (L.sorted) {
        k_group_scatter_sorted<<<L.n_units, kGroupThreads, L.ssmem, stream>>>(
            S.args, S.units, S.descs, S.H, S.grouped, S.ctl, L.range_max, L.sbatch);
    } else if (L.n_units) {
        k_group_scatter<<<L.n_units, kGroupThreads, L.gsmem, stream>>>(S.args, S.units, S.descs,
                                                                       S.H, S.grouped, S.ctl);
    }
    if (L.wide)  // neighbours below each item's node first, into the bucket array
        k_split_items<<<8 * device_cu_count(), 256, 0, stream>>>(S.ctl, S.items, S.grouped,
                                                                 S.buckets, S.descs);
    if (prof) GZ_HIP(hipEventRecord(prof->prof_ev[1], stream));
    if (with_update && L.wide)
        k_update_wide<<<L.pgrid, L.wg, L.smem, stream>>>(S.items, S.ctl, update_entries(S, true),
                                                         S.descs, L.lds_rows);
    else if (with_update)
        k_update<<<L.pgrid, L.wg, L.smem, stream>>>(S.items, S.ctl, S.grouped, S.descs,
                                                    L.lds_rows);
    GZ_HIP(hipGetLastError());
    if (prof) {
        GZ_HIP(hipEventRecord(prof->prof_ev[2], stream));
        prof->prof_calls++;
    }
    return GZ_OK;
}

// Wait until the previous call's uploads have left the pinned argument buffer.
// The runtime has been seen to report this event as recorded in a capturing
// stream (it never is: it is recorded on the caller's stream, outside any
// capture) after a long sequence of calls that included plan captures; the
// wait then falls back to a device synchronization and a fresh event.
gz_status wait_uploads(IngestScratch& S) {
    const hipError_t e = hipEventSynchronize(S.copied_ev);
    if (e != hipErrorCapturedEvent) {
        GZ_HIP(e);
        return GZ_OK;
    }
    (void)hipGetLastError();
    GZ_HIP(hipDeviceSynchronize());
    GZ_HIP(hipEventDestroy(S.copied_ev));
    S.copied_ev = nullptr;
    GZ_HIP(hipEventCreateWithFlags(&S.copied_ev, hipEventDisableTiming));
    return GZ_OK;
}

// per-call arguments through the pinned buffer, reused once the previous
// call's uploads have left it
gz_status upload_args(IngestScratch& S, const LaunchShape& L, const uint32_t* src,
                      const uint32_t* dst, uint64_t N, const uint64_t* offs_dev,
                      hipStream_t stream) {
    GZ_TRY(wait_uploads(S));
    IngestArgs& a = *S.h_args;
    a = IngestArgs{};
    a.src = src;
    a.dst = dst;
    a.offs = offs_dev;
    a.N = N;
    a.G = L.G;
    a.T = L.T;
    a.chunk = L.chunk;
    a.lds_rows = L.lds_rows;
    a.group_chunk = L.group_chunk;
    a.n_units = L.n_units;
    a.H_size = L.H_size;
    GZ_HIP(hipMemcpyAsync(S.args, S.h_args, sizeof(IngestArgs), hipMemcpyHostToDevice, stream));
    return GZ_OK;
}

gz_status check_call_error(IngestScratch& S, hipStream_t stream) {
    GZ_HIP(hipMemcpyAsync(S.h_err, S.ctl + 2, 4, hipMemcpyDeviceToHost, stream));
    GZ_HIP(hipStreamSynchronize(stream));
    if (S.h_err[0]) return fail(GZ_EINVAL, "invalid update (self-loop or node id out of range)");
    return GZ_OK;
}

// An asynchronous call reports an invalid update at each of its graphs' next
// flush: the call's error word is copied into every graph's own word.
gz_status note_async_error(IngestScratch& S, gz_graph* const* gs, uint32_t G, hipStream_t stream) {
    k_note_error<<<(G + 255) / 256, 256, 0, stream>>>(S.descs, G, S.ctl + 2);
    GZ_HIP(hipGetLastError());
    for (uint32_t k = 0; k < G; ++k) gs[k]->pending_error = true;  // flush must check
    return GZ_OK;
}

gz_status ingest_fused(gz_graph* const* gs, uint32_t G, const uint64_t* offs_host,
                       const uint32_t* src, const uint32_t* dst, uint64_t N, uint32_t flags,
                       hipStream_t stream, IngestScratch& S) {
    if (G == 0) return fail(GZ_EINVAL, "no graphs");
    for (uint32_t k = 0; k < G; ++k)
        if (gs[k]->tier) {
            if (G > 1) return fail(GZ_EINVAL, "host-tier graphs are ingested one call each");
            return tier_ingest(gs[0], src, dst, N, flags, stream);
        }
    if (N >= (1ull << 31)) return fail(GZ_EINVAL, "at most 2^31-1 updates per call");
    if (N && (!src || !dst)) return fail(GZ_EINVAL, "null stream arrays");
    std::vector<uint64_t> ranges(G + 1, 0);
    if (offs_host) {
        if (offs_host[0] != 0 || offs_host[G] != N)
            return fail(GZ_EINVAL, "update offsets must start at 0 and end at N");
        for (uint32_t k = 0; k < G; ++k)
            if (offs_host[k + 1] < offs_host[k])
                return fail(GZ_EINVAL, "update offsets must be non-decreasing");
        std::memcpy(ranges.data(), offs_host, sizeof(uint64_t) * (G + 1));
    } else {
        ranges[G] = N;
        for (uint32_t k = 1; k < G; ++k) ranges[k] = N;
    }
    LaunchShape L;
    GZ_TRY(build_shape(gs, G, ranges.data(), N, L));
    const bool host_ptr = !(flags & GZ_DEVICE_PTR);
    GZ_TRY(ensure_scratch(S, N, L.T, G, L.chunk, L.H_size, L.n_units, host_ptr,
                          L.two_pass || L.wide ? 2 * N : 0,
                          L.two_pass ? (uint64_t)(L.nbc + 1) * L.nbk + 1 + 3ull * L.pcap : 0));

    // order after earlier work on these graphs (e.g. a query on another stream),
    // and after the kernels of the previous call that used this scratch, on
    // whatever stream it ran
    GZ_HIP(fence_wait(stream, gs, G));
    GZ_HIP(hipStreamWaitEvent(stream, S.done_ev, 0));

    const uint32_t* dsrc = src;
    const uint32_t* ddst = dst;
    if (host_ptr && N) {
        GZ_HIP(hipMemcpyAsync(S.staging, src, N * 4, hipMemcpyHostToDevice, stream));
        GZ_HIP(hipMemcpyAsync(S.staging + N, dst, N * 4, hipMemcpyHostToDevice, stream));
        dsrc = S.staging;
        ddst = S.staging + N;
    }
    GZ_TRY(upload_args(S, L, dsrc, ddst, N, nullptr, stream));
    GZ_TRY(upload_shape(S, L, stream));
    GZ_HIP(hipEventRecord(S.copied_ev, stream));
    GZ_TRY(launch_sequence(S, L, stream, gs[0]->profiling ? gs[0] : nullptr));
    if (flags & GZ_ASYNC) GZ_TRY(note_async_error(S, gs, G, stream));
    GZ_HIP(hipEventRecord(S.done_ev, stream));
    GZ_HIP(fence_record(stream, gs, G));
    if (!(flags & GZ_ASYNC)) return check_call_error(S, stream);
    return GZ_OK;
}

gz_status group_only(gz_graph* g, const uint32_t* src, const uint32_t* dst, uint64_t N,
                     uint32_t flags, hipStream_t stream, UpdateLaunch* out) {
    if (N >= (1ull << 31)) return fail(GZ_EINVAL, "at most 2^31-1 updates per call");
    if (N && (!src || !dst)) return fail(GZ_EINVAL, "null stream arrays");
    IngestScratch& S = g->ing;
    const uint64_t ranges[2] = {0, N};
    gz_graph* gs[1] = {g};
    LaunchShape L;
    GZ_TRY(build_shape(gs, 1, ranges, N, L));
    const bool host_ptr = !(flags & GZ_DEVICE_PTR);
    GZ_TRY(ensure_scratch(S, N, L.T, 1, L.chunk, L.H_size, L.n_units, host_ptr,
                          L.two_pass || L.wide ? 2 * N : 0,
                          L.two_pass ? (uint64_t)(L.nbc + 1) * L.nbk + 1 + 3ull * L.pcap : 0));
    GZ_HIP(fence_wait(stream, g));
    const uint32_t* dsrc = src;
    const uint32_t* ddst = dst;
    if (host_ptr && N) {
        GZ_HIP(hipMemcpyAsync(S.staging, src, N * 4, hipMemcpyHostToDevice, stream));
        GZ_HIP(hipMemcpyAsync(S.staging + N, dst, N * 4, hipMemcpyHostToDevice, stream));
        dsrc = S.staging;
        ddst = S.staging + N;
    }
    GZ_TRY(upload_args(S, L, dsrc, ddst, N, nullptr, stream));
    GZ_TRY(upload_shape(S, L, stream));
    GZ_HIP(hipEventRecord(S.copied_ev, stream));
    GZ_TRY(launch_sequence(S, L, stream, nullptr, false));
    GZ_TRY(check_call_error(S, stream));
    out->wg = L.wg;
    out->grid = L.pgrid;
    out->smem = L.smem;
    out->lds_rows = L.lds_rows;
    out->wide = L.wide;
    return GZ_OK;
}

gz_status update_node_batch(gz_graph* g, uint32_t node, const uint32_t* nbrs, uint64_t count,
                            uint32_t flags, hipStream_t stream) {
    if (node >= g->V) return fail(GZ_EINVAL, "node id out of range");
    if (count == 0) return GZ_OK;
    if (!nbrs) return fail(GZ_EINVAL, "null neighbour array");
    if (count >= (1ull << 31)) return fail(GZ_EINVAL, "batch too large");
    IngestScratch& S = g->ing;
    const gz_tuning tune = g->tuning;
    const bool host_ptr = !(flags & GZ_DEVICE_PTR);
    if (host_ptr) {
        for (uint64_t k = 0; k < count; ++k)
            if (nbrs[k] == node || nbrs[k] >= g->V)
                return fail(GZ_EINVAL, "invalid neighbour (self-loop or id out of range)");
    }
    GZ_TRY(ensure_scratch(S, 0, g->V, 1, tune.chunk, 0, 0, false));
    GZ_HIP(fence_wait(stream, g));
    const uint32_t* d = nbrs;
    if (host_ptr) {
        if (count > S.cap_staging || !S.staging) {
            GZ_TRY(grow(&S.staging, count, "input staging"));
            S.cap_staging = count;
        }
        GZ_HIP(hipMemcpyAsync(S.staging, nbrs, count * 4, hipMemcpyHostToDevice, stream));
        d = S.staging;
    }
    // ctl[2]: the call's error word, as in the fused path
    const bool check = !(flags & GZ_UNCHECKED);
    if (check) k_fill_u32<<<1, 64, 0, stream>>>(S.ctl + 2, 1, 0);
    if (!host_ptr && check)
        k_validate_nbrs<<<grid_for(count, 256, 1024), 256, 0, stream>>>(d, count, node, g->V,
                                                                       S.ctl + 2);
    // unchecked calls point the kernel at ctl[4], a word nothing ever sets
    const uint32_t* errp = check ? S.ctl + 2 : S.ctl + 4;
    if (g->tier) {
        GZ_TRY(tier_update_node(g, node, d, (uint32_t)count, errp, stream));
    } else {
        GraphDesc gd{};
        gd.sk = g->sk;
        gd.seeds = g->seeds;
        gd.n = g->n;
        gd.V = g->V;
        gd.R = g->R;
        gd.B = g->B;
        gd.P = g->P;
        gd.node_words = g->planes * g->B * g->P;
        gd.wide = g->wide;
        gd.planes = g->planes;
        gd.err = g->err;
        // pieces of node_chunk entries, one workgroup each; by default the
        // batch is spread over about one workgroup per CU (at least 64 entries
        // a piece, below which the merge atomics outweigh the entries)
        const uint64_t cus = (uint64_t)device_cu_count();
        const uint32_t chunk =
            tune.node_chunk ? tune.node_chunk
                            : (uint32_t)std::max<uint64_t>(64, (count + cus - 1) / cus);
        const uint32_t DL = std::min(tune.lds_rows, g->B);
        const size_t smem = update_smem_bytes(tune.lds_rows, g->B, g->P, g->wide);
        const void* fn = g->wide ? (const void*)k_update_node_wide : (const void*)k_update_node;
        GZ_TRY(set_smem_limit(fn, smem));
        const uint32_t grid = (uint32_t)((count + chunk - 1) / chunk);
        if (g->wide)
            k_update_node_wide<<<grid, tune.wg_size, smem, stream>>>(d, (uint32_t)count, node, gd,
                                                                       tune.lds_rows, chunk, errp);
        else
            k_update_node<<<grid, tune.wg_size, smem, stream>>>(d, (uint32_t)count, node, gd,
                                                                  tune.lds_rows, chunk, errp);
    }
    GZ_HIP(hipGetLastError());
    GZ_HIP(fence_record(stream, g));
    if (!host_ptr && check) {
        if (!(flags & GZ_ASYNC)) {
            GZ_HIP(hipMemcpyAsync(S.h_err, S.ctl + 2, 4, hipMemcpyDeviceToHost, stream));
            GZ_HIP(hipStreamSynchronize(stream));
            if (S.h_err[0]) return fail(GZ_EINVAL, "invalid neighbour (self-loop or id out of range)");
        } else {
            k_note_error_one<<<1, 64, 0, stream>>>(g->err, S.ctl + 2);
            GZ_HIP(hipGetLastError());
            g->pending_error = true;
        }
    } else if (host_ptr) {
        // the host copy must finish before the caller may reuse its buffer
        GZ_HIP(hipStreamSynchronize(stream));
    }
    return GZ_OK;
}

// ------------------------------------------------- ingest without allocation --

// Per-call tables of a no-allocation ingest, written into the caller-provided
// scratch by a kernel that takes them by value (no host staging buffer).
__global__ void k_noalloc_setup(IngestArgs a, GraphDesc d, uint32_t nq, uint32_t n_units,
                                IngestArgs* __restrict__ args, GraphDesc* __restrict__ descs,
                                GroupUnit* __restrict__ units, uint32_t* __restrict__ ctl) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        *args = a;
        descs[0] = d;
    }
    if (t < 8) ctl[t] = 0;
    for (uint32_t i = t; i < n_units; i += gridDim.x * blockDim.x)
        units[i] = GroupUnit{0u, i / nq, i % nq, 0u};
}

namespace {
// the next 256-byte aligned region of `bytes` in [base, base + cap), or null when it
// does not fit (`*at` still advances, so the caller learns the bytes needed)
template <typename T>
T* carve(uint8_t* base, size_t cap, size_t* at, uint64_t count) {
    const size_t start = (*at + 255) & ~(size_t)255;
    *at = start + (size_t)std::max<uint64_t>(count, 1) * sizeof(T);
    return *at <= cap ? reinterpret_cast<T*>(base + start) : nullptr;
}
}  // namespace

gz_status ingest_noalloc(gz_graph* g, const uint32_t* src, const uint32_t* dst, uint64_t N,
                         uint32_t flags, hipStream_t stream, uint8_t* scratch, size_t cap) {
    if (g->tier) return fail(GZ_EINVAL, "gz_ingest_noalloc takes graphs whose sketches live in HBM");
    if (!(flags & GZ_DEVICE_PTR)) return fail(GZ_EINVAL, "gz_ingest_noalloc takes device arrays");
    if (N >= (1ull << 31)) return fail(GZ_EINVAL, "at most 2^31-1 updates per call");
    if (N == 0) return GZ_OK;
    if (!src || !dst) return fail(GZ_EINVAL, "null stream arrays");
    gz_graph* gs[1] = {g};
    const uint64_t ranges[2] = {0, N};
    LaunchShape L;
    GZ_TRY(build_shape(gs, 1, ranges, N, L));
    // the scratch laid out as ensure_scratch would allocate it for this call
    IngestScratch S{};
    size_t at = 0;
    const uint32_t T = L.T;
    S.ctl = carve<uint32_t>(scratch, cap, &at, 8);
    S.args = carve<IngestArgs>(scratch, cap, &at, 1);
    S.descs = carve<GraphDesc>(scratch, cap, &at, 1);
    S.units = carve<GroupUnit>(scratch, cap, &at, L.n_units);
    S.counts = carve<uint32_t>(scratch, cap, &at, T);
    S.cursor = carve<uint32_t>(scratch, cap, &at, T);
    S.block_sums = carve<uint64_t>(scratch, cap, &at, (uint64_t)T / kScanTile + 2);
    S.H = carve<uint32_t>(scratch, cap, &at, L.H_size + 1);
    S.grouped = carve<uint32_t>(scratch, cap, &at, 2 * N);
    S.items = carve<WorkItem>(scratch, cap, &at, (uint64_t)T + 2 * N / L.chunk + 1);
    if (L.two_pass || L.wide) S.buckets = carve<uint32_t>(scratch, cap, &at, 2 * N);
    if (L.two_pass)
        S.bbase = carve<uint32_t>(scratch, cap, &at, (uint64_t)(L.nbc + 1) * L.nbk + 1 + 3ull * L.pcap);
    if (at > cap)
        return fail(GZ_EINVAL, "gz_ingest_noalloc: this call needs " + std::to_string(at) +
                                   " bytes of scratch, more than the " + std::to_string(cap) +
                                   " the library keeps per device; split the stream into "
                                   "smaller calls");
    IngestArgs a{};
    a.src = src;
    a.dst = dst;
    a.offs = nullptr;
    a.N = N;
    a.G = 1;
    a.T = L.T;
    a.chunk = L.chunk;
    a.lds_rows = L.lds_rows;
    a.group_chunk = L.group_chunk;
    a.n_units = L.n_units;
    a.H_size = L.H_size;
    const uint32_t nq = (g->V + kGroupRange - 1) / kGroupRange;
    GZ_HIP(fence_wait(stream, g));
    k_noalloc_setup<<<grid_for(L.n_units, 256, 1024), 256, 0, stream>>>(
        a, L.descs[0], nq, L.n_units, S.args, S.descs, S.units, S.ctl);
    GZ_HIP(hipGetLastError());
    GZ_TRY(launch_sequence(S, L, stream, g->profiling ? g : nullptr));
    GZ_TRY(note_async_error(S, gs, 1, stream));
    GZ_HIP(fence_record(stream, g));
    return GZ_OK;
}

}  // namespace gz

// ------------------------------------------------------ captured ingest plan --

struct gz_plan {
    std::vector<gz_graph*> gs;
    std::vector<uint64_t> caps;
    gz::IngestScratch S;
    gz::LaunchShape L;
    uint64_t* offs_dev = nullptr;
    uint64_t* h_offs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
};

using namespace gz;

extern "C" {

gz_status gz_plan_create(gz_graph* const* gs, uint32_t G, const uint64_t* caps, hipStream_t stream,
                         gz_plan** out) {
    if (!out || !gs || !caps || G == 0) return fail(GZ_EINVAL, "null argument");
    *out = nullptr;
    std::vector<uint64_t> ranges(G + 1, 0);
    if (bad_graph_list(gs, G)) return fail(GZ_EINVAL, "null graph handle or graph listed twice");
    for (uint32_t k = 0; k < G; ++k)
        if (gs[k]->tier) return fail(GZ_EINVAL, "plans take graphs whose sketches live in HBM");
    for (uint32_t k = 0; k < G; ++k) ranges[k + 1] = ranges[k] + caps[k];
    if (ranges[G] >= (1ull << 31)) return fail(GZ_EINVAL, "capacities sum to 2^31 or more");
    gz_plan* p = new gz_plan();
    p->gs.assign(gs, gs + G);
    p->caps.assign(caps, caps + G);
    gz_status st = build_shape(gs, G, ranges.data(), ranges[G], p->L);
    if (!st)
        st = ensure_scratch(p->S, ranges[G], p->L.T, G, p->L.chunk, p->L.H_size, p->L.n_units,
                            false, p->L.two_pass || p->L.wide ? 2 * ranges[G] : 0,
                            p->L.two_pass ? (uint64_t)(p->L.nbc + 1) * p->L.nbk + 1 +
                                                3ull * p->L.pcap
                                          : 0);
    hipError_t e = hipSuccess;
    if (!st) {
        e = hipMalloc((void**)&p->offs_dev, sizeof(uint64_t) * (G + 1));
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&p->h_offs, sizeof(uint64_t) * (G + 1), hipHostMallocDefault);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) st = hip_fail(e, "plan buffers");
    }
    if (!st) st = upload_shape(p->S, p->L, stream);
    if (!st) {
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) st = hip_fail(e, "plan upload");
    }
    if (!st) {
        e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) st = hip_fail(e, "begin capture");
        if (!st) {
            gz_status lst = launch_sequence(p->S, p->L, p->cap_stream, nullptr);
            e = hipStreamEndCapture(p->cap_stream, &p->graph);
            if (lst) st = lst;
            else if (e != hipSuccess) st = hip_fail(e, "end capture");
        }
        if (!st) {
            e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) st = hip_fail(e, "graph instantiate");
        }
    }
    if (st) {
        gz_plan_free(p);
        return st;
    }
    *out = p;
    return GZ_OK;
}

gz_status gz_plan_ingest(gz_plan* p, const uint64_t* offs, const uint32_t* src, const uint32_t* dst,
                         uint32_t flags, hipStream_t stream) {
    if (!p || !offs) return fail(GZ_EINVAL, "null argument");
    if (!(flags & GZ_DEVICE_PTR)) return fail(GZ_EINVAL, "plans take device arrays");
    const uint32_t G = (uint32_t)p->gs.size();
    if (offs[0] != 0) return fail(GZ_EINVAL, "update offsets must start at 0");
    for (uint32_t k = 0; k < G; ++k) {
        if (offs[k + 1] < offs[k]) return fail(GZ_EINVAL, "update offsets must be non-decreasing");
        if (offs[k + 1] - offs[k] > p->caps[k])
            return fail(GZ_EINVAL, "a graph's updates exceed its capacity in the plan");
    }
    const uint64_t N = offs[G];
    if (N && (!src || !dst)) return fail(GZ_EINVAL, "null stream arrays");
    IngestScratch& S = p->S;
    GZ_HIP(fence_wait(stream, p->gs.data(), G));
    GZ_TRY(upload_args(S, p->L, src, dst, N, p->offs_dev, stream));
    std::memcpy(p->h_offs, offs, sizeof(uint64_t) * (G + 1));
    GZ_HIP(hipMemcpyAsync(p->offs_dev, p->h_offs, sizeof(uint64_t) * (G + 1),
                          hipMemcpyHostToDevice, stream));
    GZ_HIP(hipEventRecord(S.copied_ev, stream));
    GZ_HIP(hipGraphLaunch(p->exec, stream));
    if (flags & GZ_ASYNC) GZ_TRY(note_async_error(S, p->gs.data(), G, stream));
    GZ_HIP(fence_record(stream, p->gs.data(), G));
    if (!(flags & GZ_ASYNC)) return check_call_error(S, stream);
    return GZ_OK;
}

gz_status gz_plan_free(gz_plan* p) {
    if (!p) return GZ_OK;
    if (p->cap_stream) hipStreamSynchronize(p->cap_stream);
    if (p->S.copied_ev) hipEventSynchronize(p->S.copied_ev);
    for (gz_graph* g : p->gs)
        if (g && g->last) hipEventSynchronize(g->last->ev);
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->cap_stream) hipStreamDestroy(p->cap_stream);
    hipFree(p->offs_dev);
    hipHostFree(p->h_offs);
    free_ingest_scratch(p->S);
    delete p;
    return GZ_OK;
}

}  // extern "C"

