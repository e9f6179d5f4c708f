// Ingest path: group the stream by endpoint on the device, then apply each
// node's batch to its CubeSketches with the node tile staged in LDS.
//
// Paper: CubeSketch update (Sec. 3.2, Fig. "cube_code"); per-node batching of
// updates so that one node's sketch is touched once per batch (Sec. 4.1, 5.1);
// batch- and sketch-level parallelism (Sec. 5.1) become workgroups over node
// batches and lanes over (round, column) pairs.
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

// last graph g with offs[g] <= i (skips empty graphs)
__device__ __forceinline__ uint32_t graph_of_update(const uint64_t* __restrict__ offs, uint32_t G,
                                                    uint64_t i) {
    uint32_t lo = 0, hi = G - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
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

// ctl[2]: this call saw an invalid update; ctl[3]: sticky error for gz_flush
__global__ void k_count(const IngestArgs* __restrict__ a, const GraphDesc* __restrict__ gd,
                        uint32_t* __restrict__ counts, uint32_t* __restrict__ ctl) {
    const uint64_t N = a->N;
    const uint32_t G = a->G;
    const uint32_t* __restrict__ src = a->src;
    const uint32_t* __restrict__ dst = a->dst;
    const uint64_t* __restrict__ offs = a->offs;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < N; i += stride) {
        uint32_t g = G == 1 ? 0u : graph_of_update(offs, G, i);
        uint32_t u = src[i], v = dst[i];
        uint32_t V = gd[g].V, base = gd[g].node_base;
        if (u == v || u >= V || v >= V) {
            atomicOr(&ctl[2], 1u);
            atomicOr(&ctl[3], 1u);
            continue;
        }
        atomicAdd(&counts[base + u], 1u);
        atomicAdd(&counts[base + v], 1u);
    }
}

constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kScanPerThread = 8;
constexpr uint32_t kScanTile = kScanThreads * kScanPerThread;
constexpr uint64_t kCountMask = (1ull << 40) - 1;

__device__ __forceinline__ uint64_t packed_of(uint32_t c, uint32_t chunk) {
    uint64_t items = (c + chunk - 1) / chunk;
    return (uint64_t)c | (items << 40);
}

// exclusive scan of 256 values in LDS (Hillis-Steele), returns this thread's prefix
__device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* sh, uint64_t* total) {
    const uint32_t t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (uint32_t off = 1; off < kScanThreads; off <<= 1) {
        uint64_t add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    uint64_t incl = sh[t];
    *total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

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
    block_exclusive_scan(s, sh, &total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// one workgroup: exclusive scan of the tile sums; publishes the item count and
// resets the work ticket
__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint64_t* __restrict__ block_sums,
                                                            uint32_t nblocks,
                                                            uint64_t* __restrict__ packed,
                                                            uint32_t T, uint32_t* __restrict__ ctl) {
    __shared__ uint64_t sh[kScanThreads];
    uint64_t carry = 0;
    for (uint32_t b0 = 0; b0 < nblocks; b0 += kScanThreads) {
        uint32_t i = b0 + threadIdx.x;
        uint64_t v = i < nblocks ? block_sums[i] : 0;
        uint64_t total;
        uint64_t ex = block_exclusive_scan(v, sh, &total);
        if (i < nblocks) block_sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        packed[T] = carry;
        ctl[0] = 0;                           // ticket
        ctl[1] = (uint32_t)(carry >> 40);     // number of work items
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_final(
    const uint32_t* __restrict__ counts, uint32_t T, uint32_t chunk,
    const uint64_t* __restrict__ block_sums, uint64_t* __restrict__ packed,
    uint32_t* __restrict__ cursor, WorkItem* __restrict__ items, const GraphDesc* __restrict__ gd,
    uint32_t G, const uint32_t* __restrict__ ctl) {
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
    uint64_t pre = block_exclusive_scan(s, sh, &total) + block_sums[blockIdx.x];
    const bool skip = ctl[2] != 0;
    for (uint32_t k = 0; k < kScanPerThread; ++k) {
        uint64_t i = base + k;
        if (i < T) {
            packed[i] = pre;
            uint32_t begin = (uint32_t)(pre & kCountMask);
            uint32_t item0 = (uint32_t)(pre >> 40);
            uint32_t c = (uint32_t)(vals[k] & kCountMask);
            uint32_t ni = (uint32_t)(vals[k] >> 40);
            cursor[i] = begin;
            if (!skip && ni) {
                uint32_t g = G == 1 ? 0u : graph_of_node(gd, G, (uint32_t)i);
                for (uint32_t j = 0; j < ni; ++j) {
                    WorkItem w;
                    w.begin = begin + j * chunk;
                    w.count = min(chunk, c - j * chunk);
                    w.gnode = (uint32_t)i;
                    w.graph = g;
                    w.shared = ni > 1 ? 1u : 0u;
                    w.pad = 0;
                    items[item0 + j] = w;
                }
            }
        }
        pre += vals[k];
    }
}

__global__ void k_scatter(const IngestArgs* __restrict__ a, const GraphDesc* __restrict__ gd,
                          uint32_t* __restrict__ cursor, uint32_t* __restrict__ grouped,
                          const uint32_t* __restrict__ ctl) {
    if (ctl[2]) return;
    const uint64_t N = a->N;
    const uint32_t G = a->G;
    const uint32_t* __restrict__ src = a->src;
    const uint32_t* __restrict__ dst = a->dst;
    const uint64_t* __restrict__ offs = a->offs;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < N; i += stride) {
        uint32_t g = G == 1 ? 0u : graph_of_update(offs, G, i);
        uint32_t u = src[i], v = dst[i];
        uint32_t base = gd[g].node_base;
        uint32_t idx = edge_index(u, v);
        uint32_t pu = atomicAdd(&cursor[base + u], 1u);
        grouped[pu] = idx;
        uint32_t pv = atomicAdd(&cursor[base + v], 1u);
        grouped[pv] = idx;
    }
}

// Apply `count` staged edge indices (ent[], in LDS) to node `node` of graph `g`.
// Lanes map to (group j, pair p): J = blockDim / P groups split the entries,
// each lane hashes its pair's seeds and XORs into the exact-depth row of its
// column in the LDS tile (or straight into HBM for rows >= DL).  The tile is
// then XORed back into HBM: plain read-modify-write when this workgroup owns
// the node for the launch, atomics when the node's entries are split.
__device__ __forceinline__ void apply_entries(const uint32_t* __restrict__ ent, uint32_t count,
                                              uint32_t node, const GraphDesc& g, uint32_t DL,
                                              uint32_t Pst, uint32_t* __restrict__ tile,
                                              bool shared) {
    const uint32_t tid = threadIdx.x;
    const uint32_t P = g.P, B = g.B;
    const uint32_t J = blockDim.x / P;
    if (tid < J * P) {
        const uint32_t j = tid / P;
        const uint32_t p = tid - j * P;
        const PairSeeds s = load_pair_seeds(g.seeds, P, p);
        const uint32_t Bm1 = B - 1;
        const uint32_t plane = DL * Pst;
        for (uint32_t e = j; e < count; e += J) {
            const uint32_t x = ent[e];
            const uint32_t d = row_depth(s, x, Bm1);
            const uint32_t hi = chk_hi(s, x);
            const uint32_t lo = chk_lo(s, x);
            if (d < DL) {
                const uint32_t a = d * Pst + p;
                atomicXor(&tile[a], x);
                atomicXor(&tile[plane + a], lo);
                atomicXor(&tile[2 * plane + a], hi);
            } else {
                const uint64_t rowp = (uint64_t)B * P;
                uint32_t* w = g.sk + (uint64_t)node * kPlanes * rowp + (uint64_t)d * P + p;
                atomicXor(w, x);
                atomicXor(w + rowp, lo);
                atomicXor(w + 2 * rowp, hi);
            }
        }
    }
    __syncthreads();
    const uint32_t nw = blockDim.x >> 6, wave = tid >> 6, lane = tid & 63;
    for (uint32_t row = wave; row < kPlanes * DL; row += nw) {
        const uint32_t pl = row / DL, d = row - pl * DL;
        uint32_t* dstrow = g.sk + ((uint64_t)node * kPlanes + pl) * B * P + (uint64_t)d * P;
        const uint32_t* srow = tile + row * Pst;
        for (uint32_t p = lane; p < P; p += 64) {
            const uint32_t val = srow[p];
            if (val) {
                if (shared) atomicXor(&dstrow[p], val);
                else dstrow[p] ^= val;
            }
        }
    }
}

// Persistent fused sketch update over a device work list (all graphs of the
// launch).  Each workgroup takes work items by atomic ticket until the list is
// exhausted; every workgroup exits once the ticket passes the item count.
__global__ __launch_bounds__(1024) void k_update(const WorkItem* __restrict__ items,
                                                 uint32_t* __restrict__ ctl,
                                                 const uint32_t* __restrict__ grouped,
                                                 const GraphDesc* __restrict__ gd,
                                                 uint32_t lds_rows, uint32_t chunk) {
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t s_item;
    if (ctl[2]) return;
    const uint32_t n_items = ctl[1];
    uint32_t* ent = smem;
    uint32_t* tile = smem + chunk;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&ctl[0], 1u);
        __syncthreads();
        const uint32_t it = uniform(s_item);
        if (it >= n_items) break;
        const WorkItem w = items[it];
        const GraphDesc g = gd[w.graph];
        const uint32_t DL = min(lds_rows, g.B);
        const uint32_t Pst = (g.P + 63u) & ~63u;
        for (uint32_t i = threadIdx.x; i < w.count; i += blockDim.x) ent[i] = grouped[w.begin + i];
        for (uint32_t i = threadIdx.x; i < kPlanes * DL * Pst; i += blockDim.x) tile[i] = 0;
        __syncthreads();
        apply_entries(ent, w.count, w.gnode - g.node_base, g, DL, Pst, tile, w.shared != 0);
        __syncthreads();
    }
}

// one node's neighbour list (plain per-node path): every workgroup takes one
// chunk of the list; all validity was checked by k_validate_nbrs first
__global__ __launch_bounds__(1024) void k_update_node(const uint32_t* __restrict__ nbrs,
                                                      uint32_t count, uint32_t node, GraphDesc g,
                                                      uint32_t lds_rows, uint32_t chunk,
                                                      const uint32_t* __restrict__ err) {
    extern __shared__ uint32_t smem[];
    if (*err) return;
    uint32_t* ent = smem;
    uint32_t* tile = smem + chunk;
    const uint32_t begin = blockIdx.x * chunk;
    const uint32_t cnt = min(chunk, count - begin);
    const uint32_t DL = min(lds_rows, g.B);
    const uint32_t Pst = (g.P + 63u) & ~63u;
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) ent[i] = edge_index(node, nbrs[begin + i]);
    for (uint32_t i = threadIdx.x; i < kPlanes * DL * Pst; i += blockDim.x) tile[i] = 0;
    __syncthreads();
    apply_entries(ent, cnt, node, g, DL, Pst, tile, gridDim.x > 1);
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
gz_status grow(T** p, uint64_t have, uint64_t need, const char* what) {
    if (need <= have && *p) return GZ_OK;
    if (*p) GZ_HIP(hipFree(*p));
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, std::max<uint64_t>(need, 1) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(GZ_ENOMEM, std::string("out of device memory for ") + what);
    }
    return GZ_OK;
}

uint32_t grid_for(uint64_t n, uint32_t threads, uint32_t cap) {
    uint64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (uint32_t)b;
}

gz_status ensure_scratch(IngestScratch& S, uint64_t N, uint32_t T, uint32_t G, uint32_t chunk,
                         bool need_staging) {
    int dev = 0;
    GZ_HIP(hipGetDevice(&dev));
    if (S.device != -1 && S.device != dev) return fail(GZ_EINVAL, "graph used on another device");
    S.device = dev;
    if (!S.ctl) {
        GZ_HIP(hipMalloc((void**)&S.ctl, 4 * sizeof(uint32_t)));
        GZ_HIP(hipMemset(S.ctl, 0, 4 * sizeof(uint32_t)));
        GZ_HIP(hipMalloc((void**)&S.args, sizeof(IngestArgs)));
    }
    if (T > S.cap_nodes || !S.counts) {
        gz_status st;
        if ((st = grow(&S.counts, 0, T, "node counts"))) return st;
        if ((st = grow(&S.packed, 0, (uint64_t)T + 1, "node offsets"))) return st;
        if ((st = grow(&S.cursor, 0, T, "node cursors"))) return st;
        if ((st = grow(&S.block_sums, 0, (uint64_t)T / kScanTile + 2, "scan partials"))) return st;
        S.cap_nodes = T;
    }
    if (G > S.cap_graphs || !S.descs) {
        gz_status st;
        if ((st = grow(&S.descs, 0, G, "graph table"))) return st;
        if ((st = grow(&S.offs, 0, (uint64_t)G + 1, "update offsets"))) return st;
        S.cap_graphs = G;
    }
    uint64_t entries = 2 * N;
    if (entries > S.cap_updates || !S.grouped) {
        gz_status st;
        if ((st = grow(&S.grouped, 0, entries, "grouped updates"))) return st;
        S.cap_updates = entries;
    }
    uint64_t items = (uint64_t)T + entries / chunk + 1;
    if (items > S.cap_items || !S.items) {
        gz_status st;
        if ((st = grow(&S.items, 0, items, "work items"))) return st;
        S.cap_items = items;
    }
    if (need_staging && (2 * N > S.cap_staging || !S.staging)) {
        gz_status st;
        if ((st = grow(&S.staging, 0, 2 * N, "input staging"))) return st;
        S.cap_staging = 2 * N;
    }
    return GZ_OK;
}

size_t update_smem_bytes(uint32_t chunk, uint32_t DL, uint32_t Pmax) {
    uint32_t Pst = (Pmax + 63u) & ~63u;
    return (size_t)chunk * 4 + (size_t)kPlanes * DL * Pst * 4;
}

gz_status set_smem_limit(const void* fn, size_t bytes) {
    if (bytes > 65536) GZ_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)bytes));
    return GZ_OK;
}

}  // namespace

void free_ingest_scratch(IngestScratch& S) {
    hipFree(S.counts); hipFree(S.packed); hipFree(S.block_sums); hipFree(S.cursor);
    hipFree(S.grouped); hipFree(S.items); hipFree(S.ctl); hipFree(S.args); hipFree(S.offs);
    hipFree(S.descs); hipFree(S.staging);
    if (S.copied_ev) {
        hipEventSynchronize(S.copied_ev);
        hipEventDestroy(S.copied_ev);
    }
    hipHostFree(S.h_args); hipHostFree(S.h_descs); hipHostFree(S.h_offs); hipHostFree(S.h_err);
    S = IngestScratch{};
}

IngestScratch& shared_ingest_scratch(int device, std::unique_lock<std::mutex>& lock) {
    static std::mutex mu;
    static std::vector<IngestScratch> per_dev(64);
    lock = std::unique_lock<std::mutex>(mu);
    return per_dev[(size_t)device % per_dev.size()];
}

gz_status ingest_fused(gz_graph* const* gs, uint32_t G, const uint64_t* offs_host,
                       const uint32_t* src, const uint32_t* dst, uint64_t N, uint32_t flags,
                       hipStream_t stream, IngestScratch& S) {
    if (G == 0) return fail(GZ_EINVAL, "no graphs");
    if (N >= (1ull << 31)) return fail(GZ_EINVAL, "at most 2^31-1 updates per call");
    if (N && (!src || !dst)) return fail(GZ_EINVAL, "null stream arrays");
    // descriptor table, shapes, launch parameters
    std::vector<GraphDesc> descs(G);
    uint64_t T = 0;
    uint32_t Pmax = 0, DLmax = 1;
    const gz_tuning tune = gs[0]->tuning;
    for (uint32_t k = 0; k < G; ++k) {
        const gz_graph* g = gs[k];
        if (!g) return fail(GZ_EINVAL, "null graph handle");
        descs[k].sk = g->sk;
        descs[k].seeds = g->seeds;
        descs[k].n = g->n;
        descs[k].V = g->V;
        descs[k].R = g->R;
        descs[k].B = g->B;
        descs[k].P = g->P;
        descs[k].node_base = (uint32_t)T;
        descs[k].pad = 0;
        T += g->V;
        Pmax = std::max(Pmax, g->P);
        DLmax = std::max(DLmax, std::min(tune.lds_rows, g->B));
        if (offs_host && offs_host[k + 1] < offs_host[k])
            return fail(GZ_EINVAL, "update offsets must be non-decreasing");
    }
    if (offs_host && (offs_host[0] != 0 || offs_host[G] != N))
        return fail(GZ_EINVAL, "update offsets must start at 0 and end at N");
    if (T >= (1ull << 32)) return fail(GZ_EINVAL, "too many nodes in one call");
    const uint32_t chunk = tune.chunk;
    const uint32_t wg = tune.wg_size;
    if (wg < Pmax || wg % 64 || wg > 1024) return fail(GZ_EINVAL, "workgroup smaller than pairs");
    const bool host_ptr = !(flags & GZ_DEVICE_PTR);
    gz_status st = ensure_scratch(S, N, (uint32_t)T, G, chunk, host_ptr);
    if (st) return st;

    // order after earlier work on these graphs (e.g. a query on another stream)
    for (uint32_t k = 0; k < G; ++k) GZ_HIP(hipStreamWaitEvent(stream, gs[k]->last, 0));

    const uint32_t* dsrc = src;
    const uint32_t* ddst = dst;
    if (host_ptr && N) {
        GZ_HIP(hipMemcpyAsync(S.staging, src, N * 4, hipMemcpyHostToDevice, stream));
        GZ_HIP(hipMemcpyAsync(S.staging + N, dst, N * 4, hipMemcpyHostToDevice, stream));
        dsrc = S.staging;
        ddst = S.staging + N;
    }
    if (!S.copied_ev) {
        GZ_HIP(hipEventCreateWithFlags(&S.copied_ev, hipEventDisableTiming));
        GZ_HIP(hipHostMalloc((void**)&S.h_args, sizeof(IngestArgs), hipHostMallocDefault));
        GZ_HIP(hipHostMalloc((void**)&S.h_err, 4 * sizeof(uint32_t), hipHostMallocDefault));
    } else {
        GZ_HIP(hipEventSynchronize(S.copied_ev));  // previous uploads have left the buffers
    }
    if (G > S.cap_h_graphs || !S.h_descs) {
        if (S.h_descs) GZ_HIP(hipHostFree(S.h_descs));
        if (S.h_offs) GZ_HIP(hipHostFree(S.h_offs));
        S.h_descs = nullptr;
        S.h_offs = nullptr;
        GZ_HIP(hipHostMalloc((void**)&S.h_descs, sizeof(GraphDesc) * G, hipHostMallocDefault));
        GZ_HIP(hipHostMalloc((void**)&S.h_offs, sizeof(uint64_t) * (G + 1), hipHostMallocDefault));
        S.cap_h_graphs = G;
    }
    IngestArgs& a = *S.h_args;
    a = IngestArgs{};
    a.src = dsrc;
    a.dst = ddst;
    a.offs = S.offs;
    a.N = N;
    a.G = G;
    a.T = (uint32_t)T;
    a.chunk = chunk;
    a.lds_rows = tune.lds_rows;
    std::memcpy(S.h_descs, descs.data(), sizeof(GraphDesc) * G);
    GZ_HIP(hipMemcpyAsync(S.args, S.h_args, sizeof(IngestArgs), hipMemcpyHostToDevice, stream));
    GZ_HIP(hipMemcpyAsync(S.descs, S.h_descs, sizeof(GraphDesc) * G, hipMemcpyHostToDevice,
                          stream));
    if (G > 1) {
        std::memcpy(S.h_offs, offs_host, sizeof(uint64_t) * (G + 1));
        GZ_HIP(hipMemcpyAsync(S.offs, S.h_offs, sizeof(uint64_t) * (G + 1),
                              hipMemcpyHostToDevice, stream));
    }
    GZ_HIP(hipEventRecord(S.copied_ev, stream));

    const uint32_t Tn = (uint32_t)T;
    k_fill_u32<<<grid_for(Tn, 256, 4096), 256, 0, stream>>>(S.counts, Tn, 0);
    k_fill_u32<<<1, 64, 0, stream>>>(S.ctl, 3, 0);  // ticket, items, call error (sticky kept)
    const uint32_t ugrid = grid_for(N, 256, 8192);
    k_count<<<ugrid, 256, 0, stream>>>(S.args, S.descs, S.counts, S.ctl);
    const uint32_t nblocks = (uint32_t)((T + kScanTile - 1) / kScanTile);
    k_scan_partial<<<nblocks, kScanThreads, 0, stream>>>(S.counts, Tn, chunk, S.block_sums);
    k_scan_top<<<1, kScanThreads, 0, stream>>>(S.block_sums, nblocks, S.packed, Tn, S.ctl);
    k_scan_final<<<nblocks, kScanThreads, 0, stream>>>(S.counts, Tn, chunk, S.block_sums,
                                                       S.packed, S.cursor, S.items, S.descs, G,
                                                       S.ctl);
    k_scatter<<<ugrid, 256, 0, stream>>>(S.args, S.descs, S.cursor, S.grouped, S.ctl);
    const size_t smem = update_smem_bytes(chunk, DLmax, Pmax);
    if ((st = set_smem_limit((const void*)k_update, smem))) return st;
    const uint32_t pgrid = std::max(1u, tune.wgs_per_cu) * (uint32_t)device_cu_count();
    k_update<<<pgrid, wg, smem, stream>>>(S.items, S.ctl, S.grouped, S.descs, tune.lds_rows, chunk);
    GZ_HIP(hipGetLastError());
    for (uint32_t k = 0; k < G; ++k) GZ_HIP(hipEventRecord(gs[k]->last, stream));

    if (!(flags & GZ_ASYNC)) {
        GZ_HIP(hipMemcpyAsync(S.h_err, S.ctl + 2, 4, hipMemcpyDeviceToHost, stream));
        GZ_HIP(hipStreamSynchronize(stream));
        if (S.h_err[0]) {
            // the sticky flag is for asynchronous callers; this one is reported now
            k_fill_u32<<<1, 64, 0, stream>>>(S.ctl + 3, 1, 0);
            GZ_HIP(hipStreamSynchronize(stream));
            return fail(GZ_EINVAL, "invalid update (self-loop or node id out of range)");
        }
    } else {
        for (uint32_t k = 0; k < G; ++k) gs[k]->pending_error = true;  // flush must check
    }
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
    gz_status st = ensure_scratch(S, 0, g->V, 1, tune.chunk, false);
    if (st) return st;
    GZ_HIP(hipStreamWaitEvent(stream, g->last, 0));
    const uint32_t* d = nbrs;
    if (host_ptr) {
        if (count > S.cap_staging || !S.staging) {
            if ((st = grow(&S.staging, 0, count, "input staging"))) return st;
            S.cap_staging = count;
        }
        GZ_HIP(hipMemcpyAsync(S.staging, nbrs, count * 4, hipMemcpyHostToDevice, stream));
        d = S.staging;
    }
    // ctl[2] / ctl[3]: call error / sticky error, as in the fused path
    k_fill_u32<<<1, 64, 0, stream>>>(S.ctl + 2, 1, 0);
    if (!host_ptr)
        k_validate_nbrs<<<grid_for(count, 256, 1024), 256, 0, stream>>>(d, count, node, g->V,
                                                                       S.ctl + 2);
    GraphDesc gd{};
    gd.sk = g->sk;
    gd.seeds = g->seeds;
    gd.n = g->n;
    gd.V = g->V;
    gd.R = g->R;
    gd.B = g->B;
    gd.P = g->P;
    const uint32_t chunk = tune.chunk;
    const uint32_t DL = std::min(tune.lds_rows, g->B);
    const size_t smem = update_smem_bytes(chunk, DL, g->P);
    if ((st = set_smem_limit((const void*)k_update_node, smem))) return st;
    const uint32_t grid = (uint32_t)((count + chunk - 1) / chunk);
    k_update_node<<<grid, tune.wg_size, smem, stream>>>(d, (uint32_t)count, node, gd,
                                                          tune.lds_rows, chunk, S.ctl + 2);
    GZ_HIP(hipGetLastError());
    GZ_HIP(hipEventRecord(g->last, stream));
    if (!host_ptr) {
        if (!(flags & GZ_ASYNC)) {
            uint32_t err = 0;
            GZ_HIP(hipMemcpyAsync(&err, S.ctl + 2, 4, hipMemcpyDeviceToHost, stream));
            GZ_HIP(hipStreamSynchronize(stream));
            if (err) {
                k_fill_u32<<<1, 64, 0, stream>>>(S.ctl + 3, 1, 0);
                GZ_HIP(hipStreamSynchronize(stream));
                return fail(GZ_EINVAL, "invalid neighbour (self-loop or id out of range)");
            }
        } else {
            g->pending_error = true;
        }
    } else {
        // the host copy must finish before the caller may reuse its buffer
        GZ_HIP(hipStreamSynchronize(stream));
    }
    return GZ_OK;
}

}  // namespace gz
