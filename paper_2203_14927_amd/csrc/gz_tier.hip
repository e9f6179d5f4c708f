// Host-DRAM tier of node sketches: the sketches of a graph live in pinned host
// memory and HBM holds only the grouped batch and two slab buffers.
//
// Paper: when sketches outgrow RAM, GraphZeppelin keeps them on disk and
// applies each node's buffered updates (a full gutter) with one read and one
// write of that node's sketch (Sec. 4, Sec. 5.1).  Here HBM plays the role of
// RAM and host DRAM that of the disk: one ingest call is grouped by endpoint
// on the device as usual, then the node blocks that received entries stream
// through HBM slab by slab (a slab is a range of consecutive nodes), the copy
// in of slab k+1 and the copy out of slab k-1 overlapping the update of slab
// k.  A query copies one round's slab of every node into HBM per Boruvka
// round, the only part of the sketches a round reads.
#include <algorithm>
#include <cstring>

#include "gz_device.h"
#include "gz_internal.h"

namespace gz {

struct HostTier {
    uint32_t* h_sk = nullptr;  // pinned host memory: every node block, node-major
    uint64_t node_words = 0;
    uint32_t* stage[2] = {nullptr, nullptr};  // device slab buffers
    uint32_t slab_nodes = 0, nslabs = 0;
    hipStream_t h2d = nullptr, d2h = nullptr;
    hipEvent_t in_ev[2] = {nullptr, nullptr};   // slab copied in
    hipEvent_t upd_ev[2] = {nullptr, nullptr};  // slab updated
    hipEvent_t out_ev[2] = {nullptr, nullptr};  // slab copied out (buffer free again)
    GraphDesc* d_descs = nullptr;     // one descriptor per slab (device)
    GraphDesc* h_descs = nullptr;     // pinned
    uint32_t* d_slab_ctl = nullptr;   // per slab: ticket, item count, call error, unused
    uint32_t* d_slab_items = nullptr; // first work item of every slab, then the item count
    uint32_t* h_slab_items = nullptr; // pinned
    uint32_t* round_buf = nullptr;    // V x planes*B*C words: one round of every node (queries)
};

namespace {

constexpr uint64_t kDefaultStaging = 128ull << 20;  // both slab buffers together

// First work item of every slab: items are sorted by node, so it is the lower
// bound of the slab's first node; entry nslabs is the number of items.
__global__ void k_tier_slab_items(const WorkItem* __restrict__ items,
                                  const uint32_t* __restrict__ ctl, uint32_t slab_nodes,
                                  uint32_t nslabs, uint32_t* __restrict__ out) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nslabs) return;
    const uint32_t n = ctl[1];
    if (k == nslabs) {
        out[k] = n;
        return;
    }
    const uint64_t first = (uint64_t)k * slab_nodes;
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (items[mid].gnode < first) lo = mid + 1;
        else hi = mid;
    }
    out[k] = lo;
}

// control block of one slab's update launch: ticket, item count, no error
__global__ void k_tier_slab_ctl(uint32_t* __restrict__ ctl, uint32_t n_items) {
    if (threadIdx.x == 0) {
        ctl[0] = 0;
        ctl[1] = n_items;
        ctl[2] = 0;
        ctl[3] = 0;
    }
}

GraphDesc slab_desc(const gz_graph* g, uint32_t* sk, uint32_t first_node) {
    GraphDesc d{};
    d.sk = sk;
    d.seeds = g->seeds;
    d.n = g->n;
    d.V = g->V;
    d.R = g->R;
    d.B = g->B;
    d.P = g->P;
    d.node_base = 0;  // the graph is alone in its launches
    d.sk_first = first_node;
    d.node_words = g->planes * g->B * g->P;
    d.wide = g->wide;
    d.planes = g->planes;
    return d;
}

}  // namespace

gz_status tier_create(gz_graph* g, uint64_t staging_bytes) {
    HostTier* t = new HostTier();
    g->tier = t;
    t->node_words = (uint64_t)g->planes * g->B * g->P;
    const uint64_t node_bytes = t->node_words * 4;
    const uint64_t budget = staging_bytes ? staging_bytes : kDefaultStaging;
    t->slab_nodes = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g->V, budget / 2 / node_bytes));
    t->nslabs = (g->V + t->slab_nodes - 1) / t->slab_nodes;
    if (hipHostMalloc((void**)&t->h_sk, g->V * node_bytes, hipHostMallocDefault) != hipSuccess) {
        t->h_sk = nullptr;
        return fail(GZ_ENOMEM, "out of pinned host memory for the sketches");
    }
    std::memset(t->h_sk, 0, g->V * node_bytes);
    for (int b = 0; b < 2; ++b)
        if (hipMalloc((void**)&t->stage[b], t->slab_nodes * node_bytes) != hipSuccess) {
            t->stage[b] = nullptr;
            return fail(GZ_ENOMEM, "out of device memory for the slab buffers");
        }
    GZ_HIP(hipStreamCreateWithFlags(&t->h2d, hipStreamNonBlocking));
    GZ_HIP(hipStreamCreateWithFlags(&t->d2h, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
        GZ_HIP(hipEventCreateWithFlags(&t->in_ev[b], hipEventDisableTiming));
        GZ_HIP(hipEventCreateWithFlags(&t->upd_ev[b], hipEventDisableTiming));
        GZ_HIP(hipEventCreateWithFlags(&t->out_ev[b], hipEventDisableTiming));
        GZ_HIP(hipEventRecord(t->out_ev[b], t->d2h));
    }
    GZ_HIP(hipMalloc((void**)&t->d_descs, sizeof(GraphDesc) * t->nslabs));
    GZ_HIP(hipHostMalloc((void**)&t->h_descs, sizeof(GraphDesc) * t->nslabs, hipHostMallocDefault));
    GZ_HIP(hipMalloc((void**)&t->d_slab_ctl, 16ull * t->nslabs));
    GZ_HIP(hipMalloc((void**)&t->d_slab_items, 4ull * (t->nslabs + 1)));
    GZ_HIP(hipHostMalloc((void**)&t->h_slab_items, 4ull * (t->nslabs + 1), hipHostMallocDefault));
    return GZ_OK;
}

void tier_free(gz_graph* g) {
    HostTier* t = g->tier;
    if (!t) return;
    if (t->h2d) hipStreamSynchronize(t->h2d);
    if (t->d2h) hipStreamSynchronize(t->d2h);
    for (int b = 0; b < 2; ++b) {
        hipFree(t->stage[b]);
        for (hipEvent_t e : {t->in_ev[b], t->upd_ev[b], t->out_ev[b]})
            if (e) hipEventDestroy(e);
    }
    if (t->h2d) hipStreamDestroy(t->h2d);
    if (t->d2h) hipStreamDestroy(t->d2h);
    hipFree(t->d_descs);
    hipFree(t->d_slab_ctl);
    hipFree(t->d_slab_items);
    hipFree(t->round_buf);
    if (t->h_descs) hipHostFree(t->h_descs);
    if (t->h_slab_items) hipHostFree(t->h_slab_items);
    if (t->h_sk) hipHostFree(t->h_sk);
    delete t;
    g->tier = nullptr;
}

gz_status tier_ingest(gz_graph* g, const uint32_t* src, const uint32_t* dst, uint64_t N,
                      uint32_t flags, hipStream_t stream) {
    if (N == 0) return GZ_OK;
    HostTier* t = g->tier;
    UpdateLaunch U{};
    GZ_TRY(group_only(g, src, dst, N, flags, stream, &U));  // synchronous; validates
    IngestScratch& S = g->ing;
    k_tier_slab_items<<<(t->nslabs + 256) / 256, 256, 0, stream>>>(S.items, S.ctl, t->slab_nodes,
                                                                    t->nslabs, t->d_slab_items);
    GZ_HIP(hipMemcpyAsync(t->h_slab_items, t->d_slab_items, 4ull * (t->nslabs + 1),
                          hipMemcpyDeviceToHost, stream));
    GZ_HIP(hipStreamSynchronize(stream));
    // slabs with work take the two buffers in turn
    int buf = 0;
    for (uint32_t k = 0; k < t->nslabs; ++k) {
        t->h_descs[k] = slab_desc(g, t->stage[buf], k * t->slab_nodes);
        if (t->h_slab_items[k + 1] > t->h_slab_items[k]) buf ^= 1;
    }
    GZ_HIP(hipMemcpyAsync(t->d_descs, t->h_descs, sizeof(GraphDesc) * t->nslabs,
                          hipMemcpyHostToDevice, stream));
    const void* upd = U.wide ? (const void*)k_update_wide : (const void*)k_update;
    GZ_TRY(set_smem_limit(upd, U.smem));
    const uint64_t node_bytes = t->node_words * 4;
    buf = 0;
    for (uint32_t k = 0; k < t->nslabs; ++k) {
        const uint32_t ia = t->h_slab_items[k], ib = t->h_slab_items[k + 1];
        if (ia == ib) continue;  // no node of this slab has entries: it stays in host DRAM
        const uint64_t first = (uint64_t)k * t->slab_nodes;
        const uint64_t bytes = std::min<uint64_t>(t->slab_nodes, g->V - first) * node_bytes;
        uint32_t* host = t->h_sk + first * t->node_words;
        GZ_HIP(hipStreamWaitEvent(t->h2d, t->out_ev[buf], 0));
        GZ_HIP(hipMemcpyAsync(t->stage[buf], host, bytes, hipMemcpyHostToDevice, t->h2d));
        GZ_HIP(hipEventRecord(t->in_ev[buf], t->h2d));
        GZ_HIP(hipStreamWaitEvent(stream, t->in_ev[buf], 0));
        k_tier_slab_ctl<<<1, 64, 0, stream>>>(t->d_slab_ctl + 4 * k, ib - ia);
        if (U.wide)
            k_update_wide<<<U.grid, U.wg, U.smem, stream>>>(S.items + ia, t->d_slab_ctl + 4 * k,
                                                            update_entries(S, true),
                                                            t->d_descs + k, U.lds_rows);
        else
            k_update<<<U.grid, U.wg, U.smem, stream>>>(S.items + ia, t->d_slab_ctl + 4 * k,
                                                       S.grouped, t->d_descs + k, U.lds_rows);
        GZ_HIP(hipGetLastError());
        GZ_HIP(hipEventRecord(t->upd_ev[buf], stream));
        GZ_HIP(hipStreamWaitEvent(t->d2h, t->upd_ev[buf], 0));
        GZ_HIP(hipMemcpyAsync(host, t->stage[buf], bytes, hipMemcpyDeviceToHost, t->d2h));
        GZ_HIP(hipEventRecord(t->out_ev[buf], t->d2h));
        buf ^= 1;
    }
    // the call is complete once both buffers are copied out
    GZ_HIP(hipStreamWaitEvent(stream, t->out_ev[0], 0));
    GZ_HIP(hipStreamWaitEvent(stream, t->out_ev[1], 0));
    GZ_HIP(fence_record(stream, g));
    if (!(flags & GZ_ASYNC)) GZ_HIP(hipStreamSynchronize(stream));
    return GZ_OK;
}

gz_status tier_update_node(gz_graph* g, uint32_t node, const uint32_t* nbrs, uint32_t count,
                           const uint32_t* errp, hipStream_t stream) {
    HostTier* t = g->tier;
    const gz_tuning tune = g->tuning;
    uint32_t* host = t->h_sk + (uint64_t)node * t->node_words;
    const uint64_t bytes = t->node_words * 4;
    GZ_HIP(hipStreamWaitEvent(stream, t->out_ev[0], 0));
    GZ_HIP(hipMemcpyAsync(t->stage[0], host, bytes, hipMemcpyHostToDevice, stream));
    const GraphDesc gd = slab_desc(g, t->stage[0], node);
    const uint32_t chunk = tune.chunk;
    const uint32_t DL = std::min(tune.lds_rows, g->B);
    const size_t smem = update_smem_bytes(tune.lds_rows, g->B, g->P, g->wide);
    const void* fn = g->wide ? (const void*)k_update_node_wide : (const void*)k_update_node;
    GZ_TRY(set_smem_limit(fn, smem));
    const uint32_t grid = (count + chunk - 1) / chunk;
    if (g->wide)
        k_update_node_wide<<<grid, tune.wg_size, smem, stream>>>(nbrs, count, node, gd,
                                                                   tune.lds_rows, chunk, errp);
    else
        k_update_node<<<grid, tune.wg_size, smem, stream>>>(nbrs, count, node, gd, tune.lds_rows,
                                                              chunk, errp);
    GZ_HIP(hipGetLastError());
    GZ_HIP(hipMemcpyAsync(host, t->stage[0], bytes, hipMemcpyDeviceToHost, stream));
    GZ_HIP(hipEventRecord(t->out_ev[0], stream));
    return GZ_OK;
}

gz_status tier_reset(gz_graph* g) {
    GZ_HIP(hipEventSynchronize(g->last->ev));
    std::memset(g->tier->h_sk, 0, g->V * g->tier->node_words * 4);
    return GZ_OK;
}

gz_status tier_fetch(gz_graph* g, uint32_t lo, uint32_t hi, hipStream_t stream, uint32_t** out) {
    HostTier* t = g->tier;
    const uint64_t bytes = (uint64_t)(hi - lo) * t->node_words * 4;
    *out = nullptr;
    if (hipMalloc((void**)out, std::max<uint64_t>(bytes, 4)) != hipSuccess) {
        *out = nullptr;
        return fail(GZ_ENOMEM, "export buffer");
    }
    GZ_HIP(fence_wait(stream, g));
    GZ_HIP(hipMemcpyAsync(*out, t->h_sk + (uint64_t)lo * t->node_words, bytes,
                          hipMemcpyHostToDevice, stream));
    return GZ_OK;
}

gz_status tier_round(gz_graph* g, uint32_t r, hipStream_t stream, uint32_t** round_buf) {
    HostTier* t = g->tier;
    const uint64_t slab = (uint64_t)g->planes * g->B * kC;  // words of one round of one node
    if (!t->round_buf) {
        if (hipMalloc((void**)&t->round_buf, g->V * slab * 4) != hipSuccess) {
            t->round_buf = nullptr;
            return fail(GZ_ENOMEM, "out of device memory for the query round buffer");
        }
    }
    GZ_HIP(hipMemcpy2DAsync(t->round_buf, slab * 4, t->h_sk + sk_word_n(g->planes, g->B, r, 0, 0, 0),
                            t->node_words * 4, slab * 4, g->V, hipMemcpyHostToDevice, stream));
    *round_buf = t->round_buf;
    return GZ_OK;
}

}  // namespace gz
