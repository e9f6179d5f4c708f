// Sketch update kernels: a node's batch of endpoint entries applied to its
// CubeSketches with the node tile staged in LDS.
//
// Paper: CubeSketch update (Sec. 3.2, Fig. "cube_code", Eq. 1-2); per-node
// batching so that one node's sketch is touched once per batch (Sec. 4.1,
// 5.1); batch- and sketch-level parallelism (Sec. 5.1) become workgroups over
// node batches and lanes over (round, column) pairs.
//
// Two contracts share the code.  Graphs with V <= 2^16 key their hashes by the
// 31-bit edge index and keep three planes per bucket (alpha, gamma low, gamma
// high); "wide" graphs (V > 2^16) key them by the node pair, need 64-bit
// indices and keep four planes (alpha low, alpha high, gamma low, gamma high).
// An entry is the edge index for the former and the neighbour id for the latter.
#include <type_traits>

#include "gz_device.h"
#include "gz_internal.h"

namespace gz {

// ------------------------------------------------------------ sketch update --

// The LDS tile interleaves the planes bucket by bucket: with three planes,
// word (d * S + p) * 3 + plane holds plane `plane` of row d of pair p, so one
// 24-bit multiply-add gives the address and the planes are immediate offsets.
// The row stride S is P rounded up to a multiple of 64, so the bank of a lane
// (word mod 64) is 3p + plane mod 64 whatever row its entry hashed to: the
// lanes of a wave never collide, however their rows differ.  With four planes
// a pair takes words 4p + p/16 + plane of its row (one pad word per 16 pairs),
// which keeps the 64 lanes of a wave in 64 distinct banks as well.
template <bool kWide>
struct Layout {
    static constexpr uint32_t kPl = kWide ? kPlanesWide : kPlanes;
    __device__ __forceinline__ static uint32_t lane_word(uint32_t p) {
        return kWide ? kPl * p + (p >> 4) : kPl * p;
    }
};

template <bool kWide>
using SeedsOf = typename std::conditional<kWide, WideSeeds, PairSeeds>::type;

// Per-lane state of the update: the lane's (round, column) pair p within group
// j of J, the pair's seeds, and the lane's offsets in a tile row and in a
// node's HBM block.  It depends only on the graph, so a workgroup keeps it
// across consecutive work items of one graph.
template <bool kWide>
struct Lane {
    SeedsOf<kWide> s;
    uint32_t j, J, p;
    uint32_t tile_bytes;  // byte offset of the lane's bucket in a tile row
    uint32_t hbm_word;    // word of (round, plane 0, row 0, column) in a node block
    bool active;
};

template <bool kWide>
__device__ __forceinline__ Lane<kWide> make_lane(const GraphDesc& g) {
    Lane<kWide> ln{};
    const uint32_t tid = threadIdx.x;
    ln.J = blockDim.x / g.P;
    ln.j = tid / g.P;
    ln.p = tid - ln.j * g.P;
    ln.active = tid < ln.J * g.P;
    if (ln.active) {
        if constexpr (kWide) ln.s = load_wide_seeds(g.seeds, g.P, ln.p);
        else ln.s = load_pair_seeds(g.seeds, g.P, ln.p);
    }
    ln.tile_bytes = Layout<kWide>::lane_word(ln.p) * 4;
    ln.hbm_word = sk_word_n(Layout<kWide>::kPl, g.B, ln.p / kC, 0, 0, ln.p % kC);
    return ln;
}

// Hash one entry for this lane's pair and XOR it into the exact-depth row of
// the LDS tile; rows >= DL (kAllRows == false only) go straight to HBM with
// atomics (`skl` is the lane's bucket of row 0, plane 0, in the node block).
template <bool kAllRows, bool kWide>
__device__ __forceinline__ void xor_entry(uint32_t x, uint32_t node, const Lane<kWide>& ln,
                                          uint32_t Bm1, uint32_t DL, uint32_t row_bytes,
                                          uint8_t* __restrict__ tile, uint32_t* __restrict__ skl,
                                          uint32_t plane_words) {
    if constexpr (!kWide) {
        const uint32_t d = row_depth(ln.s, x, Bm1);
        const uint32_t hi = chk_hi(ln.s, x);
        const uint32_t lo = chk_lo(ln.s, x);
        if (kAllRows || d < DL) {
            uint32_t* a = (uint32_t*)(tile + (__umul24(d, row_bytes) + ln.tile_bytes));
            atomicXor(a, x);
            atomicXor(a + 1, lo);
            atomicXor(a + 2, hi);
        } else {
            uint32_t* w = skl + d * kC;
            atomicXor(w, x);
            atomicXor(w + plane_words, lo);
            atomicXor(w + 2 * plane_words, hi);
        }
    } else {
        // x is the neighbour: the edge is {node, x}
        const uint32_t u = min(node, x), v = max(node, x);
        const uint32_t d = wide_row_depth(ln.s, u, v, Bm1);
        const uint32_t hi = pair_hash(ln.s.h[1], u, v);
        const uint32_t lo = pair_hash(ln.s.h[2], u, v);
        const uint64_t idx = edge_index64(u, v);
        const uint32_t ilo = (uint32_t)idx, ihi = (uint32_t)(idx >> 32);
        if (kAllRows || d < DL) {
            uint32_t* a = (uint32_t*)(tile + (d * row_bytes + ln.tile_bytes));
            atomicXor(a, ilo);
            atomicXor(a + 1, ihi);
            atomicXor(a + 2, lo);
            atomicXor(a + 3, hi);
        } else {
            uint32_t* w = skl + d * kC;
            atomicXor(w, ilo);
            atomicXor(w + plane_words, ihi);
            atomicXor(w + 2 * plane_words, lo);
            atomicXor(w + 3 * plane_words, hi);
        }
    }
}

// Entry sources: the grouped entries of the fused path, or a node's raw
// neighbour list in the plain per-node path (for three-plane graphs the index
// is computed on the fly; wide graphs take neighbour ids as entries anyway).
// Both read four consecutive entries with one 16-byte load when the address
// is 16-byte aligned (the caller aligns the quads).
struct GroupedEntries {
    const uint32_t* __restrict__ p;
    __device__ __forceinline__ uint32_t one(uint32_t e) const { return p[e]; }
    __device__ __forceinline__ uint4 quad(uint32_t e) const {
        return *reinterpret_cast<const uint4*>(p + e);
    }
    __device__ __forceinline__ uint32_t misalign() const {
        return (uint32_t)(((uintptr_t)p >> 2) & 3u);
    }
};
struct NeighbourEntries {
    const uint32_t* __restrict__ p;
    uint32_t node;
    __device__ __forceinline__ uint32_t one(uint32_t e) const { return edge_index(node, p[e]); }
    __device__ __forceinline__ uint4 quad(uint32_t e) const {
        uint4 v = *reinterpret_cast<const uint4*>(p + e);
        return make_uint4(edge_index(node, v.x), edge_index(node, v.y), edge_index(node, v.z),
                          edge_index(node, v.w));
    }
    __device__ __forceinline__ uint32_t misalign() const {
        return (uint32_t)(((uintptr_t)p >> 2) & 3u);
    }
};

// Walk over the tile rows d < DL of a node in HBM order of the round-major
// block: flat index i over planes * DL * P words, row = i / P (by a reciprocal
// multiply, exact for i * P < 2^32), p = i mod P, d = row / planes,
// plane = row mod planes.  Consecutive lanes take consecutive pairs of one
// (plane, row), so their LDS words fall in distinct banks and their HBM words
// form runs of C columns.
template <bool kWide>
struct TileWalk {
    static constexpr uint32_t kPl = Layout<kWide>::kPl;
    uint32_t P, B, DL, RW, n, recip;
    __device__ __forceinline__ TileWalk(uint32_t P_, uint32_t B_, uint32_t DL_)
        : P(P_), B(B_), DL(DL_), RW(tile_row_words(P_, kWide)), n(kPl * DL_ * P_),
          recip(0xFFFFFFFFu / P_ + 1u) {}
    __device__ __forceinline__ void at(uint32_t i, uint32_t* t, uint32_t* h) const {
        const uint32_t row = __umulhi(i, recip);
        const uint32_t p = i - row * P;
        const uint32_t d = row / kPl;
        const uint32_t pl = row - d * kPl;
        *t = d * RW + Layout<kWide>::lane_word(p) + pl;
        *h = sk_word_n(kPl, B, p / kC, pl, d, p % kC);
    }
};

// Tile set-up.  A node this workgroup owns for the launch starts from its HBM
// rows (loads batched four per lane so they overlap); a node shared with other
// workgroups starts from zero and is merged with atomics.
template <bool kWide>
__device__ __forceinline__ void tile_load(uint32_t* __restrict__ tile,
                                          const uint32_t* __restrict__ skn,
                                          const TileWalk<kWide>& tw) {
    for (uint32_t base = threadIdx.x; base < tw.n; base += 4 * blockDim.x) {
        uint32_t v[4], t[4];
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const uint32_t i = base + k * blockDim.x;
            uint32_t h = 0;
            t[k] = kNone;
            if (i < tw.n) tw.at(i, &t[k], &h);
            v[k] = i < tw.n ? skn[h] : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k)
            if (t[k] != kNone) tile[t[k]] = v[k];
    }
}

template <bool kWide>
__device__ __forceinline__ void tile_zero(uint32_t* __restrict__ tile, const TileWalk<kWide>& tw) {
    for (uint32_t i = threadIdx.x; i < tw.DL * tw.RW; i += blockDim.x) tile[i] = 0;
}

// Write-back: owned nodes store the whole tile, shared nodes XOR non-zero words
// in with atomics.
template <bool kWide>
__device__ __forceinline__ void tile_store(const uint32_t* __restrict__ tile,
                                           uint32_t* __restrict__ skn, const TileWalk<kWide>& tw,
                                           bool shared) {
    for (uint32_t i = threadIdx.x; i < tw.n; i += blockDim.x) {
        uint32_t t, h;
        tw.at(i, &t, &h);
        const uint32_t val = tile[t];
        if (!shared) skn[h] = val;
        else if (val) atomicXor(&skn[h], val);
    }
}

// Apply `count` entries to one node.  The J groups of P lanes each take a
// contiguous share of the entries, read in 16-byte quads, eight entries per
// iteration with the next eight in flight.  The first quads are issued before
// the tile set-up so that both loads overlap; the barriers around the XOR
// phase are inside (every thread of the workgroup calls this).
template <bool kAllRows, bool kWide, typename Src>
__device__ __forceinline__ void apply_entries(const Src& ent, uint32_t count, uint32_t node,
                                              const Lane<kWide>& ln, const GraphDesc& g,
                                              uint32_t DL, uint32_t* __restrict__ tile,
                                              uint32_t* __restrict__ skn, bool shared) {
    const TileWalk<kWide> tw(g.P, g.B, DL);
    uint32_t e = 0, ea = 0, e1 = 0;
    bool pipe = false;
    uint4 a = make_uint4(0, 0, 0, 0), b = a, c = a, d = a;
    const uint32_t mis = ent.misalign();
    if (ln.active) {
        // group ranges start on 16-byte boundaries of the source array
        const uint32_t J = ln.J, j = ln.j;
        const uint32_t head = (4u - mis) & 3u;
        if (count <= head + 8u * J) {
            e = j == 0 ? 0u : count;
            e1 = count;
        } else {
            const uint32_t quads = (count - head) >> 2;
            e = j == 0 ? 0u : head + 4u * (uint32_t)(((uint64_t)quads * j) / J);
            e1 = j + 1 == J ? count : head + 4u * (uint32_t)(((uint64_t)quads * (j + 1)) / J);
        }
        ea = min(e1, e + ((4u - ((e + mis) & 3u)) & 3u));
        pipe = ea + 8 <= e1;
        if (pipe) {
            a = ent.quad(ea);
            b = ent.quad(ea + 4);
        }
    }
    if (shared) tile_zero(tile, tw);
    else tile_load(tile, skn, tw);
    __syncthreads();
    if (ln.active) {
        const uint32_t Bm1 = g.B - 1;
        const uint32_t row_bytes = tw.RW * 4;
        const uint32_t plane_words = g.B * kC;
        uint8_t* tb = (uint8_t*)tile;
        uint32_t* skl = skn + ln.hbm_word;
#define GZ_XOR(x) \
    xor_entry<kAllRows, kWide>((x), node, ln, Bm1, DL, row_bytes, tb, skl, plane_words)
        for (; e < ea; ++e) GZ_XOR(ent.one(e));  // unaligned head (group 0 only)
        if (pipe) {
            // two register sets in turn: while one set is hashed the other is in flight
            for (;;) {
                const bool more1 = e + 16 <= e1;
                if (more1) { c = ent.quad(e + 8); d = ent.quad(e + 12); }
                GZ_XOR(a.x); GZ_XOR(a.y); GZ_XOR(a.z); GZ_XOR(a.w);
                GZ_XOR(b.x); GZ_XOR(b.y); GZ_XOR(b.z); GZ_XOR(b.w);
                e += 8;
                if (!more1) break;
                const bool more2 = e + 16 <= e1;
                if (more2) { a = ent.quad(e + 8); b = ent.quad(e + 12); }
                GZ_XOR(c.x); GZ_XOR(c.y); GZ_XOR(c.z); GZ_XOR(c.w);
                GZ_XOR(d.x); GZ_XOR(d.y); GZ_XOR(d.z); GZ_XOR(d.w);
                e += 8;
                if (!more2) break;
            }
        }
        for (; e < e1; ++e) GZ_XOR(ent.one(e));
#undef GZ_XOR
    }
    __syncthreads();
    tile_store(tile, skn, tw, shared);
}

// Rows an item keeps in LDS: an entry reaches depth d with probability
// 2^-(d+1), so an item of `count` entries puts about count * 2^-(bitlen(count)+k)
// entries per pair below row bitlen(count) + k.  Rows up to that depth stay in
// LDS; the few deeper entries go straight to HBM with atomics, which is cheaper
// than reading and writing mostly empty rows.  Items large enough that the
// extra rows cost little next to their entries keep every row (when the tile
// allows) and take the branch-free path.
constexpr uint32_t kDepthSlack = 3;
constexpr uint32_t kAllRowsPerRow = 16;  // entries per extra row that justify all rows

__device__ __forceinline__ uint32_t item_rows(uint32_t count, uint32_t B, uint32_t lds_rows) {
    const uint32_t need = (32u - __builtin_clz(count | 1u)) + kDepthSlack;
    if (need >= B || (B <= lds_rows && count >= kAllRowsPerRow * (B - need))) return min(B, lds_rows);
    return min(need, lds_rows);
}

// Persistent fused sketch update over a device work list (all graphs of the
// launch).  Each workgroup takes runs of consecutive work items by atomic
// ticket until the list is exhausted (a run is one item when items are few,
// longer when there are millions of small ones, so that the ticket counter is
// not the bottleneck); every workgroup exits once the ticket passes the list.
// The next item's descriptor is loaded while the current one is processed,
// and the lane state is kept while the graph stays the same.  Items whose
// tile holds every row take the branch-free path.
template <bool kWide>
__device__ __forceinline__ void update_items(const WorkItem* __restrict__ items,
                                             uint32_t* __restrict__ ctl,
                                             const uint32_t* __restrict__ grouped,
                                             const GraphDesc* __restrict__ gd, uint32_t lds_rows,
                                             uint32_t* __restrict__ tile, uint32_t* s_ticket) {
    if (ctl[2]) return;
    const uint32_t n_items = ctl[1];
    const uint32_t run = max(1u, n_items / (gridDim.x * 16u));
    uint32_t it = 0, it_end = 0, cur = kNone;
    WorkItem nxt{};
    GraphDesc g{};
    Lane<kWide> ln{};
    for (;;) {
        if (it == it_end) {
            if (threadIdx.x == 0) *s_ticket = atomicAdd(&ctl[0], 1u);
            __syncthreads();
            const uint32_t t = uniform(*s_ticket);
            if ((uint64_t)t * run >= n_items) break;
            it = t * run;
            it_end = min(n_items, it + run);
            nxt = items[it];
        }
        const WorkItem w = nxt;
        if (++it < it_end) nxt = items[it];  // in flight during this item
        if (w.graph != cur) {
            cur = w.graph;
            g = gd[cur];
            ln = make_lane<kWide>(g);
        }
        const uint32_t DL = uniform(item_rows(w.count, g.B, lds_rows));
        const GroupedEntries src{grouped + w.begin};
        const uint32_t node = w.gnode - g.node_base;  // graph-local id (wide hashes key on it)
        uint32_t* skn = g.sk + (uint64_t)(node - g.sk_first) * Layout<kWide>::kPl * g.B * g.P;
        if (DL == g.B)
            apply_entries<true, kWide>(src, w.count, node, ln, g, DL, tile, skn, w.shared != 0);
        else
            apply_entries<false, kWide>(src, w.count, node, ln, g, DL, tile, skn, w.shared != 0);
        __syncthreads();  // the tile is reused by the next item
    }
}

__global__ __launch_bounds__(1024) void k_update(const WorkItem* __restrict__ items,
                                                 uint32_t* __restrict__ ctl,
                                                 const uint32_t* __restrict__ grouped,
                                                 const GraphDesc* __restrict__ gd,
                                                 uint32_t lds_rows) {
    extern __shared__ uint32_t tile[];
    __shared__ uint32_t s_ticket;
    update_items<false>(items, ctl, grouped, gd, lds_rows, tile, &s_ticket);
}

__global__ __launch_bounds__(1024) void k_update_wide(const WorkItem* __restrict__ items,
                                                      uint32_t* __restrict__ ctl,
                                                      const uint32_t* __restrict__ grouped,
                                                      const GraphDesc* __restrict__ gd,
                                                      uint32_t lds_rows) {
    extern __shared__ uint32_t tile[];
    __shared__ uint32_t s_ticket;
    update_items<true>(items, ctl, grouped, gd, lds_rows, tile, &s_ticket);
}

// one node's neighbour list (plain per-node path): every workgroup takes one
// chunk of the list; all validity was checked by k_validate_nbrs first
__global__ __launch_bounds__(1024) void k_update_node(const uint32_t* __restrict__ nbrs,
                                                      uint32_t count, uint32_t node, GraphDesc g,
                                                      uint32_t lds_rows, uint32_t chunk,
                                                      const uint32_t* __restrict__ err) {
    extern __shared__ uint32_t tile[];
    if (*err) return;
    const uint32_t begin = blockIdx.x * chunk;
    const uint32_t cnt = min(chunk, count - begin);
    const uint32_t DL = min(lds_rows, g.B);
    const Lane<false> ln = make_lane<false>(g);
    uint32_t* skn = g.sk + (uint64_t)(node - g.sk_first) * kPlanes * g.B * g.P;
    apply_entries<false, false>(NeighbourEntries{nbrs + begin, node}, cnt, node, ln, g, DL, tile,
                                skn, gridDim.x > 1);
}

__global__ __launch_bounds__(1024) void k_update_node_wide(const uint32_t* __restrict__ nbrs,
                                                           uint32_t count, uint32_t node,
                                                           GraphDesc g, uint32_t lds_rows,
                                                           uint32_t chunk,
                                                           const uint32_t* __restrict__ err) {
    extern __shared__ uint32_t tile[];
    if (*err) return;
    const uint32_t begin = blockIdx.x * chunk;
    const uint32_t cnt = min(chunk, count - begin);
    const uint32_t DL = min(lds_rows, g.B);
    const Lane<true> ln = make_lane<true>(g);
    uint32_t* skn = g.sk + (uint64_t)(node - g.sk_first) * kPlanesWide * g.B * g.P;
    apply_entries<false, true>(GroupedEntries{nbrs + begin}, cnt, node, ln, g, DL, tile, skn,
                               gridDim.x > 1);
}

}  // namespace gz
