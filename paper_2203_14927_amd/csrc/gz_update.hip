// Sketch update kernels: a node's batch of endpoint entries applied to its
// CubeSketches with the node tile staged in LDS.
//
// Paper: CubeSketch update (Sec. 3.1, Fig. "cube_code", Eq. 1-2); per-node
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

// The LDS tile holds rows d < DL of a node's pairs.  With three planes, word
// (d * S + p) * 3 + plane holds plane `plane` of row d of pair p, so one 24-bit
// multiply-add gives the address and the planes are immediate offsets.  The
// row stride S is P rounded up to a multiple of 64, so the bank of a lane
// (word mod 64) is 3p + plane mod 64 whatever row its entry hashed to: the
// lanes of a wave never collide, however their rows differ.  With four planes
// the pairs of a row go in blocks of 64, each block holding its four planes
// one after another (word d * 4S + 256 * (p / 64) + 64 * plane + p mod 64):
// the bank is p mod 64 for every row and plane, and the planes are again
// immediate offsets.
template <bool kWide>
struct Layout {
    static constexpr uint32_t kPl = kWide ? kPlanesWide : kPlanes;
    static constexpr uint32_t kPlaneStep = kWide ? 64u : 1u;  // words between planes
    __device__ __forceinline__ static uint32_t lane_word(uint32_t p) {
        return kWide ? ((p >> 6) << 8) + (p & 63u) : kPl * p;
    }
};

// Three-plane graphs keep their pair's seeds in registers for the whole launch;
// wide graphs derive per-item constants from the seed table instead (below).
struct NoSeeds {};
template <bool kWide>
using SeedsOf = typename std::conditional<kWide, NoSeeds, PairSeeds>::type;

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

// Which neighbours a run of entries of a wide graph holds: all below the node,
// all above it, or either (tested per entry).  Three-plane graphs ignore it.
enum : int { kAnySide = 0, kBelow = 1, kAbove = 2 };

// Per-item constants of a wide graph's lane for one side of the node.  Within
// an item the node is fixed, so each pair hash is one multiply-add in the
// neighbour x away from a constant.  With x below the node (u = x, v = node)
// h = hi32(c + alo*x) + ahi*x for c = (a2*node + b) mod 2^64; with x above it
// (u = node, v = x) h = hi32(c + a2lo*x) + a2hi*x for c = (a*node + b) mod 2^64.
// A run of one side keeps only that side's multipliers and constants live.
struct SideConsts {
    uint32_t mlo[3], mhi[3];
    uint64_t c[3];
};
struct BothConsts {  // runs of mixed sides (the per-node path)
    SideConsts below, above;
};
struct NoConsts {};
template <bool kWide, int kSide>
using ConstsOf = typename std::conditional<
    !kWide, NoConsts,
    typename std::conditional<kSide == kAnySide, BothConsts, SideConsts>::type>::type;

__device__ __forceinline__ uint64_t mul64_add(uint32_t mlo, uint32_t mhi, uint32_t x, uint64_t c) {
    const uint64_t t = (uint64_t)mlo * x + c;
    return t + ((uint64_t)(mhi * x) << 32);
}

// word (k*3 + j)*2 + half of pair p sits at seeds[w*P + p] (k: row, checksum
// high, checksum low; j: a, a2, b)
template <int kSide>
__device__ __forceinline__ SideConsts side_consts(const uint32_t* __restrict__ seeds, uint32_t P,
                                                  uint32_t p, uint32_t node) {
    SideConsts sc;
    // the multiplier of x: a below the node, a2 above it; the other one multiplies the node
    constexpr uint32_t jx = kSide == kBelow ? 0u : 1u, jn = 1u - jx;
#pragma unroll
    for (uint32_t k = 0; k < 3; ++k) {
        const uint32_t w = k * 6;
        sc.mlo[k] = seeds[(w + 2 * jx) * P + p];
        sc.mhi[k] = seeds[(w + 2 * jx + 1) * P + p];
        const uint32_t nlo = seeds[(w + 2 * jn) * P + p];
        const uint32_t nhi = seeds[(w + 2 * jn + 1) * P + p];
        const uint64_t b = (uint64_t)seeds[(w + 4) * P + p] | ((uint64_t)seeds[(w + 5) * P + p] << 32);
        sc.c[k] = mul64_add(nlo, nhi, node, b);
    }
    return sc;
}

template <bool kWide, int kSide>
__device__ __forceinline__ ConstsOf<kWide, kSide> item_consts(const GraphDesc& g, uint32_t p,
                                                              uint32_t node) {
    ConstsOf<kWide, kSide> cs{};
    if constexpr (kWide && kSide == kAnySide) {
        cs.below = side_consts<kBelow>(g.seeds, g.P, p, node);
        cs.above = side_consts<kAbove>(g.seeds, g.P, p, node);
    } else if constexpr (kWide) {
        cs = side_consts<kSide>(g.seeds, g.P, p, node);
    }
    return cs;
}

template <bool kWide>
__device__ __forceinline__ Lane<kWide> make_lane(const GraphDesc& g) {
    Lane<kWide> ln{};
    const uint32_t tid = threadIdx.x;
    ln.J = blockDim.x / g.P;
    ln.j = tid / g.P;
    ln.p = tid - ln.j * g.P;
    ln.active = tid < ln.J * g.P;
    if constexpr (!kWide)
        if (ln.active) ln.s = load_pair_seeds(g.seeds, g.P, ln.p);
    ln.tile_bytes = Layout<kWide>::lane_word(ln.p) * 4;
    ln.hbm_word = sk_word_n(Layout<kWide>::kPl, g.B, ln.p / kC, 0, 0, ln.p % kC);
    return ln;
}

// The three hash words of an entry for this lane's pair (row hash, checksum
// high, checksum low) and its 64-bit index (wide graphs; three-plane graphs
// use the entry itself as the index).
template <bool kWide, int kSide>
__device__ __forceinline__ void hash_side(uint32_t x, uint32_t node, const SideConsts& sc,
                                          uint32_t* h, uint64_t* idx) {
#pragma unroll
    for (uint32_t k = 0; k < 3; ++k) {
        const uint64_t t = (uint64_t)sc.mlo[k] * x + sc.c[k];
        h[k] = (uint32_t)(t >> 32) + sc.mhi[k] * x;
    }
    if (kSide == kAbove) *idx = (((uint64_t)x * (x - 1u)) >> 1) + node;
    else *idx = (((uint64_t)node * (node - 1u)) >> 1) + x;
}

template <bool kWide, int kSide>
__device__ __forceinline__ void hash_entry(uint32_t x, uint32_t node, const Lane<kWide>& ln,
                                           const ConstsOf<kWide, kSide>& cs, uint32_t* h,
                                           uint64_t* idx) {
    if constexpr (!kWide) {
        h[0] = mas_hash(ln.s.row_mlo, ln.s.row_mhi, ln.s.row_inc, x);
        h[1] = chk_hi(ln.s, x);
        h[2] = chk_lo(ln.s, x);
        *idx = x;
    } else if constexpr (kSide == kAnySide) {
        // x is the neighbour: the edge is {node, x}
        if (x > node) hash_side<kWide, kAbove>(x, node, cs.above, h, idx);
        else hash_side<kWide, kBelow>(x, node, cs.below, h, idx);
    } else {
        hash_side<kWide, kSide>(x, node, cs, h, idx);
    }
}

__device__ __forceinline__ uint32_t depth_of(uint32_t h, uint32_t Bm1) {
    const uint32_t tz = __builtin_ctzg(h, 32);
    return tz < Bm1 ? tz : Bm1;
}

// Hash one entry for this lane's pair and XOR it into the exact-depth row of
// the LDS tile.  Without kAllRows an entry deeper than the item's DL rows goes
// to row DL instead, a sink that is never written back, and the call returns
// true: the caller then applies that entry to HBM with xor_entry_deep.  (Deep
// entries are rare, so the common path stays free of branches.)
template <bool kAllRows, bool kWide, int kSide>
__device__ __forceinline__ bool xor_entry(uint32_t x, uint32_t node, const Lane<kWide>& ln,
                                          const ConstsOf<kWide, kSide>& nc, uint32_t Bm1, uint32_t DL,
                                          uint32_t row_bytes, uint8_t* __restrict__ tile) {
    uint32_t h[3];
    uint64_t idx;
    hash_entry<kWide, kSide>(x, node, ln, nc, h, &idx);
    const uint32_t d = depth_of(h[0], Bm1);
    const uint32_t row = kAllRows ? d : min(d, DL);
    uint32_t* a = (uint32_t*)(tile + (__umul24(row, row_bytes) + ln.tile_bytes));
    if constexpr (!kWide) {
        atomicXor(a, x);
        atomicXor(a + 1, h[2]);
        atomicXor(a + 2, h[1]);
    } else {
        atomicXor(a, (uint32_t)idx);
        atomicXor(a + 64, (uint32_t)(idx >> 32));
        atomicXor(a + 128, h[2]);
        atomicXor(a + 192, h[1]);
    }
    return !kAllRows && d >= DL;
}

// The HBM side of an entry deeper than the item's rows (`skl` is the lane's
// bucket of row 0, plane 0, in the node block; the planes of a bucket are
// plane_words apart, the rows of a round kPl * C); shallower entries do nothing.
template <bool kWide, int kSide>
__device__ __forceinline__ void xor_entry_deep(uint32_t x, uint32_t node, const Lane<kWide>& ln,
                                               const ConstsOf<kWide, kSide>& nc, uint32_t Bm1,
                                               uint32_t DL, uint32_t* __restrict__ skl,
                                               uint32_t plane_words, const GraphDesc& g) {
    uint32_t h[3];
    uint64_t idx;
    hash_entry<kWide, kSide>(x, node, ln, nc, h, &idx);
    uint32_t d = depth_of(h[0], Bm1);
    if constexpr (kWide) {
        // a zero low word of the 64-bit row hash: the depth continues into its high
        // word (such entries always get here: tiles of wide graphs keep at most 32
        // rows when B > 33)
        if (h[0] == 0 && Bm1 > kLowRowLimit) {
            const uint32_t u = min(x, node), v = max(x, node);
            const uint32_t hh = wide_row_hash_high(g.seeds, g.P, ln.p, u, v);
            d = min(kLowRowLimit + (uint32_t)__builtin_ctzg(hh, 32), Bm1);
        }
    }
    if (d < DL) return;
    uint32_t* w = skl + d * (Layout<kWide>::kPl * kC);
    atomicXor(w, (uint32_t)idx);
    if constexpr (!kWide) {
        atomicXor(w + plane_words, h[2]);
        atomicXor(w + 2 * plane_words, h[1]);
    } else {
        atomicXor(w + plane_words, (uint32_t)(idx >> 32));
        atomicXor(w + 2 * plane_words, h[2]);
        atomicXor(w + 3 * plane_words, h[1]);
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

// Walk over the tile rows d < DL of a node, four words (16 bytes) at a time.
// In a node block the rows of a round are contiguous, each row holding its
// planes side by side (kPl * C words), and every row starts on a 32-byte
// boundary.  A unit covers columns 4 * c4 .. + 3 of one plane of one row of one
// round, and units go in groups of four rows: u = (((dhi * R + r) * 4 + dlo) *
// kPl + pl) * 2 + c4, row d = 4 * dhi + dlo (units past row DL - 1 do nothing).
// A group is 4 * kPl * C contiguous words of HBM (three 128-byte lines for
// three planes), and consecutive groups are other rounds: in the LDS tile,
// whose rows all start on the same bank, a wave's lanes then fall on different
// pairs, planes and rounds, at most four on one bank (walking all DL rows of
// one round first put up to DL lanes on a bank; walking row by row across all
// rounds spread them fully but had a wave touch three times as many 128-byte
// lines, and was slower on small items).  The four words of a unit are the
// same row and plane of four consecutive pairs: kLdsStep words apart in the
// tile (three with three planes interleaved per pair, one in the four-plane
// blocks of 64 pairs, which a unit never crosses).
template <bool kWide>
struct TileWalk {
    static constexpr uint32_t kPl = Layout<kWide>::kPl;
    static constexpr uint32_t kLdsStep = kWide ? 1u : kPlanes;
    uint32_t P, B, DL, R, RW, n4, recip;
    __device__ __forceinline__ TileWalk(uint32_t P_, uint32_t B_, uint32_t DL_)
        : P(P_), B(B_), DL(DL_), R(P_ / kC), RW(tile_row_words(P_, kWide)),
          n4(kPl * ((DL_ + 3u) & ~3u) * P_ / 4u), recip(0xFFFFFFFFu / (P_ / kC) + 1u) {}
    // false for the units of rows past DL - 1; else the LDS word of the unit's first
    // column and the unit's 16-byte index in the node block
    __device__ __forceinline__ bool at(uint32_t u, uint32_t* t, uint32_t* h4) const {
        const uint32_t c4 = u & 1u;
        const uint32_t v = u >> 1;
        const uint32_t w = v / kPl;
        const uint32_t pl = v - w * kPl;
        const uint32_t dlo = w & 3u;
        const uint32_t q = w >> 2;
        // R = 1 has no 32-bit reciprocal (it would be 2^32); the quotient is exact
        // for q < 2^32 / R
        const uint32_t dhi = R == 1u ? q : __umulhi(q, recip);
        const uint32_t r = q - dhi * R;
        const uint32_t d = dhi * 4u + dlo;
        *t = d * RW + Layout<kWide>::lane_word(r * kC + 4u * c4) + pl * Layout<kWide>::kPlaneStep;
        *h4 = ((r * B + d) * kPl + pl) * (kC / 4u) + c4;  // sk_word_n(kPl, B, r, pl, d, 4c4) / 4
        return d < DL;
    }
};

// Tile set-up.  A node this workgroup owns for the launch starts from its HBM
// rows (16-byte loads, two per lane in flight: more would take the update
// kernels past 64 VGPRs and cost them a wave per SIMD); a node shared with
// other workgroups starts from zero and is merged with atomics.
constexpr uint32_t kTileLoads = 2;

template <bool kWide>
__device__ __forceinline__ void tile_load(uint32_t* __restrict__ tile,
                                          const uint32_t* __restrict__ skn,
                                          const TileWalk<kWide>& tw) {
    constexpr uint32_t s = TileWalk<kWide>::kLdsStep;
    const uint4* __restrict__ skn4 = reinterpret_cast<const uint4*>(skn);
    for (uint32_t base = threadIdx.x; base < tw.n4; base += kTileLoads * blockDim.x) {
        uint4 v[kTileLoads];
        uint32_t t[kTileLoads];
#pragma unroll
        for (uint32_t k = 0; k < kTileLoads; ++k) {
            const uint32_t u = base + k * blockDim.x;
            uint32_t h4 = 0;
            t[k] = kNone;
            if (u < tw.n4 && !tw.at(u, &t[k], &h4)) t[k] = kNone;
            v[k] = t[k] != kNone ? skn4[h4] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (uint32_t k = 0; k < kTileLoads; ++k)
            if (t[k] != kNone) {
                tile[t[k]] = v[k].x;
                tile[t[k] + s] = v[k].y;
                tile[t[k] + 2 * s] = v[k].z;
                tile[t[k] + 3 * s] = v[k].w;
            }
    }
}

template <bool kWide>
__device__ __forceinline__ void tile_zero(uint32_t* __restrict__ tile, const TileWalk<kWide>& tw) {
    for (uint32_t i = threadIdx.x; i < tw.DL * tw.RW; i += blockDim.x) tile[i] = 0;
}

// Write-back: owned nodes store the whole tile (16-byte stores), shared nodes
// XOR non-zero words in with atomics.
template <bool kWide>
__device__ __forceinline__ void tile_store(const uint32_t* __restrict__ tile,
                                           uint32_t* __restrict__ skn, const TileWalk<kWide>& tw,
                                           bool shared) {
    constexpr uint32_t s = TileWalk<kWide>::kLdsStep;
    uint4* __restrict__ skn4 = reinterpret_cast<uint4*>(skn);
    for (uint32_t u = threadIdx.x; u < tw.n4; u += blockDim.x) {
        uint32_t t, h4;
        if (!tw.at(u, &t, &h4)) continue;
        const uint4 v = make_uint4(tile[t], tile[t + s], tile[t + 2 * s], tile[t + 3 * s]);
        if (!shared) {
            skn4[h4] = v;
        } else {
            uint32_t* w = skn + 4u * h4;
            if (v.x) atomicXor(w, v.x);
            if (v.y) atomicXor(w + 1, v.y);
            if (v.z) atomicXor(w + 2, v.z);
            if (v.w) atomicXor(w + 3, v.w);
        }
    }
}

// The share of entries [lo, hi) that group j of J takes: contiguous, starting
// on 16-byte boundaries of the source array (group 0 also takes the unaligned
// head), read in quads through a two-deep pipeline when it is long enough.
struct GroupShare {
    uint32_t e, ea, e1;  // first entry, first aligned entry, end
    bool pipe;
};

template <typename Src>
__device__ __forceinline__ GroupShare group_share(const Src& ent, uint32_t lo, uint32_t hi,
                                                  uint32_t J, uint32_t j) {
    GroupShare r;
    const uint32_t mis = ent.misalign();
    const uint32_t count = hi - lo;
    const uint32_t head = (4u - ((mis + lo) & 3u)) & 3u;
    if (count <= head + 8u * J) {
        r.e = j == 0 ? lo : hi;
        r.e1 = hi;
    } else {
        const uint32_t quads = (count - head) >> 2;
        r.e = j == 0 ? lo : lo + head + 4u * (uint32_t)(((uint64_t)quads * j) / J);
        r.e1 = j + 1 == J ? hi : lo + head + 4u * (uint32_t)(((uint64_t)quads * (j + 1)) / J);
    }
    r.ea = min(r.e1, r.e + ((4u - ((r.e + mis) & 3u)) & 3u));
    r.pipe = r.ea + 8 <= r.e1;
    return r;
}

// XOR one group's share into the tile: eight entries per iteration with the
// next eight in flight (a and b hold the first eight when r.pipe).
template <bool kAllRows, bool kWide, int kSide, typename Src>
__device__ __forceinline__ void xor_share(const Src& ent, GroupShare r, uint4 a, uint4 b,
                                          uint32_t node, const Lane<kWide>& ln,
                                          const ConstsOf<kWide, kSide>& nc, uint32_t Bm1,
                                          uint32_t DL, uint32_t row_bytes, uint8_t* tb,
                                          uint32_t* skl, uint32_t plane_words,
                                          const GraphDesc& g) {
    uint32_t e = r.e;
    uint4 c = make_uint4(0, 0, 0, 0), d = c;
#define GZ_XOR(x) xor_entry<kAllRows, kWide, kSide>((x), node, ln, nc, Bm1, DL, row_bytes, tb)
#define GZ_DEEP(x) xor_entry_deep<kWide, kSide>((x), node, ln, nc, Bm1, DL, skl, plane_words, g)
    // A set of eight entries.  Three-plane graphs apply a deep entry to HBM at
    // once (their small items keep few rows, so deep entries are common there);
    // wide graphs, whose items are long, note them and apply the set's deep
    // entries after it, keeping the eight entries free of branches.
#define GZ_SET(p, q)                                                               \
    if constexpr (!kWide) {                                                        \
        GZ_ONE(p.x); GZ_ONE(p.y); GZ_ONE(p.z); GZ_ONE(p.w);                        \
        GZ_ONE(q.x); GZ_ONE(q.y); GZ_ONE(q.z); GZ_ONE(q.w);                        \
    } else {                                                                       \
        bool deep = GZ_XOR(p.x);                                                   \
        deep |= GZ_XOR(p.y); deep |= GZ_XOR(p.z); deep |= GZ_XOR(p.w);             \
        deep |= GZ_XOR(q.x); deep |= GZ_XOR(q.y); deep |= GZ_XOR(q.z);             \
        deep |= GZ_XOR(q.w);                                                       \
        if (!kAllRows && deep) deep_set(e);                                        \
    }
#define GZ_ONE(x) \
    if (GZ_XOR(x)) GZ_DEEP(x)
    // the rare deep entries of the set at [e0, e0 + 8): the set is read again
    // (the barrier keeps the compiler from holding the first read, or its
    // hashes, in registers across the set) and re-hashed
    auto deep_set = [&](uint32_t e0) {
        asm volatile("" ::: "memory");
#pragma unroll 1
        for (uint32_t k = 0; k < 8; ++k) GZ_DEEP(ent.one(e0 + k));
    };
    for (; e < r.ea; ++e) {  // unaligned head (group 0 only)
        const uint32_t x = ent.one(e);
        GZ_ONE(x);
    }
    if (r.pipe) {
        // two register sets in turn: while one set is hashed the other is in flight;
        // entries of a set that went deeper than the tile are applied to HBM after it
        for (;;) {
            const bool more1 = e + 16 <= r.e1;
            if (more1) { c = ent.quad(e + 8); d = ent.quad(e + 12); }
            GZ_SET(a, b);
            e += 8;
            if (!more1) break;
            const bool more2 = e + 16 <= r.e1;
            if (more2) { a = ent.quad(e + 8); b = ent.quad(e + 12); }
            GZ_SET(c, d);
            e += 8;
            if (!more2) break;
        }
    }
    for (; e < r.e1; ++e) {
        const uint32_t x = ent.one(e);
        GZ_ONE(x);
    }
#undef GZ_XOR
#undef GZ_DEEP
#undef GZ_ONE
#undef GZ_SET
}

// Apply `count` entries to one node.  The J groups of P lanes each take a
// share of the entries.  With kSide1 == kBelow (wide graphs, grouped entries)
// entries [0, split) have neighbours below the node and [split, count) above
// it, and each run is hashed with its own straight-line code; otherwise split
// == count.  The first quads are issued before the tile set-up so that both
// loads overlap; the barriers around the XOR phase are inside (every thread of
// the workgroup calls this).
// A small item's entries staged in LDS: group j of J takes entries j, j + J,
// j + 2J, ... of [lo, hi) (any split of the entries gives the same XOR), four
// at a time; every lane of a group reads the same words (broadcast reads).
template <bool kWide, int kSide>
__device__ __forceinline__ void xor_staged(const uint32_t* __restrict__ st, uint32_t lo,
                                           uint32_t hi, uint32_t node, const Lane<kWide>& ln,
                                           const ConstsOf<kWide, kSide>& nc, const GraphDesc& g,
                                           uint32_t DL, uint32_t row_bytes, uint8_t* tb,
                                           uint32_t* skl) {
    const uint32_t Bm1 = g.B - 1;
    const uint32_t J = ln.J;
    const uint32_t plane_words = kC;
#define GZ_ONE_S(x)                                                                 \
    if (xor_entry<false, kWide, kSide>((x), node, ln, nc, Bm1, DL, row_bytes, tb)) \
    xor_entry_deep<kWide, kSide>((x), node, ln, nc, Bm1, DL, skl, plane_words, g)
    uint32_t e = lo + ln.j;
    for (; e + 3 * J < hi; e += 4 * J) {
        const uint32_t x0 = st[e], x1 = st[e + J], x2 = st[e + 2 * J], x3 = st[e + 3 * J];
        GZ_ONE_S(x0);
        GZ_ONE_S(x1);
        GZ_ONE_S(x2);
        GZ_ONE_S(x3);
    }
    for (; e < hi; e += J) {
        const uint32_t x = st[e];
        GZ_ONE_S(x);
    }
#undef GZ_ONE_S
}

// The XOR phase of one item (lanes of active groups; wide graphs with grouped
// entries take the two sides of the node one after the other).
template <bool kAllRows, bool kWide, int kSide1, typename Src>
__device__ __forceinline__ void xor_item(const Src& ent, GroupShare r, uint4 a, uint4 b,
                                         uint32_t count, uint32_t split, uint32_t node,
                                         const Lane<kWide>& ln,
                                         const ConstsOf<kWide, kSide1>& nc, const GraphDesc& g,
                                         uint32_t DL, const TileWalk<kWide>& tw, uint32_t* tile,
                                         uint32_t* skn) {
    const uint32_t Bm1 = g.B - 1;
    const uint32_t row_bytes = tw.RW * 4;
    const uint32_t plane_words = kC;  // the planes of a row sit side by side
    uint8_t* tb = (uint8_t*)tile;
    uint32_t* skl = skn + ln.hbm_word;
    xor_share<kAllRows, kWide, kSide1>(ent, r, a, b, node, ln, nc, Bm1, DL, row_bytes, tb, skl,
                                       plane_words, g);
    if constexpr (kSide1 == kBelow) {
        if (split < count) {
            const GroupShare r2 = group_share(ent, split, count, ln.J, ln.j);
            uint4 a2 = make_uint4(0, 0, 0, 0), b2 = a2;
            if (r2.pipe) {
                a2 = ent.quad(r2.ea);
                b2 = ent.quad(r2.ea + 4);
            }
            const ConstsOf<kWide, kAbove> nc2 = item_consts<kWide, kAbove>(g, ln.p, node);
            xor_share<kAllRows, kWide, kAbove>(ent, r2, a2, b2, node, ln, nc2, Bm1, DL,
                                               row_bytes, tb, skl, plane_words, g);
        }
    }
}

// Apply `count` entries to one node.  The J groups of P lanes each take a
// share of the entries.  With kSide1 == kBelow (wide graphs, grouped entries)
// entries [0, split) have neighbours below the node and [split, count) above
// it, and each run is hashed with its own straight-line code; otherwise split
// == count.  The barriers around the XOR phase are inside (every thread of the
// workgroup calls this).
// A large item issues its first entry quads before the tile set-up, so that
// both loads overlap, and reads the rest from HBM while it hashes.  A small
// item (stage non-null: at most two entries per thread) loads all its entries
// together with the tile into LDS: its XOR phase then waits on no HBM load,
// and the item costs one memory latency instead of one per set of entries
// (small items are too short to hide those behind hashing).
template <bool kAllRows, bool kWide, int kSide1, typename Src>
__device__ __forceinline__ void apply_entries(const Src& ent, uint32_t count, uint32_t split,
                                              uint32_t node, const Lane<kWide>& ln,
                                              const GraphDesc& g, uint32_t DL,
                                              uint32_t* __restrict__ tile,
                                              uint32_t* __restrict__ skn, bool shared,
                                              uint32_t* __restrict__ stage) {
    const TileWalk<kWide> tw(g.P, g.B, DL);
    ConstsOf<kWide, kSide1> nc{};
    GroupShare r{};
    uint4 a = make_uint4(0, 0, 0, 0), b = a;
    const uint32_t t = threadIdx.x;
    uint32_t s0 = 0, s1 = 0;
    if (!kWide && stage) {
        if (t < count) s0 = ent.one(t);
        if (t + blockDim.x < count) s1 = ent.one(t + blockDim.x);
        if (ln.active) nc = item_consts<kWide, kSide1>(g, ln.p, node);
    } else if (ln.active) {
        nc = item_consts<kWide, kSide1>(g, ln.p, node);
        r = group_share(ent, 0, split, ln.J, ln.j);
        if (r.pipe) {
            a = ent.quad(r.ea);
            b = ent.quad(r.ea + 4);
        }
    }
    if (shared) tile_zero(tile, tw);
    else tile_load(tile, skn, tw);
    if (!kWide && stage) {
        if (t < count) stage[t] = s0;
        if (t + blockDim.x < count) stage[t + blockDim.x] = s1;
    }
    __syncthreads();
    if (ln.active) {
        if (!kWide && stage) {
            uint8_t* tb = (uint8_t*)tile;
            uint32_t* skl = skn + ln.hbm_word;
            xor_staged<kWide, kSide1>(stage, 0, split, node, ln, nc, g, DL, tw.RW * 4, tb, skl);
            if constexpr (kSide1 == kBelow) {
                if (split < count) {
                    const ConstsOf<kWide, kAbove> nc2 = item_consts<kWide, kAbove>(g, ln.p, node);
                    xor_staged<kWide, kAbove>(stage, split, count, node, ln, nc2, g, DL,
                                              tw.RW * 4, tb, skl);
                }
            }
        } else {
            xor_item<kAllRows, kWide, kSide1>(ent, r, a, b, count, split, node, ln, nc, g, DL,
                                              tw, tile, skn);
        }
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
                                             uint32_t* __restrict__ smem, uint32_t* s_ticket) {
    uint32_t* tile = smem + (kWide ? 0u : kItemStageWords);
    const uint32_t stage_max = min(kItemStageWords, 2u * blockDim.x);
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
        uint32_t DL = uniform(item_rows(w.count, g.B, lds_rows));
        // wide graphs deeper than 33 rows keep at most 32 in LDS: an entry whose
        // row hash has a zero low word then takes the deep path, which reads the
        // hash's high word
        if (kWide && g.B > kLowRowLimit + 1) DL = min(DL, kLowRowLimit);
        const GroupedEntries src{grouped + w.begin};
        const uint32_t node = w.gnode - g.node_base;  // graph-local id (wide hashes key on it)
        uint32_t* skn = g.sk + (uint64_t)(node - g.sk_first) * Layout<kWide>::kPl * g.B * g.P;
        constexpr int kS = kWide ? kBelow : kAnySide;
        const uint32_t split = kWide ? w.split : w.count;
        // (wide graphs, whose update kernel is at its register limit, do not stage)
        uint32_t* stage = !kWide && w.count <= stage_max ? smem : nullptr;
        if (DL == g.B)
            apply_entries<true, kWide, kS>(src, w.count, split, node, ln, g, DL, tile, skn,
                                           w.shared != 0, stage);
        else
            apply_entries<false, kWide, kS>(src, w.count, split, node, ln, g, DL, tile, skn,
                                            w.shared != 0, stage);
        __syncthreads();  // the tile is reused by the next item
    }
}

__global__ __launch_bounds__(1024) void k_update(const WorkItem* __restrict__ items,
                                                 uint32_t* __restrict__ ctl,
                                                 const uint32_t* __restrict__ grouped,
                                                 const GraphDesc* __restrict__ gd,
                                                 uint32_t lds_rows) {
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t s_ticket;
    update_items<false>(items, ctl, grouped, gd, lds_rows, smem, &s_ticket);
}

__global__ __launch_bounds__(1024) void k_update_wide(const WorkItem* __restrict__ items,
                                                      uint32_t* __restrict__ ctl,
                                                      const uint32_t* __restrict__ grouped,
                                                      const GraphDesc* __restrict__ gd,
                                                      uint32_t lds_rows) {
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t s_ticket;
    update_items<true>(items, ctl, grouped, gd, lds_rows, smem, &s_ticket);
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
    apply_entries<false, false, kAnySide>(NeighbourEntries{nbrs + begin, node}, cnt, cnt, node,
                                          ln, g, DL, tile, skn, gridDim.x > 1, nullptr);
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
    const uint32_t DL = min(min(lds_rows, g.B), g.B > kLowRowLimit + 1 ? kLowRowLimit : g.B);
    const Lane<true> ln = make_lane<true>(g);
    uint32_t* skn = g.sk + (uint64_t)(node - g.sk_first) * kPlanesWide * g.B * g.P;
    apply_entries<false, true, kAnySide>(GroupedEntries{nbrs + begin}, cnt, cnt, node, ln, g, DL,
                                         tile, skn, gridDim.x > 1, nullptr);
}

// Wide graphs: order each work item's entries so that neighbours below the
// node come first (copied from `grouped` into the same positions of `out`),
// and record their number in the item.  Order within a side is arbitrary: the
// sketch update is a sum over Z2.  One wave per item, 64 entries at a time:
// the lanes' places come from ballots, so no barrier or LDS is involved.
constexpr uint32_t kSplitBatch = 4;  // groups of 64 entries loaded per step

__global__ __launch_bounds__(256) void k_split_items(const uint32_t* __restrict__ ctl,
                                                     WorkItem* __restrict__ items,
                                                     const uint32_t* __restrict__ grouped,
                                                     uint32_t* __restrict__ out,
                                                     const GraphDesc* __restrict__ gd) {
    if (ctl[2]) return;
    const uint32_t n_items = ctl[1];
    const uint32_t lane = __lane_id();
    const uint64_t below_lane = (1ull << lane) - 1ull;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < n_items;
         i += waves) {
        const WorkItem w = items[i];
        const uint32_t node = w.gnode - gd[w.graph].node_base;
        const uint32_t* src = grouped + w.begin;
        uint32_t* lo_out = out + w.begin;
        uint32_t* hi_out = out + w.begin + w.count - 1u;
        uint32_t nlo = 0, nhi = 0;
        for (uint32_t e0 = 0; e0 < w.count; e0 += 64 * kSplitBatch) {
            uint32_t xs[kSplitBatch];
#pragma unroll
            for (uint32_t k = 0; k < kSplitBatch; ++k) {  // loads in flight together
                const uint32_t e = e0 + k * 64 + lane;
                xs[k] = e < w.count ? src[e] : 0u;
            }
#pragma unroll
            for (uint32_t k = 0; k < kSplitBatch; ++k) {
                const uint32_t e = e0 + k * 64 + lane;
                const bool valid = e < w.count;
                const uint32_t x = xs[k];
                const bool lo = valid && x < node;
                const uint64_t mlo = __ballot(lo), mhi = __ballot(valid && !lo);
                if (lo) lo_out[nlo + (uint32_t)__popcll(mlo & below_lane)] = x;
                else if (valid) *(hi_out - (nhi + (uint32_t)__popcll(mhi & below_lane))) = x;
                nlo += (uint32_t)__popcll(mlo);
                nhi += (uint32_t)__popcll(mhi);
            }
        }
        if (lane == 0) items[i].split = nlo;
    }
}

}  // namespace gz
