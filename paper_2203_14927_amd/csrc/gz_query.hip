// Query path: Boruvka over XOR-merged node sketches, fully on the device.
//
// Paper: Boruvka emulated on characteristic vectors (Sec. 2.2), with one
// fresh CubeSketch per round; each round (Sec. 4.2) (1) recovers an edge from
// the sketch of every current component, (2) merges components along the
// recovered edges, (3) sums the merged components' sketches.  Step (3) is done
// lazily: the next round XOR-reduces the round-r rows of each component's
// members.  CubeSketch query: Sec. 3.1 and Fig. "cube_code".
//
// Merging is deterministic: the recovered edges form a functional graph over
// components (out-degree <= 1); its cycles are found by pointer doubling
// (successor and running minimum) and each cycle drops the edge of its
// smallest component; the kept edges join the forest and every resulting tree
// takes its smallest component id as label.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "gz_device.h"
#include "gz_internal.h"

namespace gz {

// one workgroup of the component reduce: consecutive nodes of one graph
struct ReduceSpan {
    uint32_t v0;     // first node (global id)
    uint32_t n;      // nodes, at most 2048
    uint32_t graph;  // descriptor of the span's graph
    uint32_t whole;  // the span holds every node of its graph
};

struct QueryScratch {
    int device = -1;
    uint32_t cap_nodes = 0, cap_graphs = 0, cap_wpr = 0;
    uint32_t *comp = nullptr, *L = nullptr, *L2 = nullptr, *A = nullptr, *slot = nullptr;
    uint32_t *done = nullptr, *hook = nullptr, *s = nullptr, *s2 = nullptr;
    uint64_t* hedge = nullptr;  // index of each component's hook edge
    uint32_t *m = nullptr, *m2 = nullptr, *rootOf = nullptr, *newlab = nullptr, *merged = nullptr;
    uint32_t *gof = nullptr, *acc = nullptr, *ctl = nullptr, *labels = nullptr;
    uint32_t *gcount = nullptr, *gfail = nullptr, *foff = nullptr, *fcur = nullptr;
    uint32_t* gcomp = nullptr;  // components of each graph a round leaves (two sets of G)
    uint32_t *fcnt = nullptr;
    uint32_t *fpairs = nullptr;
    uint64_t *forest = nullptr, *fsorted = nullptr;
    GraphDesc* descs = nullptr;
    ReduceSpan* spans = nullptr;  // the reduce's workgroup table
    uint32_t cap_spans = 0;
    uint32_t* pos = nullptr;      // list position of every current component
    uint32_t* host_na = nullptr;  // pinned: active components of each round, then the list
                                  // length each round leaves for the next
    hipEvent_t round_ev[2] = {nullptr, nullptr};
};

constexpr uint32_t kMaxRounds = 64;  // R <= 25 for V <= 2^24
constexpr uint32_t kEndBlocks = 1024;

// ctl words
// Q_STOP is set at the end of the first round with no active component; every
// round kernel then returns at once, so the host may enqueue rounds ahead of
// the device without waiting for each round's outcome.
// Q_MULTI: the query spans several graphs; a forest key is then (graph << 32 |
// index), else the 64-bit index alone (wide graphs are queried one at a time).
// Q_DONE counts the workgroups of a round's last kernel that have finished.
enum : uint32_t {
    Q_NL = 0, Q_NA = 1, Q_NL2 = 2, Q_NF = 3, Q_STOP = 4, Q_ROUNDS = 5, Q_MULTI = 6, Q_DONE = 7
};

__device__ __forceinline__ uint64_t forest_key(const uint32_t* __restrict__ ctl, uint32_t graph,
                                               uint64_t idx) {
    return ctl[Q_MULTI] ? ((uint64_t)graph << 32) | idx : idx;
}
__device__ __forceinline__ uint32_t key_graph(const uint32_t* __restrict__ ctl, uint64_t key) {
    return ctl[Q_MULTI] ? (uint32_t)(key >> 32) : 0u;
}
__device__ __forceinline__ uint64_t key_index(const uint32_t* __restrict__ ctl, uint64_t key) {
    return ctl[Q_MULTI] ? (key & 0xFFFFFFFFull) : key;
}

// ---------------------------------------------------------------- kernels --

// Positions in a list whose length counter the whole grid shares: one atomic
// per workgroup.  Same-address atomics from across the chip serialise (the
// compiler already merges a wave's into one), so a list of millions of
// components built with one atomic per wave spent most of its time on them.
// Every thread of the workgroup calls it, in workgroup-uniform control flow;
// threads with take set get distinct positions, the others a value they must
// not use.  sh holds kMaxWaves + 1 words.
constexpr uint32_t kAppendThreads = 1024;
constexpr uint32_t kMaxWaves = kAppendThreads / 64;

__device__ __forceinline__ uint32_t block_append(uint32_t* __restrict__ counter, bool take,
                                                 uint32_t* sh) {
    const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
    const uint64_t m = __ballot(take);
    if (lane == 0) sh[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sum = 0;
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) {
            const uint32_t c = sh[w];
            sh[w] = sum;
            sum += c;
        }
        sh[kMaxWaves] = sum ? atomicAdd(counter, sum) : 0u;
    }
    __syncthreads();
    const uint32_t at = sh[kMaxWaves] + sh[wave] + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    __syncthreads();  // sh is reused by the next call
    return at;
}

__device__ __forceinline__ uint32_t q_graph_of_node(const GraphDesc* __restrict__ gd, uint32_t G,
                                                    uint32_t node) {
    uint32_t lo = 0, hi = G - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (gd[mid].node_base <= node) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void k_q_init(uint32_t T, const GraphDesc* __restrict__ gd, uint32_t G,
                         uint32_t* __restrict__ comp, uint32_t* __restrict__ L,
                         uint32_t* __restrict__ done, uint32_t* __restrict__ gof,
                         uint32_t* __restrict__ ctl) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0) {
        ctl[Q_NL] = T;
        ctl[Q_NA] = 0;
        ctl[Q_NL2] = 0;
        ctl[Q_NF] = 0;
        ctl[Q_STOP] = 0;
        ctl[Q_ROUNDS] = 0;
        ctl[Q_MULTI] = G > 1 ? 1u : 0u;
        ctl[Q_DONE] = 0;
    }
    if (v < T) {
        comp[v] = v;
        L[v] = v;
        done[v] = 0;
        gof[v] = G == 1 ? 0u : q_graph_of_node(gd, G, v);
    }
}

// How a round learns that a component holds every node of its graph: such a
// component's sketch sums every edge twice, so it is zero and the component
// is finished without being reduced or queried (linearity, Sec. 3.1).
enum : uint32_t {
    WHOLE_OFF = 0,     // not tracked
    WHOLE_SINGLE = 1,  // one graph: the list has one entry
    WHOLE_COUNT = 2,   // several graphs: the round before counted each graph's components
};

__global__ __launch_bounds__(kAppendThreads) void k_q_select(
    uint32_t r, const uint32_t* __restrict__ L, uint32_t* __restrict__ ctl,
    uint32_t* __restrict__ done, const uint32_t* __restrict__ gof,
    const GraphDesc* __restrict__ gd, uint32_t* __restrict__ slot, uint32_t* __restrict__ A,
    uint32_t* __restrict__ hook, uint32_t* __restrict__ newlab, uint32_t* __restrict__ merged,
    uint32_t* __restrict__ pos, uint32_t whole_mode, uint32_t G,
    const uint32_t* __restrict__ gcomp_prev, uint32_t* __restrict__ gcomp_next) {
    __shared__ uint32_t sh[kMaxWaves + 1];
    if (ctl[Q_STOP]) return;
    const uint32_t nL = ctl[Q_NL];
    if (whole_mode == WHOLE_COUNT)
        for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < G;
             g += gridDim.x * blockDim.x)
            gcomp_next[g] = 0;
    for (uint32_t i0 = blockIdx.x * blockDim.x; i0 < nL; i0 += gridDim.x * blockDim.x) {
        const uint32_t i = i0 + threadIdx.x;
        bool act = false;
        uint32_t X = 0;
        if (i < nL) {
            X = L[i];
            pos[X] = i;
            hook[X] = kNone;
            newlab[X] = kNone;
            merged[X] = 0;
            const uint32_t g = gof[X];
            act = !done[X] && r < gd[g].R;
            const bool whole = r > 0 && ((whole_mode == WHOLE_SINGLE && nL == 1) ||
                                         (whole_mode == WHOLE_COUNT && gcomp_prev[g] == 1));
            if (act && whole) {
                done[X] = 1;
                act = false;
            }
        }
        const uint32_t a = block_append(&ctl[Q_NA], act, sh);
        if (i < nL) slot[X] = act ? a : kNone;
        if (act) A[a] = X;
    }
}

// XOR the round-r rows of every active component's members into the
// component's accumulator [slot][plane][d][c].  A workgroup takes a span of
// consecutive nodes of one graph and first sorts the span's members by
// component in LDS (a bitonic network over (slot, position) keys; nodes of
// finished components sort last and drop out).  It then walks the members with
// one thread per accumulator word, keeping a running XOR and flushing it when
// the component changes, so a span costs one flush per word for each component
// it meets however the components interleave in node order (in node order, a
// few large interleaved components took one atomic per member).  A span that
// holds its whole graph holds every member of its components: it stores their
// sums, which needs no zeroed accumulator; other spans XOR theirs in with
// atomics into accumulators zeroed before the first reduce and by each query
// after reading them.  Loads are issued kReduceRun members at a time so that
// they are in flight together; blockIdx.y picks the block of accumulator
// words.  Spans of one large graph grow with its size (up to kReduceSpanCap)
// so that its giant component does not take one device-scope atomic per word
// from tens of thousands of workgroups.
constexpr uint32_t kReduceRun = 16;
constexpr uint32_t kReduceSpan = 64;
constexpr uint32_t kReduceSpanCap = 1024;  // spans that cut a graph
constexpr uint32_t kReduceSpanMax = 2048;  // spans that hold a whole graph
constexpr uint32_t kReduceBlocks = 1024;   // spans double while a round takes > 2x this many

uint32_t reduce_span(uint32_t T, uint32_t yblocks) {
    uint32_t span = kReduceSpan;
    while (span < kReduceSpanCap &&
           ((uint64_t)T + span - 1) / span * yblocks > 2ull * kReduceBlocks)
        span *= 2;
    return span;
}

__global__ __launch_bounds__(256) void k_q_reduce(uint32_t r, const ReduceSpan* __restrict__ spans,
                                                  const uint32_t* __restrict__ comp,
                                                  const uint32_t* __restrict__ slot,
                                                  const GraphDesc* __restrict__ gd, uint32_t wpr,
                                                  uint32_t* __restrict__ acc,
                                                  const uint32_t* __restrict__ ctl) {
    __shared__ uint64_t s_key[kReduceSpanMax];  // slot << 32 | position; ~0 if not active
    __shared__ uint32_t s_nact;
    if (ctl[Q_STOP]) return;
    const ReduceSpan sp = spans[blockIdx.x];
    uint32_t np = kReduceSpan;  // sorting width: a power of two >= the span's nodes
    while (np < sp.n) np <<= 1;
    if (threadIdx.x == 0) s_nact = 0;
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < np; t += blockDim.x) {
        uint64_t key = ~0ull;
        if (t < sp.n) {
            const uint32_t sl = slot[comp[sp.v0 + t]];
            if (sl != kNone) key = ((uint64_t)sl << 32) | t;
        }
        s_key[t] = key;
        const uint64_t m = __ballot(key != ~0ull);
        if (__lane_id() == 0 && m) atomicAdd(&s_nact, (uint32_t)__popcll(m));
    }
    __syncthreads();
    for (uint32_t k = 2; k <= np; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < np / 2; i += blockDim.x) {
                const uint32_t lo = ((i & ~(j - 1u)) << 1) | (i & (j - 1u));
                const uint32_t hi = lo + j;
                const uint64_t x = s_key[lo], y = s_key[hi];
                if ((x > y) == ((lo & k) == 0)) {
                    s_key[lo] = y;
                    s_key[hi] = x;
                }
            }
            __syncthreads();
        }
    }
    const uint32_t na = s_nact;
    const GraphDesc& g = gd[sp.graph];
    // word w = (d * planes + plane) * C + c of the round's contiguous rows
    const uint32_t w = blockIdx.y * blockDim.x + threadIdx.x;
    if (w >= g.planes * g.B * kC) return;
    const uint32_t stride = g.node_words;
    const uint32_t* base = g.sk + (uint64_t)(sp.v0 - g.node_base) * stride +
                           (g.round_view ? 0u : sk_word_n(g.planes, g.B, r, 0, 0, 0)) + w;
    const bool whole = sp.whole != 0;
    uint32_t run = 0, run_slot = kNone;
    for (uint32_t b = 0; b < na; b += kReduceRun) {
        uint32_t val[kReduceRun];
#pragma unroll
        for (uint32_t i = 0; i < kReduceRun; ++i) {
            const uint32_t j = b + i;
            val[i] = j < na ? base[(uint64_t)(uint32_t)s_key[j] * stride] : 0u;
        }
#pragma unroll
        for (uint32_t i = 0; i < kReduceRun; ++i) {
            const uint32_t j = b + i;
            const uint32_t sl = j < na ? (uint32_t)(s_key[j] >> 32) : kNone;
            if (sl != kNone && sl != run_slot) {
                if (run_slot != kNone) {
                    uint32_t* dst = &acc[(uint64_t)run_slot * wpr + w];
                    if (whole) *dst = run;
                    else if (run) atomicXor(dst, run);
                }
                run = 0;
                run_slot = sl;
            }
            run ^= val[i];
        }
    }
    if (run_slot != kNone) {
        uint32_t* dst = &acc[(uint64_t)run_slot * wpr + w];
        if (whole) *dst = run;
        else if (run) atomicXor(dst, run);
    }
}

// zero the accumulators of this round's active components (count on the device)
__global__ void k_q_zero_acc(const uint32_t* __restrict__ ctl, uint32_t wpr,
                             uint32_t* __restrict__ acc) {
    if (ctl[Q_STOP]) return;
    const uint64_t n = (uint64_t)ctl[Q_NA] * wpr;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        acc[i] = 0;
}

// kDirect: every component is a single node (first round), read its sketch
// rows in place instead of an accumulator
// One component per 8 lanes (one lane per column): scan the column's nested
// rows from the deepest up (suffix XOR of the exact-depth basis) and keep the
// first good bucket in column-major, row-ascending order; ZERO marks the
// component done, FAIL leaves it without a hook.
constexpr uint32_t kQueryRows = 4;

template <bool kDirect>
__device__ __forceinline__ void query_component(uint32_t r, uint32_t gtid, uint32_t nA,
                                                const uint32_t* __restrict__ A,
                                                uint32_t* __restrict__ acc, uint32_t wpr,
                                                uint32_t zero_after,
                                                const uint32_t* __restrict__ gof,
                                                const GraphDesc* __restrict__ gd,
                                                const uint32_t* __restrict__ comp,
                                                uint32_t* __restrict__ hook,
                                                uint64_t* __restrict__ hedge,
                                                uint32_t* __restrict__ done) {
    const uint32_t a = gtid >> 3;
    const uint32_t c = gtid & 7;
    const bool valid = a < nA;
    uint32_t X = 0, key = kNone, nonempty = 0;
    uint64_t alpha_best = 0;
    if (valid) {
        X = A[a];
        const GraphDesc g = gd[gof[X]];
        const uint32_t p = r * kC + c;
        const uint32_t B = g.B;
        // word (row b, plane) of column c: row b of the round starts at b * planes * C
        const uint32_t* in;
        if (kDirect)
            in = g.sk + (uint64_t)(X - g.node_base) * g.node_words +
                 (g.round_view ? c : sk_word_n(g.planes, B, r, 0, 0, c));
        else
            in = acc + (uint64_t)a * wpr + c;
        // rows are read kQueryRows at a time, deepest first, so that their
        // loads are in flight together; a later (shallower) good row replaces
        // an earlier one
        int b = (int)B - 1;
        if (!g.wide) {
            const PairSeeds s = load_pair_seeds(g.seeds, g.P, p);
            uint32_t al = 0, glo = 0, ghi = 0;
            auto row = [&](int bb, uint32_t xa, uint32_t xg, uint32_t xh) {
                al ^= xa;
                glo ^= xg;
                ghi ^= xh;
                if (al | glo | ghi) {
                    nonempty = 1;
                    if ((uint64_t)al < g.n && chk_lo(s, al) == glo && chk_hi(s, al) == ghi) {
                        key = c * B + (uint32_t)bb;
                        alpha_best = al;
                    }
                }
            };
            for (; b >= (int)kQueryRows - 1; b -= kQueryRows) {
                uint32_t xa[kQueryRows], xg[kQueryRows], xh[kQueryRows];
#pragma unroll
                for (uint32_t q = 0; q < kQueryRows; ++q) {
                    xa[q] = in[((b - q) * kPlanes + 0) * kC];
                    xg[q] = in[((b - q) * kPlanes + 1) * kC];
                    xh[q] = in[((b - q) * kPlanes + 2) * kC];
                }
#pragma unroll
                for (uint32_t q = 0; q < kQueryRows; ++q) row(b - (int)q, xa[q], xg[q], xh[q]);
            }
            for (; b >= 0; --b)
                row(b, in[(b * kPlanes + 0) * kC], in[(b * kPlanes + 1) * kC],
                    in[(b * kPlanes + 2) * kC]);
        } else {
            // 64-bit alpha; the checksum is of the pair the index encodes
            const WideSeeds s = load_wide_seeds(g.seeds, g.P, p);
            uint32_t al = 0, ah = 0, glo = 0, ghi = 0;
            auto row = [&](int bb, uint32_t xa, uint32_t xah, uint32_t xg, uint32_t xh) {
                al ^= xa;
                ah ^= xah;
                glo ^= xg;
                ghi ^= xh;
                if (al | ah | glo | ghi) {
                    nonempty = 1;
                    const uint64_t i = ((uint64_t)ah << 32) | al;
                    if (i < g.n) {
                        uint32_t u, v;
                        edge_pair64(i, &u, &v);
                        if (pair_hash(s.h[2], u, v) == glo && pair_hash(s.h[1], u, v) == ghi) {
                            key = c * B + (uint32_t)bb;
                            alpha_best = i;
                        }
                    }
                }
            };
            for (; b >= (int)kQueryRows - 1; b -= kQueryRows) {
                uint32_t xa[kQueryRows], xah[kQueryRows], xg[kQueryRows], xh[kQueryRows];
#pragma unroll
                for (uint32_t q = 0; q < kQueryRows; ++q) {
                    xa[q] = in[((b - q) * kPlanesWide + 0) * kC];
                    xah[q] = in[((b - q) * kPlanesWide + 1) * kC];
                    xg[q] = in[((b - q) * kPlanesWide + 2) * kC];
                    xh[q] = in[((b - q) * kPlanesWide + 3) * kC];
                }
#pragma unroll
                for (uint32_t q = 0; q < kQueryRows; ++q)
                    row(b - (int)q, xa[q], xah[q], xg[q], xh[q]);
            }
            for (; b >= 0; --b)
                row(b, in[(b * kPlanesWide + 0) * kC], in[(b * kPlanesWide + 1) * kC],
                    in[(b * kPlanesWide + 2) * kC], in[(b * kPlanesWide + 3) * kC]);
        }
        // the next round's atomics find this accumulator zeroed (its slots
        // are a subset of this round's)
        if (!kDirect && zero_after) {
            uint32_t* w = acc + (uint64_t)a * wpr + c;
            for (uint32_t k = 0; k < g.planes * B; ++k) w[k * kC] = 0;
        }
    }
    // reduce over the 8 lanes of this component: smallest key, any non-empty
    for (uint32_t off = 1; off < 8; off <<= 1) {
        const uint32_t k2 = __shfl_xor(key, off, 8);
        const uint32_t alo2 = __shfl_xor((uint32_t)alpha_best, off, 8);
        const uint32_t ahi2 = __shfl_xor((uint32_t)(alpha_best >> 32), off, 8);
        const uint32_t n2 = __shfl_xor(nonempty, off, 8);
        if (k2 < key) {
            key = k2;
            alpha_best = ((uint64_t)ahi2 << 32) | alo2;
        }
        nonempty |= n2;
    }
    if (!valid || c != 0) return;
    if (!nonempty) {  // ZERO: no edge leaves X
        done[X] = 1;
        return;
    }
    if (key == kNone) return;  // FAIL
    uint32_t u, v;
    edge_pair64(alpha_best, &u, &v);
    const GraphDesc g = gd[gof[X]];
    const uint32_t cu = comp[g.node_base + u], cv = comp[g.node_base + v];
    const bool iu = cu == X, iv = cv == X;
    if (iu == iv) return;  // the edge does not leave X: treated as FAIL
    hook[X] = iu ? cv : cu;
    hedge[X] = alpha_best;
}

// kDirect: every component is a single node (first round), read its sketch
// rows in place instead of an accumulator.  The grid strides over the active
// components (their count is known only on the device).
template <bool kDirect>
__global__ void k_q_query(uint32_t r, const uint32_t* __restrict__ A, const uint32_t* __restrict__ ctl,
                          uint32_t* __restrict__ acc, uint32_t wpr, uint32_t zero_after,
                          const uint32_t* __restrict__ gof, const GraphDesc* __restrict__ gd,
                          const uint32_t* __restrict__ comp, uint32_t* __restrict__ hook,
                          uint64_t* __restrict__ hedge, uint32_t* __restrict__ done) {
    if (ctl[Q_STOP]) return;
    const uint32_t nA = ctl[Q_NA];
    const uint64_t lanes = (uint64_t)nA * 8;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < lanes;
         base += (uint64_t)gridDim.x * blockDim.x)
        query_component<kDirect>(r, (uint32_t)(base + threadIdx.x), nA, A, acc, wpr, zero_after,
                                 gof, gd, comp, hook, hedge, done);
}

__global__ void k_q_double_init(const uint32_t* __restrict__ L, const uint32_t* __restrict__ ctl,
                                const uint32_t* __restrict__ hook, uint32_t* __restrict__ s,
                                uint32_t* __restrict__ m, uint32_t lds_cap) {
    if (ctl[Q_STOP]) return;
    const uint32_t nL = ctl[Q_NL];
    if (nL <= lds_cap) return;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nL; i += gridDim.x * blockDim.x) {
        const uint32_t X = L[i];
        const uint32_t h = hook[X];
        s[X] = h == kNone ? X : h;
        m[X] = X;
    }
}

// one doubling step: s2 = s o s, m2 = min(m, m o s)
__global__ void k_q_double(const uint32_t* __restrict__ L, const uint32_t* __restrict__ ctl,
                           const uint32_t* __restrict__ s, const uint32_t* __restrict__ m,
                           uint32_t* __restrict__ s2, uint32_t* __restrict__ m2,
                           uint32_t lds_cap) {
    if (ctl[Q_STOP]) return;
    const uint32_t nL = ctl[Q_NL];
    if (nL <= lds_cap) return;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nL; i += gridDim.x * blockDim.x) {
        const uint32_t X = L[i];
        const uint32_t y = s[X];
        s2[X] = s[y];
        m2[X] = min(m[X], m[y]);
    }
}

// all K doubling steps in one workgroup (lists of up to a few ten thousand
// components): the arrays stay in global memory, visible to the whole
// workgroup after each barrier; ping-pong between (s, m) and (s2, m2)
__global__ __launch_bounds__(1024) void k_q_double_all(const uint32_t* __restrict__ L,
                                                        const uint32_t* __restrict__ ctl,
                                                        uint32_t K, uint32_t* s, uint32_t* m,
                                                        uint32_t* s2, uint32_t* m2,
                                                        uint32_t lds_cap) {
    if (ctl[Q_STOP]) return;
    const uint32_t nL = ctl[Q_NL];
    if (nL <= lds_cap) return;
    // A step that changes nothing leaves both buffers equal on the list (so
    // the caller's choice of buffer by the parity of K still holds) and has
    // reached the K-step result: every successor then lies on a cycle whose
    // length divides 2^k, and its minimum spans that cycle.
    for (uint32_t k = 0; k < K; ++k) {
        uint32_t* si = (k & 1) ? s2 : s;
        uint32_t* mi = (k & 1) ? m2 : m;
        uint32_t* so = (k & 1) ? s : s2;
        uint32_t* mo = (k & 1) ? m : m2;
        int changed = 0;
        for (uint32_t i = threadIdx.x; i < nL; i += blockDim.x) {
            const uint32_t X = L[i];
            const uint32_t y = si[X];
            const uint32_t ns = si[y], nm = min(mi[X], mi[y]);
            changed |= (ns != y) | (nm != mi[X]);
            so[X] = ns;
            mo[X] = nm;
        }
        if (!__syncthreads_or(changed)) break;
    }
}

// newlab[R] = min(newlab[R], X).  A label only decreases, so a plain read that
// is already at or below X (stale or not) makes the atomic a no-op; skipping it
// spares the root of a large tree one serialised atomic per member.  Callers
// also skip members above R: R itself takes part, so the label ends at most R.
__device__ __forceinline__ void label_min(uint32_t* __restrict__ lab, uint32_t X) {
    if (X < *lab) atomicMin(lab, X);
}

// after enough doubling steps s[X] lies on X's terminal cycle and m[s[X]] is
// that cycle's smallest component: the root of X's tree once its edge is cut
__global__ __launch_bounds__(kAppendThreads) void k_q_root(
    const uint32_t* __restrict__ L, uint32_t* __restrict__ ctl, const uint32_t* __restrict__ s,
    const uint32_t* __restrict__ m, const uint32_t* __restrict__ hook,
    const uint64_t* __restrict__ hedge, const uint32_t* __restrict__ gof,
    uint32_t* __restrict__ rootOf, uint32_t* __restrict__ newlab, uint32_t* __restrict__ merged,
    uint64_t* __restrict__ forest, uint32_t lds_cap) {
    __shared__ uint32_t sh[kMaxWaves + 1];
    if (ctl[Q_STOP]) return;
    const uint32_t nL = ctl[Q_NL];
    if (nL <= lds_cap) return;
    for (uint32_t i0 = blockIdx.x * blockDim.x; i0 < nL; i0 += gridDim.x * blockDim.x) {
        const uint32_t i = i0 + threadIdx.x;
        bool kept = false;
        uint32_t X = 0;
        if (i < nL) {
            X = L[i];
            const uint32_t R = m[s[X]];
            rootOf[X] = R;
            if (X <= R) label_min(&newlab[R], X);
            kept = hook[X] != kNone && X != R;
            if (kept) merged[R] = 1;
        }
        const uint32_t f = block_append(&ctl[Q_NF], kept, sh);
        if (kept) forest[f] = forest_key(ctl, gof[X], hedge[X]);
    }
}

// The same resolution for lists of up to kLdsResolve components in one
// workgroup, with the successor and running minimum packed in one 64-bit LDS
// word per component (list position of the successor, minimum id above it).
// Doubling runs in place: a lane reads its successor's (position, minimum)
// pair in one access, so its word always describes one path segment
// [X, successor) and its minimum; in-place steps advance at least as far as
// synchronous ones, so K steps still reach every terminal cycle.
// When every node id of the query fits 16 bits (T <= 65536) the pair packs
// into 32 bits: half the LDS traffic of the doubling, and lists of up to
// kLdsResolveNarrow components fit one workgroup.
constexpr uint32_t kLdsResolve = 16384;
constexpr uint32_t kLdsResolveNarrow = 36864;
constexpr uint32_t kResolveBatch = 8;

template <bool kNarrowIds>
__global__ __launch_bounds__(1024) void k_q_resolve_lds(
    const uint32_t* __restrict__ L, uint32_t* __restrict__ ctl, uint32_t K,
    const uint32_t* __restrict__ hook, const uint64_t* __restrict__ hedge,
    const uint32_t* __restrict__ pos, const uint32_t* __restrict__ gof,
    uint32_t* __restrict__ rootOf, uint32_t* __restrict__ newlab, uint32_t* __restrict__ merged,
    uint64_t* __restrict__ forest) {
    using W = typename std::conditional<kNarrowIds, uint32_t, uint64_t>::type;
    constexpr uint32_t kCap = kNarrowIds ? kLdsResolveNarrow : kLdsResolve;
    constexpr uint32_t kS = kNarrowIds ? 16u : 32u;  // minimum << kS | successor position
    constexpr W kPosMask = ((W)1 << kS) - 1;
    __shared__ W st[kCap];
    if (ctl[Q_STOP]) return;
    const uint32_t nL = ctl[Q_NL];
    if (nL > kCap) return;
    const uint32_t bd = blockDim.x;
    // global loads in batches of kResolveBatch per lane, so that a lane waits
    // once per dependent step of a batch rather than once per component
    for (uint32_t i0 = threadIdx.x; i0 < nL; i0 += kResolveBatch * bd) {
        uint32_t X[kResolveBatch], h[kResolveBatch], sp[kResolveBatch];
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q) {
            const uint32_t i = i0 + q * bd;
            X[q] = i < nL ? L[i] : 0u;
        }
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q)
            h[q] = i0 + q * bd < nL ? hook[X[q]] : kNone;
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q)
            sp[q] = h[q] == kNone ? i0 + q * bd : pos[h[q]];
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q)
            if (i0 + q * bd < nL) st[i0 + q * bd] = ((W)X[q] << kS) | sp[q];
    }
    __syncthreads();
    // A path to a cycle and the cycle hold at most nL components.  A step that
    // changes no word has reached a fixed point: every successor is then a word
    // whose segment starts and ends at itself, a root (empty segment) or a whole
    // number of turns of its cycle (minimum = the cycle's), so the roots below
    // are those the remaining steps would give.
    const uint32_t steps = min(K, nL > 1 ? 32u - (uint32_t)__clz(nL - 1) : 0u);
    for (uint32_t k = 0; k < steps; ++k) {
        int changed = 0;
        for (uint32_t i0 = threadIdx.x; i0 < nL; i0 += 4 * bd) {
            W v[4], w[4];
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q) v[q] = i0 + q * bd < nL ? st[i0 + q * bd] : (W)0;
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q) w[q] = st[(uint32_t)(v[q] & kPosMask)];
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q)
                if (i0 + q * bd < nL) {
                    const W nv = (min(v[q] >> kS, w[q] >> kS) << kS) | (w[q] & kPosMask);
                    changed |= nv != v[q];
                    st[i0 + q * bd] = nv;
                }
        }
        if (!__syncthreads_or(changed)) break;
    }
    // roots and new labels; the kept hook edges are counted first so that one
    // atomic and a workgroup scan place them (an atomic that returns a value
    // costs a round trip, one per component was most of this kernel's time)
    auto root_at = [&](uint32_t i) { return (uint32_t)(st[(uint32_t)(st[i] & kPosMask)] >> kS); };
    uint32_t cnt = 0;
    for (uint32_t i0 = threadIdx.x; i0 < nL; i0 += kResolveBatch * bd) {
        uint32_t X[kResolveBatch], h[kResolveBatch];
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q) X[q] = i0 + q * bd < nL ? L[i0 + q * bd] : 0u;
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q)
            h[q] = i0 + q * bd < nL ? hook[X[q]] : kNone;
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q)
            cnt += (h[q] != kNone && X[q] != root_at(i0 + q * bd)) ? 1u : 0u;
    }
    __shared__ uint32_t s_scan[kMaxWaves + 1];
    const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
    uint32_t incl = cnt;
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    if (lane == 63) s_scan[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sum = 0;
        for (uint32_t w = 0; w < (bd >> 6); ++w) {
            const uint32_t c = s_scan[w];
            s_scan[w] = sum;
            sum += c;
        }
        s_scan[kMaxWaves] = sum ? atomicAdd(&ctl[Q_NF], sum) : 0u;
    }
    __syncthreads();
    uint32_t f = s_scan[kMaxWaves] + s_scan[wave] + incl - cnt;
    for (uint32_t i0 = threadIdx.x; i0 < nL; i0 += kResolveBatch * bd) {
        uint32_t X[kResolveBatch], h[kResolveBatch], R[kResolveBatch], lab[kResolveBatch];
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q) X[q] = i0 + q * bd < nL ? L[i0 + q * bd] : 0u;
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q) {
            const bool in = i0 + q * bd < nL;
            h[q] = in ? hook[X[q]] : kNone;
            R[q] = in ? root_at(i0 + q * bd) : 0u;
        }
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q)
            lab[q] = i0 + q * bd < nL ? newlab[R[q]] : 0u;
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q) {
            if (i0 + q * bd >= nL) continue;
            rootOf[X[q]] = R[q];
            if (X[q] <= R[q] && X[q] < lab[q]) atomicMin(&newlab[R[q]], X[q]);  // label_min
        }
#pragma unroll
        for (uint32_t q = 0; q < kResolveBatch; ++q) {
            if (h[q] == kNone || X[q] == R[q]) continue;  // also every position >= nL
            merged[R[q]] = 1;
            forest[f++] = forest_key(ctl, gof[X[q]], hedge[X[q]]);
        }
    }
}

// The first round of a query over several graphs of at most kGraphResolve
// nodes: one workgroup per graph resolves its hooks in LDS, as
// k_q_resolve_lds does for one list.  In that round the list is every node in
// order, so a graph's components are its node range and every hook stays in
// it; this replaces the grid-wide doubling (a dozen launches over millions of
// components).
// The same kernel, one workgroup of 1024 lanes, takes the first round of a
// single graph of up to kGraphResolveOne nodes (the list is every node then
// too), in place of the list-indexed k_q_resolve_lds.
constexpr uint32_t kGraphResolve = 4096;
constexpr uint32_t kGraphResolveThreads = 256;
constexpr uint32_t kGraphResolveOne = 16384;

template <uint32_t kCap, uint32_t kThreads>
__global__ __launch_bounds__(kThreads) void k_q_resolve_graphs(
    const GraphDesc* __restrict__ gd, uint32_t* __restrict__ ctl,
    const uint32_t* __restrict__ hook, const uint64_t* __restrict__ hedge,
    uint32_t* __restrict__ rootOf, uint32_t* __restrict__ newlab, uint32_t* __restrict__ merged,
    uint64_t* __restrict__ forest) {
    // a lane's nodes are tid + q * blockDim for q < kItems; their hooks stay in
    // registers and every global load is issued for all of them at once
    constexpr uint32_t kItems = kCap / kThreads;
    __shared__ uint64_t st[kCap];
    __shared__ uint32_t s_scan[kThreads / 64 + 1];
    if (ctl[Q_STOP]) return;
    const uint32_t graph = blockIdx.x, tid = threadIdx.x, bd = blockDim.x;
    const uint32_t n = gd[graph].V, v0 = gd[graph].node_base;
    uint32_t h[kItems];
#pragma unroll
    for (uint32_t q = 0; q < kItems; ++q) h[q] = tid + q * bd < n ? hook[v0 + tid + q * bd] : kNone;
#pragma unroll
    for (uint32_t q = 0; q < kItems; ++q) {
        const uint32_t i = tid + q * bd;
        if (i < n) st[i] = ((uint64_t)(v0 + i) << 32) | (h[q] == kNone ? i : h[q] - v0);
    }
    __syncthreads();
    // in-place doubling with the fixed-point stop of k_q_resolve_lds
    const uint32_t steps = n > 1 ? 32u - (uint32_t)__clz(n - 1) : 0u;
    for (uint32_t k = 0; k < steps; ++k) {
        int changed = 0;
        for (uint32_t i = tid; i < n; i += bd) {
            const uint64_t v = st[i];
            const uint64_t w = st[(uint32_t)v];
            const uint64_t nv = (min(v >> 32, w >> 32) << 32) | (uint32_t)w;
            changed |= nv != v;
            st[i] = nv;
        }
        if (!__syncthreads_or(changed)) break;
    }
    // roots, and the kept hook edges: counted, then placed with one atomic per graph
    uint32_t R[kItems], cnt = 0;
#pragma unroll
    for (uint32_t q = 0; q < kItems; ++q) {
        const uint32_t i = tid + q * bd;
        R[q] = i < n ? (uint32_t)(st[(uint32_t)st[i]] >> 32) : 0u;
        cnt += (h[q] != kNone && v0 + i != R[q]) ? 1u : 0u;  // h is kNone past n
    }
    const uint32_t lane = __lane_id(), wave = tid >> 6;
    uint32_t incl = cnt;
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    if (lane == 63) s_scan[wave] = incl;
    __syncthreads();
    if (tid == 0) {
        uint32_t sum = 0;
        for (uint32_t w = 0; w < (bd >> 6); ++w) {
            const uint32_t c = s_scan[w];
            s_scan[w] = sum;
            sum += c;
        }
        s_scan[bd >> 6] = sum ? atomicAdd(&ctl[Q_NF], sum) : 0u;
    }
    __syncthreads();
    uint32_t f = s_scan[bd >> 6] + s_scan[wave] + incl - cnt;
    uint32_t lab[kItems];
    uint64_t e[kItems];
#pragma unroll
    for (uint32_t q = 0; q < kItems; ++q) {
        const uint32_t i = tid + q * bd;
        const bool kept = h[q] != kNone && v0 + i != R[q];
        lab[q] = i < n && v0 + i <= R[q] ? newlab[R[q]] : 0u;
        e[q] = kept ? hedge[v0 + i] : 0ull;
    }
#pragma unroll
    for (uint32_t q = 0; q < kItems; ++q) {
        const uint32_t i = tid + q * bd;
        if (i >= n) continue;
        const uint32_t X = v0 + i;
        rootOf[X] = R[q];
        if (X <= R[q] && X < lab[q]) atomicMin(&newlab[R[q]], X);  // as label_min
        if (h[q] != kNone && X != R[q]) {
            merged[R[q]] = 1;
            forest[f++] = forest_key(ctl, graph, e[q]);
        }
    }
}

// The next round's component list: the roots of this round's trees, and every
// node's new label (the relabel of the round).  The last workgroup to finish
// also ends the round: it publishes the round's active
// count and the new list length to the host (pinned memory), makes the new
// list current, and stops the query once a round had no active component.
__global__ __launch_bounds__(kAppendThreads) void k_q_newcomps(
    uint32_t r, uint32_t T, uint32_t* __restrict__ comp, const uint32_t* __restrict__ L,
    uint32_t* __restrict__ ctl, const uint32_t* __restrict__ rootOf,
    const uint32_t* __restrict__ newlab, const uint32_t* __restrict__ merged,
    uint32_t* __restrict__ done, uint32_t* __restrict__ L2, uint32_t* __restrict__ host_na,
    const uint32_t* __restrict__ gof, uint32_t* __restrict__ gcomp_next) {
    __shared__ uint32_t sh[kMaxWaves + 1];
    __shared__ uint32_t s_last;
    if (ctl[Q_STOP]) return;
    const uint32_t nL = ctl[Q_NL];
    for (uint32_t i0 = blockIdx.x * blockDim.x; i0 < nL; i0 += gridDim.x * blockDim.x) {
        const uint32_t i = i0 + threadIdx.x;
        bool root = false;
        uint32_t X = 0;
        if (i < nL) {
            X = L[i];
            const uint32_t R = rootOf[X];
            root = newlab[R] == X;
            if (root && merged[R]) done[X] = 0;
        }
        const uint32_t at = block_append(&ctl[Q_NL2], root, sh);
        if (root) L2[at] = X;
        if (gcomp_next) {
            // each graph's components, one atomic per graph a wave meets
            const uint32_t g = root ? gof[X] : kNone;
            uint64_t pending = __ballot(root);
            while (pending) {
                const uint32_t leader = (uint32_t)__ffsll((unsigned long long)pending) - 1u;
                const uint32_t gl = __shfl(g, (int)leader);
                const uint64_t same = __ballot(root && g == gl);
                if (__lane_id() == leader) atomicAdd(&gcomp_next[gl], (uint32_t)__popcll(same));
                pending &= ~same;
            }
        }
    }
    // every node's label: the new label of its component's tree
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < T; v += gridDim.x * blockDim.x)
        comp[v] = newlab[rootOf[comp[v]]];
    // No fence: the last workgroup reads only counters that every workgroup
    // updated with atomics it waited for (block_append uses the result)
    // before counting itself done; the list and the counters it writes reach
    // the next kernel at the kernel boundary.  (A device-scope fence in every
    // workgroup cost tens of microseconds per launch.)
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(&ctl[Q_DONE], 1u) == gridDim.x - 1;
    __syncthreads();
    if (!s_last || threadIdx.x != 0) return;
    const uint32_t na = atomicAdd(&ctl[Q_NA], 0u);
    const uint32_t nl = atomicAdd(&ctl[Q_NL2], 0u);
    if (na == 0) ctl[Q_STOP] = 1;
    else ctl[Q_ROUNDS] = r + 1;
    ctl[Q_NL] = nl;
    ctl[Q_NL2] = 0;
    ctl[Q_NA] = 0;
    ctl[Q_DONE] = 0;
    host_na[r] = na;
    host_na[kMaxRounds + r] = nl;
}

__global__ void k_q_finish(const uint32_t* __restrict__ L, const uint32_t* __restrict__ ctl,
                           const uint32_t* __restrict__ done, const uint32_t* __restrict__ gof,
                           uint32_t* __restrict__ gcount, uint32_t* __restrict__ gfail) {
    const uint32_t nL = ctl[Q_NL];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nL; i += gridDim.x * blockDim.x) {
        const uint32_t X = L[i];
        const uint32_t g = gof[X];
        const bool open = !done[X];
        // lanes of one graph (neighbours in the list, mostly) add with one
        // atomic: same-address atomics from every lane serialise
        uint64_t pending = __ballot(true);
        while (pending) {
            const uint32_t leader = (uint32_t)__ffsll((unsigned long long)pending) - 1u;
            const uint32_t gl = __shfl(g, (int)leader);
            const uint64_t same = __ballot(g == gl);
            const uint64_t fail = __ballot(open && g == gl);
            if (__lane_id() == leader) {
                atomicAdd(&gcount[gl], (uint32_t)__popcll(same));
                if (fail) atomicOr(&gfail[gl], 1u);
            }
            pending &= ~same;
        }
    }
}

__global__ void k_q_labels(uint32_t T, const uint32_t* __restrict__ comp,
                           const uint32_t* __restrict__ gof, const GraphDesc* __restrict__ gd,
                           uint32_t* __restrict__ out) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < T; v += gridDim.x * blockDim.x)
        out[v] = comp[v] - gd[gof[v]].node_base;
}

// forest: keys per graph (their offsets in the output), then the keys sorted
__global__ void k_q_fcount(const uint64_t* __restrict__ forest, const uint32_t* __restrict__ ctl,
                           uint32_t* __restrict__ fcnt) {
    const uint32_t nF = ctl[Q_NF];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nF; i += gridDim.x * blockDim.x)
        atomicAdd(&fcnt[key_graph(ctl, forest[i])], 1u);
}

__global__ void k_q_fscan(const uint32_t* __restrict__ fcnt, uint32_t G, uint32_t* __restrict__ foff,
                          uint32_t* __restrict__ fcur) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t g = 0; g < G; ++g) {
            const uint32_t c = fcnt[g];
            foff[g] = acc;
            fcur[g] = acc;
            acc += c;
        }
        foff[G] = acc;
    }
}

constexpr uint32_t kSingleBlockDoubling = 65536;  // component lists up to this length

// The forest keys (distinct: the graph above the edge index when several graphs
// are queried) are sorted ascending, which orders them by graph and, within a
// graph, by edge index: tiles of kFTile keys are sorted in LDS by a bitonic
// network, then runs of width w, 2w, ... are merged pairwise, each key placed
// at its index in its run plus the number of keys of the partner run below it
// (a binary search), so every pass is one read and one write per key.
constexpr uint32_t kFTile = 2048;

__global__ __launch_bounds__(1024) void k_q_fsort_tile(uint64_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ ctl) {
    __shared__ uint64_t t[kFTile];
    const uint32_t nF = ctl[Q_NF];
    const uint32_t base = blockIdx.x * kFTile;
    if (base >= nF) return;
    const uint32_t n = min(kFTile, nF - base);
    for (uint32_t i = threadIdx.x; i < kFTile; i += blockDim.x)
        t[i] = i < n ? keys[base + i] : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= kFTile; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t q = threadIdx.x; q < kFTile / 2; q += blockDim.x) {
                const uint32_t i = 2 * q - (q & (j - 1));  // lower element of the pair
                const uint64_t x = t[i], y = t[i + j];
                const bool up = (i & k) == 0;
                if ((x > y) == up) {
                    t[i] = y;
                    t[i + j] = x;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) keys[base + i] = t[i];
}

__global__ void k_q_fmerge(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                           const uint32_t* __restrict__ ctl, uint32_t w) {
    const uint32_t nF = ctl[Q_NF];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nF; i += gridDim.x * blockDim.x) {
        const uint32_t run = i / w;
        const uint32_t a0 = (run & ~1u) * w;
        const uint32_t b0 = min(a0 + w, nF), b1 = min(b0 + w, nF);
        const uint64_t x = in[i];
        // the partner run: B for keys of A, A for keys of B
        uint32_t lo = (run & 1u) ? a0 : b0;
        uint32_t hi = (run & 1u) ? b0 : b1;
        const uint32_t first = lo;
        while (lo < hi) {  // first partner key above x (keys are distinct)
            const uint32_t mid = (lo + hi) >> 1;
            if (in[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        const uint32_t own = (run & 1u) ? i - b0 : i - a0;
        out[a0 + own + (lo - first)] = x;
    }
}

// sorted keys -> (u, v) pairs
__global__ void k_q_fpairs(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ ctl,
                           uint32_t* __restrict__ pairs) {
    const uint32_t nF = ctl[Q_NF];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nF; i += gridDim.x * blockDim.x) {
        uint32_t u, v;
        edge_pair64(key_index(ctl, keys[i]), &u, &v);
        pairs[2 * i] = u;
        pairs[2 * i + 1] = v;
    }
}

// ------------------------------------------------------------------- host --

namespace {

template <typename T>
gz_status qalloc(T** p, uint64_t n) {
    if (*p) GZ_HIP(hipFree(*p));
    *p = nullptr;
    if (hipMalloc((void**)p, std::max<uint64_t>(n, 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return fail(GZ_ENOMEM, "out of device memory for the query scratch");
    }
    return GZ_OK;
}

gz_status ensure_query(QueryScratch& Q, uint32_t T, uint32_t G, uint32_t wpr) {
    int dev = 0;
    GZ_HIP(hipGetDevice(&dev));
    Q.device = dev;
    gz_status st;
    if (T > Q.cap_nodes || !Q.comp) {
        uint32_t** arrs[] = {&Q.comp, &Q.L, &Q.L2, &Q.A, &Q.slot, &Q.done, &Q.hook,
                             &Q.s, &Q.s2, &Q.m, &Q.m2, &Q.rootOf, &Q.newlab, &Q.merged, &Q.gof,
                             &Q.labels, &Q.pos};
        for (auto a : arrs)
            if ((st = qalloc(a, T))) return st;
        if ((st = qalloc(&Q.fpairs, 2ull * T))) return st;
        if ((st = qalloc(&Q.hedge, T))) return st;
        if ((st = qalloc(&Q.forest, T))) return st;
        if ((st = qalloc(&Q.fsorted, T))) return st;
        if (!Q.ctl && (st = qalloc(&Q.ctl, 8))) return st;
        if (!Q.host_na) GZ_HIP(hipHostMalloc((void**)&Q.host_na, 8 * kMaxRounds, hipHostMallocDefault));
        for (hipEvent_t& e : Q.round_ev)
            if (!e) GZ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        Q.cap_nodes = T;
        Q.cap_wpr = 0;
    }
    if (wpr > Q.cap_wpr || !Q.acc) {
        if ((st = qalloc(&Q.acc, (uint64_t)T * wpr))) return st;
        Q.cap_wpr = wpr;
    }
    if (G > Q.cap_graphs || !Q.descs) {
        if ((st = qalloc(&Q.descs, G))) return st;
        if ((st = qalloc(&Q.gcount, G))) return st;
        if ((st = qalloc(&Q.gcomp, 2ull * G))) return st;
        if ((st = qalloc(&Q.gfail, G))) return st;
        if ((st = qalloc(&Q.foff, (uint64_t)G + 1))) return st;
        if ((st = qalloc(&Q.fcur, G))) return st;
        if ((st = qalloc(&Q.fcnt, G))) return st;
        Q.cap_graphs = G;
    }
    return GZ_OK;
}

uint32_t blocks_for(uint64_t n, uint32_t threads) {
    uint64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 65535) b = 65535;
    return (uint32_t)b;
}

uint32_t bitlen32(uint32_t x) {
    uint32_t n = 0;
    while (x) { ++n; x >>= 1; }
    return n;
}

}  // namespace

void free_query_scratch(QueryScratch* q) {
    if (!q) return;
    hipFree(q->hedge);
    uint32_t* arrs[] = {q->comp, q->L, q->L2, q->A, q->slot, q->done, q->hook, q->s,
                        q->s2, q->m, q->m2, q->rootOf, q->newlab, q->merged, q->gof, q->acc,
                        q->ctl, q->labels, q->gcount, q->gfail, q->foff, q->fcur, q->fpairs,
                        q->fcnt, q->pos};
    for (auto a : arrs) hipFree(a);
    hipFree(q->forest);
    hipFree(q->fsorted);
    hipFree(q->descs);
    hipFree(q->spans);
    if (q->host_na) hipHostFree(q->host_na);
    for (hipEvent_t e : q->round_ev)
        if (e) hipEventDestroy(e);
    delete q;
}

// Fused queries share a few scratch sets per device, so that runs on several
// threads need not wait for each other and no graph holds query memory of its
// own (allocating and freeing it while other work runs would stall the device).
// A run holds its set's lock until its stream has finished with the set.
QueryScratch& shared_query_scratch(int device, std::unique_lock<std::mutex>& lock) {
    // never destroyed: nothing of the library is torn down by static destructors
    // at process exit (device memory still held then goes with the process)
    constexpr size_t kDevices = 64, kSets = 4;
    static std::vector<std::mutex>* mus = new std::vector<std::mutex>(kDevices * kSets);
    static std::vector<QueryScratch>* sets = new std::vector<QueryScratch>(kDevices * kSets);
    const size_t base = (size_t)device % kDevices * kSets;
    for (size_t i = 0; i < kSets; ++i) {
        std::unique_lock<std::mutex> l((*mus)[base + i], std::try_to_lock);
        if (l.owns_lock()) {
            lock = std::move(l);
            return (*sets)[base + i];
        }
    }
    lock = std::unique_lock<std::mutex>((*mus)[base]);
    return (*sets)[base];
}

gz_status boruvka(gz_graph* const* gs, uint32_t G, bool want_forest, QueryResult& out,
                  uint32_t* labels_out, bool shared_scratch) {
    if (G == 0) return fail(GZ_EINVAL, "no graphs");
    std::vector<GraphDesc> descs(G);
    uint64_t T64 = 0;
    uint32_t Rmax = 0, Bmax = 0, Vmax = 0, PLmax = 0;
    for (uint32_t k = 0; k < G; ++k) {
        const gz_graph* g = gs[k];
        if (!g) return fail(GZ_EINVAL, "null graph handle");
        descs[k] = GraphDesc{};
        descs[k].sk = g->sk;
        descs[k].seeds = g->seeds;
        descs[k].n = g->n;
        descs[k].V = g->V;
        descs[k].R = g->R;
        descs[k].B = g->B;
        descs[k].P = g->P;
        descs[k].node_base = (uint32_t)T64;
        descs[k].node_words = g->planes * g->B * g->P;
        descs[k].wide = g->wide;
        descs[k].planes = g->planes;
        T64 += g->V;
        Rmax = std::max(Rmax, g->R);
        Bmax = std::max(Bmax, g->B);
        Vmax = std::max(Vmax, g->V);
        PLmax = std::max(PLmax, g->planes);
        if (G > 1 && g->wide)
            return fail(GZ_EINVAL, "graphs with V > 65536 are queried one at a time");
    }
    if (T64 >= (1ull << 31)) return fail(GZ_EINVAL, "too many nodes in one query");
    // a host-tier graph is queried alone: every round its round slabs are
    // copied into a device buffer that the round's kernels read in place of
    // the node blocks
    gz_graph* tier_g = G == 1 && gs[0]->tier ? gs[0] : nullptr;
    if (!tier_g)
        for (uint32_t k = 0; k < G; ++k)
            if (gs[k]->tier) return fail(GZ_EINVAL, "host-tier graphs are queried one at a time");
    if (Rmax > kMaxRounds) return fail(GZ_EINVAL, "too many rounds");
    const uint32_t T = (uint32_t)T64;
    const uint32_t wpr = PLmax * Bmax * kC;

    // single-graph queries keep the graph's own scratch; fused ones (of any
    // number of graphs) take a shared set
    std::unique_lock<std::mutex> lock;
    QueryScratch* Q = nullptr;
    if (!shared_scratch) {
        if (!gs[0]->q) gs[0]->q = new QueryScratch();
        Q = gs[0]->q;
    } else {
        int dev = 0;
        GZ_HIP(hipGetDevice(&dev));
        Q = &shared_query_scratch(dev, lock);
    }
    gz_status st = ensure_query(*Q, T, G, wpr);
    if (st) return st;

    hipStream_t qs = nullptr;
    GZ_HIP(query_stream(gs[0], &qs));
    GZ_HIP(fence_wait(qs, gs, G));
    if (tier_g) {
        uint32_t* buf = nullptr;
        GZ_TRY(tier_round(tier_g, 0, qs, &buf));
        descs[0].sk = buf;
        descs[0].node_words = tier_g->planes * tier_g->B * kC;
        descs[0].round_view = 1;
    }
    GZ_HIP(hipMemcpyAsync(Q->descs, descs.data(), sizeof(GraphDesc) * G, hipMemcpyHostToDevice, qs));
    const uint32_t tb = blocks_for(T, 256);
    const uint32_t ta = blocks_for(T, kAppendThreads);
    k_q_init<<<(T + 255) / 256, 256, 0, qs>>>(T, Q->descs, G, Q->comp, Q->L, Q->done, Q->gof,
                                               Q->ctl);
    const uint32_t K = std::max(1u, bitlen32(Vmax - 1));  // 2^K >= any tail + cycle length
    uint32_t* s = Q->s;
    uint32_t* s2 = Q->s2;
    uint32_t* m = Q->m;
    uint32_t* m2 = Q->m2;
    const uint32_t qgrid = blocks_for(8ull * T, 256);
    const uint32_t zgrid = 2048;
    const uint32_t ry = (wpr + 255) / 256;
    // reduce workgroups: spans of consecutive nodes of one graph; several
    // graphs that each fit kReduceSpanMax nodes take one span per graph, so
    // that no accumulator needs zeroing or atomics
    uint32_t rspan = reduce_span(T, ry);
    if (G > 1 && Vmax <= kReduceSpanMax) {
        rspan = kReduceSpan;
        while (rspan < Vmax) rspan <<= 1;
    }
    std::vector<ReduceSpan> spans;
    bool all_whole = true;
    for (uint32_t k = 0; k < G; ++k) {
        const uint32_t V = descs[k].V;
        for (uint32_t v = 0; v < V; v += rspan)
            spans.push_back(ReduceSpan{descs[k].node_base + v, std::min(rspan, V - v), k,
                                       V <= rspan ? 1u : 0u});
        all_whole = all_whole && V <= rspan;
    }
    // largest spans first: the graphs of a fused query differ in size many
    // times over, and a large one started last would hold up the whole round
    std::stable_sort(spans.begin(), spans.end(),
                     [](const ReduceSpan& a, const ReduceSpan& b) { return a.n > b.n; });
    const uint32_t rgrid = (uint32_t)spans.size();
    if (rgrid > Q->cap_spans || !Q->spans) {
        if ((st = qalloc(&Q->spans, rgrid))) return st;
        Q->cap_spans = rgrid;
    }
    GZ_HIP(hipMemcpyAsync(Q->spans, spans.data(), sizeof(ReduceSpan) * rgrid,
                          hipMemcpyHostToDevice, qs));
    for (uint32_t r = 0; r < 2 * kMaxRounds; ++r) Q->host_na[r] = kNone;
    // Rounds are enqueued ahead of the device; before round r the host waits
    // for the end of round r-2 and stops once a round had no active component
    // (kernels of rounds after that one return at once).  Lists only shrink,
    // so once round r-2 left a list that fits one workgroup's LDS, the
    // grid-wide doubling is not launched again.
    // The component list alternates between two buffers: round r reads Lc and
    // writes the next round's list to Ln.  After the round that stops the query
    // (no active component, so every component is its own root) both hold the
    // same components, so rounds enqueued past it may swap them freely.
    uint32_t nl_bound = T;
    const bool narrow_ids = T <= 65536;  // node ids and list positions fit 16 bits
    const uint32_t lds_cap = narrow_ids ? kLdsResolveNarrow : kLdsResolve;
    uint32_t* Lc = Q->L;
    uint32_t* Ln = Q->L2;
    // components that hold their whole graph finish unread: known from the
    // list length for one graph, from per-graph counts for many small graphs
    // (larger graphs would cost many same-address atomics per count)
    const uint32_t whole_mode =
        G == 1 ? WHOLE_SINGLE : (Vmax <= kGraphResolve ? WHOLE_COUNT : WHOLE_OFF);
    for (uint32_t r = 0; r < Rmax; ++r) {
        uint32_t* gcomp_prev = Q->gcomp + ((r + 1) & 1) * (uint64_t)G;
        uint32_t* gcomp_next = Q->gcomp + (r & 1) * (uint64_t)G;
        if (r >= 2) {
            GZ_HIP(hipEventSynchronize(Q->round_ev[r & 1]));
            if (Q->host_na[r - 2] == 0) break;
            nl_bound = std::min(nl_bound, Q->host_na[kMaxRounds + r - 2]);
        }
        if (tier_g && r > 0) {
            uint32_t* buf = nullptr;
            GZ_TRY(tier_round(tier_g, r, qs, &buf));  // after round r-1's kernels on qs
        }
        k_q_select<<<ta, kAppendThreads, 0, qs>>>(r, Lc, Q->ctl, Q->done, Q->gof, Q->descs,
                                                  Q->slot, Q->A, Q->hook, Q->newlab, Q->merged,
                                                  Q->pos, whole_mode, G, gcomp_prev, gcomp_next);
        if (r == 0) {
            k_q_query<true><<<qgrid, 256, 0, qs>>>(r, Q->A, Q->ctl, Q->acc, wpr, 0u, Q->gof,
                                                   Q->descs, Q->comp, Q->hook, Q->hedge, Q->done);
        } else {
            // spans that cut a graph XOR into zeroed accumulators: zeroed here for
            // the first reduce, then by each round's query after reading them
            if (!all_whole && r == 1) k_q_zero_acc<<<zgrid, 256, 0, qs>>>(Q->ctl, wpr, Q->acc);
            k_q_reduce<<<dim3(rgrid, ry), 256, 0, qs>>>(r, Q->spans, Q->comp, Q->slot, Q->descs,
                                                        wpr, Q->acc, Q->ctl);
            k_q_query<false><<<qgrid, 256, 0, qs>>>(r, Q->A, Q->ctl, Q->acc, wpr,
                                                    all_whole ? 0u : 1u, Q->gof,
                                                    Q->descs, Q->comp, Q->hook, Q->hedge,
                                                    Q->done);
        }
        // hooks -> roots: per graph in LDS in the first round of many small
        // graphs; in LDS when the list is short (on the device's count); else
        // by grid-wide pointer doubling
        if (r == 0 && G > 1 && Vmax <= kGraphResolve) {
            k_q_resolve_graphs<kGraphResolve, kGraphResolveThreads><<<G, kGraphResolveThreads, 0, qs>>>(
                Q->descs, Q->ctl, Q->hook, Q->hedge, Q->rootOf, Q->newlab, Q->merged, Q->forest);
        } else if (r == 0 && G == 1 && T <= kGraphResolveOne) {
            k_q_resolve_graphs<kGraphResolveOne, 1024><<<1, 1024, 0, qs>>>(
                Q->descs, Q->ctl, Q->hook, Q->hedge, Q->rootOf, Q->newlab, Q->merged, Q->forest);
        } else {
            if (narrow_ids)
                k_q_resolve_lds<true><<<1, 1024, 0, qs>>>(Lc, Q->ctl, K, Q->hook, Q->hedge, Q->pos,
                                                          Q->gof, Q->rootOf, Q->newlab, Q->merged,
                                                          Q->forest);
            else
                k_q_resolve_lds<false><<<1, 1024, 0, qs>>>(Lc, Q->ctl, K, Q->hook, Q->hedge,
                                                           Q->pos, Q->gof, Q->rootOf, Q->newlab,
                                                           Q->merged, Q->forest);
            if (nl_bound > lds_cap) {
                const uint32_t cap = lds_cap;
                k_q_double_init<<<tb, 256, 0, qs>>>(Lc, Q->ctl, Q->hook, s, m, cap);
                if (T <= kSingleBlockDoubling) {
                    k_q_double_all<<<1, 1024, 0, qs>>>(Lc, Q->ctl, K, s, m, s2, m2, cap);
                    if (K & 1) {
                        std::swap(s, s2);
                        std::swap(m, m2);
                    }
                } else {
                    for (uint32_t k = 0; k < K; ++k) {
                        k_q_double<<<tb, 256, 0, qs>>>(Lc, Q->ctl, s, m, s2, m2, cap);
                        std::swap(s, s2);
                        std::swap(m, m2);
                    }
                }
                k_q_root<<<ta, kAppendThreads, 0, qs>>>(Lc, Q->ctl, s, m, Q->hook, Q->hedge, Q->gof,
                                                        Q->rootOf, Q->newlab, Q->merged, Q->forest,
                                                        cap);
            }
        }
        // at most kEndBlocks workgroups: each takes one returning atomic to
        // find the last (4233 of them took 40 us per round on 4.3 M nodes)
        k_q_newcomps<<<std::min(ta, kEndBlocks), kAppendThreads, 0, qs>>>(
            r, T, Q->comp, Lc, Q->ctl, Q->rootOf, Q->newlab, Q->merged, Q->done, Ln, Q->host_na,
            Q->gof, whole_mode == WHOLE_COUNT ? gcomp_next : nullptr);
        std::swap(Lc, Ln);
        GZ_HIP(hipEventRecord(Q->round_ev[r & 1], qs));
    }
    GZ_HIP(hipMemsetAsync(Q->gcount, 0, 4ull * G, qs));
    GZ_HIP(hipMemsetAsync(Q->gfail, 0, 4ull * G, qs));
    k_q_finish<<<tb, 256, 0, qs>>>(Lc, Q->ctl, Q->done, Q->gof, Q->gcount, Q->gfail);
    if (labels_out) {
        k_q_labels<<<tb, 256, 0, qs>>>(T, Q->comp, Q->gof, Q->descs, Q->labels);
        GZ_HIP(hipMemcpyAsync(labels_out, Q->labels, 4ull * T, hipMemcpyDeviceToHost, qs));
    }
    out.num_cc.resize(G);
    std::vector<uint32_t> gfail(G);
    GZ_HIP(hipMemcpyAsync(out.num_cc.data(), Q->gcount, 4ull * G, hipMemcpyDeviceToHost, qs));
    GZ_HIP(hipMemcpyAsync(gfail.data(), Q->gfail, 4ull * G, hipMemcpyDeviceToHost, qs));
    uint32_t tail[Q_ROUNDS + 1] = {};
    GZ_HIP(hipMemcpyAsync(tail, Q->ctl, sizeof(tail), hipMemcpyDeviceToHost, qs));
    if (want_forest) {
        GZ_HIP(hipMemsetAsync(Q->fcnt, 0, 4ull * G, qs));
        k_q_fcount<<<tb, 256, 0, qs>>>(Q->forest, Q->ctl, Q->fcnt);
        k_q_fscan<<<1, 1, 0, qs>>>(Q->fcnt, G, Q->foff, Q->fcur);
        // passes for the largest possible forest; kernels past the device's
        // count return at once
        const uint32_t fgrid = blocks_for(T, 256) < 2048 ? blocks_for(T, 256) : 2048;
        k_q_fsort_tile<<<(T + kFTile - 1) / kFTile, 1024, 0, qs>>>(Q->forest, Q->ctl);
        uint64_t* fin = Q->forest;
        uint64_t* fout = Q->fsorted;
        for (uint64_t w = kFTile; w < T; w <<= 1) {
            k_q_fmerge<<<fgrid, 256, 0, qs>>>(fin, fout, Q->ctl, (uint32_t)w);
            std::swap(fin, fout);
        }
        k_q_fpairs<<<fgrid, 256, 0, qs>>>(fin, Q->ctl, Q->fpairs);
    }
    GZ_HIP(hipGetLastError());
    GZ_HIP(hipStreamSynchronize(qs));
    const uint32_t nF = tail[Q_NF];
    if (want_forest) {
        std::vector<uint32_t> foff(G + 1);
        GZ_HIP(hipMemcpy(foff.data(), Q->foff, 4ull * (G + 1), hipMemcpyDeviceToHost));
        out.forest.resize(2ull * nF);
        if (nF)
            GZ_HIP(hipMemcpy(out.forest.data(), Q->fpairs, 8ull * nF, hipMemcpyDeviceToHost));
        out.forest_off.assign(foff.begin(), foff.end());
    } else {
        out.forest.clear();
        out.forest_off.clear();
    }
    out.status.resize(G);
    for (uint32_t k = 0; k < G; ++k) out.status[k] = gfail[k] ? GZ_ESKETCH_FAIL : GZ_OK;
    out.rounds = tail[Q_ROUNDS];
    return GZ_OK;
}

}  // namespace gz
