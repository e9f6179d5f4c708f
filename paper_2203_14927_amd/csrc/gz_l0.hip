// The standard l0-sampler that CubeSketch replaces (Sec. 3, Fig. "agm_code"),
// on the GPU, for the comparison of update cost the paper makes in Fig.
// "l0speedup".  Node sketches of a graph with V <= 2^16 nodes, one sampler per
// Boruvka round per node, C = 8 columns and B rows as for CubeSketch.
//
// A bucket holds a = sum of index * Delta, b = sum of Delta and a checksum
// c = sum of Delta * z^index modulo p = 2^61 - 1.  Node vectors are signed:
// edge {u, v}, u < v, at index v(v-1)/2 + u carries +Delta in u's vector and
// -Delta in v's (insert: Delta = +1, delete: -1), so the edges inside a node
// set cancel when its sketches are added.  Row membership uses the CubeSketch
// row hash of the same round and column; z of a round and column is
// 1 + (m mod (p - 1)) for its checksum-high multiplier m of the seed stream.
//
// Storage (device, private): per node, round-major, rows of a round
// contiguous, columns side by side, four 64-bit words per bucket in the
// exact-depth basis (row d holds the indices whose depth is exactly d; the
// figure's nested row b is the sum of rows d >= b): a and b as two's
// complement sums, and the checksum as two sums of the low 32 and the high 29
// bits of its terms Delta * z^index mod p (each term taken in [0, p)), so that
// every merge is a plain 64-bit add; c = (hi sum * 2^32 + lo sum) mod p.  The
// sums are exact while a node's buckets take fewer than 2^32 terms.
#include <cstring>
#include <vector>

#include "gz_device.h"
#include "gz_internal.h"

namespace gz {

constexpr uint64_t kP61 = 0x1FFFFFFFFFFFFFFFull;  // 2^61 - 1
constexpr uint32_t kL0Words = 4;                  // a, b, checksum low sum, checksum high sum
constexpr uint32_t kL0Bits = 31;                  // indices are < 2^31
constexpr uint32_t kL0Rows = 8;                   // exact-depth rows kept in LDS per item
constexpr uint32_t kL0Chunk = 4096;               // entries per work item
constexpr uint32_t kL0Groups = 4;                 // groups of lanes per workgroup

struct L0Item {
    uint32_t node, begin, count, pad;
};

namespace {

// x * y mod p for x, y < p: the 122-bit product is hi * 2^64 + lo, and with
// p = 2^61 - 1, x * y = (x * y >> 61) * 2^61 + (x * y mod 2^61) = the two parts
// summed modulo p.
__device__ __forceinline__ uint64_t mulmod61(uint64_t x, uint64_t y) {
    const uint64_t lo = x * y;
    const uint64_t hi = __umul64hi(x, y);
    uint64_t r = (lo & kP61) + ((lo >> 61) | (hi << 3));
    r = r >= kP61 ? r - kP61 : r;
    return r >= kP61 ? r - kP61 : r;
}

__device__ __forceinline__ uint64_t addmod61(uint64_t x, uint64_t y) {
    const uint64_t r = x + y;
    return r >= kP61 ? r - kP61 : r;
}

// z^e mod p from the table z^(2^k), k < 31, of the lane's pair (`stride`
// words between powers): one multiply per set bit of e
__device__ __forceinline__ uint64_t pow_from_table(const uint64_t* tab, uint32_t stride,
                                                   uint32_t e) {
    uint64_t acc = 1;
    while (e) {
        const uint32_t k = __builtin_ctz(e);
        acc = mulmod61(acc, tab[k * stride]);
        e &= e - 1u;
    }
    return acc;
}

__device__ __forceinline__ uint32_t l0_word(uint32_t B, uint32_t r, uint32_t d, uint32_t c,
                                            uint32_t k) {
    return ((r * B + d) * kC + c) * kL0Words + k;
}

// ---------------------------------------------------------------- grouping --

__global__ void k_l0_count(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                           uint64_t N, uint32_t V, uint32_t* __restrict__ cnt,
                           uint32_t* __restrict__ err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const uint32_t u = src[i], v = dst[i];
        if (u == v || u >= V || v >= V) {
            bad = true;
            continue;
        }
        atomicAdd(&cnt[u], 1u);
        atomicAdd(&cnt[v], 1u);
    }
    if (bad) atomicOr(err, 1u);
}

// one workgroup: node offsets and work items (exclusive scans over V nodes)
constexpr uint32_t kL0ScanThreads = 1024;
__global__ __launch_bounds__(kL0ScanThreads) void k_l0_scan(
    const uint32_t* __restrict__ cnt, uint32_t V, uint32_t* __restrict__ off,
    uint32_t* __restrict__ cursor, L0Item* __restrict__ items, uint32_t* __restrict__ ctl) {
    __shared__ uint32_t s_e[kL0ScanThreads], s_i[kL0ScanThreads];
    if (ctl[2]) return;
    const uint32_t per = (V + kL0ScanThreads - 1) / kL0ScanThreads;
    const uint32_t v0 = threadIdx.x * per, v1 = min(V, v0 + per);
    uint32_t e = 0, it = 0;
    for (uint32_t v = v0; v < v1; ++v) {
        e += cnt[v];
        it += (cnt[v] + kL0Chunk - 1) / kL0Chunk;
    }
    s_e[threadIdx.x] = e;
    s_i[threadIdx.x] = it;
    __syncthreads();
    // Hillis-Steele inclusive scan of both sums
    for (uint32_t o = 1; o < kL0ScanThreads; o <<= 1) {
        const uint32_t ae = threadIdx.x >= o ? s_e[threadIdx.x - o] : 0u;
        const uint32_t ai = threadIdx.x >= o ? s_i[threadIdx.x - o] : 0u;
        __syncthreads();
        s_e[threadIdx.x] += ae;
        s_i[threadIdx.x] += ai;
        __syncthreads();
    }
    uint32_t pe = s_e[threadIdx.x] - e, pi = s_i[threadIdx.x] - it;
    for (uint32_t v = v0; v < v1; ++v) {
        const uint32_t c = cnt[v];
        off[v] = pe;
        cursor[v] = pe;
        for (uint32_t b = 0; b < c; b += kL0Chunk)
            items[pi++] = L0Item{v, pe + b, min(kL0Chunk, c - b), 0u};
        pe += c;
    }
    if (threadIdx.x == kL0ScanThreads - 1) {
        ctl[0] = 0;                // ticket
        ctl[1] = s_i[threadIdx.x];  // items
    }
}

// entry = neighbour id | (1 << 31) for a deletion
__global__ void k_l0_scatter(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                             const uint8_t* __restrict__ op, uint64_t N,
                             uint32_t* __restrict__ cursor, uint32_t* __restrict__ grouped,
                             const uint32_t* __restrict__ ctl) {
    if (ctl[2]) return;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const uint32_t u = src[i], v = dst[i];
        const uint32_t del = (op && op[i] == 0) ? 0x80000000u : 0u;
        grouped[atomicAdd(&cursor[u], 1u)] = v | del;
        grouped[atomicAdd(&cursor[v], 1u)] = u | del;
    }
}

// -------------------------------------------------------------- the update --

struct L0Desc {
    uint64_t* sk;                // node blocks
    const uint32_t* seeds;       // CubeSketch layout: row-hash words at S_ROW_* * P + p
    const uint64_t* pow;         // z^(2^k) of pair p at [k * P + p]
    uint32_t V, R, B, P;
};

// Persistent over work items (a node's entries, up to kL0Chunk of them).  The
// workgroup holds kL0Groups groups of GW lanes (GW = P rounded up to 64, so
// every wave lies in one group and its lanes process the same entry); lane p
// of a group owns pair p.  Rows d < kL0Rows of the item go to an LDS tile by
// 64-bit LDS atomics (groups share it); deeper rows go to HBM atomics; the
// tile is then added into the node's HBM block (every merge is an add).
__global__ __launch_bounds__(1024) void k_l0_update(const L0Item* __restrict__ items,
                                                    uint32_t* __restrict__ ctl,
                                                    const uint32_t* __restrict__ grouped,
                                                    L0Desc g, uint32_t GW) {
    extern __shared__ uint64_t smem[];
    __shared__ uint32_t s_ticket;
    if (ctl[2]) return;
    const uint32_t P = g.P, B = g.B;
    const uint32_t DL = min(B, kL0Rows);
    uint64_t* pow_tab = smem;                     // kL0Bits * P
    uint64_t* tile = smem + kL0Bits * P;          // DL * P * 4
    for (uint32_t i = threadIdx.x; i < kL0Bits * P; i += blockDim.x) pow_tab[i] = g.pow[i];
    const uint32_t j = threadIdx.x / GW, p = threadIdx.x - j * GW;
    const uint32_t J = blockDim.x / GW;
    const bool active = p < P;
    uint32_t mlo = 0, mhi = 0;
    uint64_t inc = 0;
    if (active) {
        mlo = g.seeds[S_ROW_MLO * P + p];
        mhi = g.seeds[S_ROW_MHI * P + p];
        inc = (uint64_t)g.seeds[S_ROW_ILO * P + p] | ((uint64_t)g.seeds[S_ROW_IHI * P + p] << 32);
    }
    const uint32_t r = p / kC, c = p - (p / kC) * kC;
    const uint32_t n_items = ctl[1];
    const uint32_t tile_words = DL * P * kL0Words;
    for (;;) {
        if (threadIdx.x == 0) s_ticket = atomicAdd(&ctl[0], 1u);
        __syncthreads();
        const uint32_t t = s_ticket;
        if (t >= n_items) break;
        const L0Item w = items[t];
        for (uint32_t i = threadIdx.x; i < tile_words; i += blockDim.x) tile[i] = 0;
        __syncthreads();
        uint64_t* skn = g.sk + (uint64_t)w.node * P * B * kL0Words;
        if (active) {
            for (uint32_t e = j; e < w.count; e += J) {
                const uint32_t x = grouped[w.begin + e];
                const uint32_t nbr = x & 0x7FFFFFFFu;
                const uint32_t idx = edge_index(w.node, nbr);
                // +Delta at the smaller endpoint, -Delta at the larger
                const bool neg = (nbr < w.node) != ((x >> 31) != 0);
                const uint32_t h = mas_hash(mlo, mhi, inc, idx);
                const uint32_t d = min((uint32_t)__builtin_ctzg(h, 32), B - 1u);
                const uint64_t chk = pow_from_table(pow_tab + p, P, idx);
                const uint64_t term = neg ? (chk ? kP61 - chk : 0ull) : chk;
                const uint64_t da = neg ? (uint64_t)(-(int64_t)idx) : (uint64_t)idx;
                const uint64_t db = neg ? ~0ull : 1ull;
                unsigned long long* dst;
                if (d < DL) dst = (unsigned long long*)(tile + (d * P + p) * kL0Words);
                else dst = (unsigned long long*)(skn + l0_word(B, r, d, c, 0));
                atomicAdd(dst, (unsigned long long)da);
                atomicAdd(dst + 1, (unsigned long long)db);
                atomicAdd(dst + 2, (unsigned long long)(term & 0xFFFFFFFFull));
                atomicAdd(dst + 3, (unsigned long long)(term >> 32));
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < tile_words; i += blockDim.x) {
            const uint64_t val = tile[i];
            if (!val) continue;
            const uint32_t k = i % kL0Words, q = i / kL0Words;
            const uint32_t d = q / P, pp = q - d * P;
            atomicAdd((unsigned long long*)(skn + l0_word(B, pp / kC, d, pp % kC, k)),
                      (unsigned long long)val);
        }
        __syncthreads();
    }
}

// nested (canonical) buckets of nodes [lo, hi): row b = sum of exact rows d >= b
__global__ void k_l0_export(const uint64_t* __restrict__ sk, uint32_t lo, uint32_t hi, uint32_t R,
                            uint32_t B, int64_t* __restrict__ a, int64_t* __restrict__ b,
                            uint64_t* __restrict__ c) {
    const uint32_t P = R * kC;
    const uint64_t total = (uint64_t)(hi - lo) * P;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = lo + (uint32_t)(t / P), p = (uint32_t)(t % P);
        const uint32_t r = p / kC, col = p % kC;
        const uint64_t* node = sk + (uint64_t)v * P * B * kL0Words;
        const uint64_t out0 = (t / P) * (uint64_t)P * B + (uint64_t)p * B;
        uint64_t sa = 0, sb = 0, slo = 0, shi = 0;
        for (int row = (int)B - 1; row >= 0; --row) {
            const uint64_t* q = node + l0_word(B, r, (uint32_t)row, col, 0);
            sa += q[0];
            sb += q[1];
            slo += q[2];
            shi += q[3];
            a[out0 + row] = (int64_t)sa;
            b[out0 + row] = (int64_t)sb;
            // (shi * 2^32 + slo) mod p
            c[out0 + row] = addmod61(mulmod61(shi % kP61, 1ull << 32), slo % kP61);
        }
    }
}

// Fig. "agm_code" query of every node's round-r sampler: 8 lanes per node, one
// per column; the first passing bucket in column order, rows ascending.
// kind: 0 zero vector, 1 sample, 2 failure.
__global__ void k_l0_sample(const uint64_t* __restrict__ sk, L0Desc g, uint64_t n, uint32_t r,
                            int32_t* __restrict__ kind, uint64_t* __restrict__ idx_out,
                            int64_t* __restrict__ mult_out) {
    const uint32_t gt = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t v = gt >> 3, col = gt & 7u;
    const bool valid = v < g.V;
    const uint32_t P = g.P, B = g.B;
    uint32_t key = kNone, nonzero = 0;
    uint64_t best_i = 0;
    int64_t best_m = 0;
    if (valid) {
        const uint64_t* node = sk + (uint64_t)v * P * B * kL0Words;
        const uint32_t p = r * kC + col;
        uint64_t sa = 0, sb = 0, slo = 0, shi = 0;
        for (int row = (int)B - 1; row >= 0; --row) {
            const uint64_t* q = node + l0_word(B, r, (uint32_t)row, col, 0);
            sa += q[0];
            sb += q[1];
            slo += q[2];
            shi += q[3];
            const uint64_t cm = addmod61(mulmod61(shi % kP61, 1ull << 32), slo % kP61);
            const int64_t A = (int64_t)sa, Bv = (int64_t)sb;
            if (A == 0 && Bv == 0 && cm == 0) continue;
            nonzero = 1;
            if (Bv == 0 || A % Bv != 0) continue;
            const int64_t q2 = A / Bv;
            if (q2 < 0 || (uint64_t)q2 >= n) continue;
            const uint64_t bm = Bv > 0 ? (uint64_t)Bv % kP61
                                       : (kP61 - (uint64_t)(-Bv) % kP61) % kP61;
            if (cm == mulmod61(bm, pow_from_table(g.pow + p, P, (uint32_t)q2))) {
                key = col * B + (uint32_t)row;  // rows descend: the last pass is the smallest row
                best_i = (uint64_t)q2;
                best_m = Bv;
            }
        }
    }
    for (uint32_t off = 1; off < 8; off <<= 1) {
        const uint32_t k2 = __shfl_xor(key, off, 8);
        const uint64_t i2 = __shfl_xor(best_i, off, 8);
        const int64_t m2 = __shfl_xor(best_m, off, 8);
        nonzero |= __shfl_xor(nonzero, off, 8);
        if (k2 < key) {
            key = k2;
            best_i = i2;
            best_m = m2;
        }
    }
    if (!valid || col != 0) return;
    kind[v] = key != kNone ? 1 : (nonzero ? 2 : 0);
    idx_out[v] = key != kNone ? best_i : 0;
    mult_out[v] = key != kNone ? best_m : 0;
}

uint64_t host_mulmod61(uint64_t x, uint64_t y) {
    return (uint64_t)(((unsigned __int128)x * y) % kP61);
}

}  // namespace
}  // namespace gz

using namespace gz;

struct gz_l0 {
    int device = 0;
    uint32_t V = 0, R = 0, B = 0, P = 0;
    uint64_t n = 0;
    uint64_t* sk = nullptr;
    uint64_t sk_words = 0;
    uint32_t* seeds = nullptr;
    uint64_t* pow = nullptr;
    // grouping scratch (grown on demand)
    uint32_t *cnt = nullptr, *off = nullptr, *cursor = nullptr, *ctl = nullptr;
    uint32_t* grouped = nullptr;
    uint64_t cap_entries = 0;
    L0Item* items = nullptr;
    uint64_t cap_items = 0;
    uint32_t* staging = nullptr;  // host inputs: src, dst, op bytes
    uint64_t cap_staging = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    float last_update_ms = 0;
    bool timed = false;
};

namespace {
template <typename T>
gz_status grow_buf(T** p, uint64_t need, uint64_t* cap, const char* what) {
    if (*p && need <= *cap) return GZ_OK;
    if (*p) {
        GZ_HIP(hipDeviceSynchronize());
        GZ_HIP(hipFree(*p));
        *p = nullptr;
    }
    if (hipMalloc((void**)p, std::max<uint64_t>(need, 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        *cap = 0;
        return fail(GZ_ENOMEM, std::string("out of device memory for ") + what);
    }
    *cap = need;
    return GZ_OK;
}
}  // namespace

extern "C" {

gz_status gz_l0_init(gz_l0** out, uint32_t V, uint64_t seed) {
    if (!out) return fail(GZ_EINVAL, "null output handle");
    *out = nullptr;
    if (V < 2 || V > kMaxNarrow) return fail(GZ_EINVAL, "V must be in [2, 65536]");
    gz_l0* s = new gz_l0();
    GZ_HIP(hipGetDevice(&s->device));
    s->V = V;
    s->n = (uint64_t)V * (V - 1) / 2;
    uint32_t bits = 0;
    for (uint64_t x = V - 1; x; x >>= 1) ++bits;
    s->R = bits + 1;
    bits = 0;
    for (uint64_t x = s->n - 1; x; x >>= 1) ++bits;
    s->B = bits + 1;
    s->P = s->R * kC;
    // the CubeSketch seed stream: (multiplier, increment) of the row hash, the
    // checksum-high and the checksum-low hash per (round, column)
    std::vector<uint32_t> soa((size_t)kSeedWords * s->P);
    std::vector<uint64_t> pw((size_t)kL0Bits * s->P);
    uint64_t st = seed;
    for (uint32_t p = 0; p < s->P; ++p) {
        uint64_t w[6];
        for (int k = 0; k < 6; ++k) w[k] = splitmix64_next(st);
        for (int k = 0; k < 6; ++k) {
            soa[(size_t)(2 * k) * s->P + p] = (uint32_t)w[k];
            soa[(size_t)(2 * k + 1) * s->P + p] = (uint32_t)(w[k] >> 32);
        }
        uint64_t z = 1 + w[2] % (kP61 - 1);
        for (uint32_t k = 0; k < kL0Bits; ++k) {
            pw[(size_t)k * s->P + p] = z;
            z = host_mulmod61(z, z);
        }
    }
    s->sk_words = (uint64_t)V * s->P * s->B * kL0Words;
    hipError_t e = hipMalloc((void**)&s->sk, s->sk_words * 8);
    if (e == hipSuccess) e = hipMalloc((void**)&s->seeds, soa.size() * 4);
    if (e == hipSuccess) e = hipMalloc((void**)&s->pow, pw.size() * 8);
    if (e == hipSuccess) e = hipMalloc((void**)&s->cnt, (size_t)V * 4);
    if (e == hipSuccess) e = hipMalloc((void**)&s->off, (size_t)V * 4);
    if (e == hipSuccess) e = hipMalloc((void**)&s->cursor, (size_t)V * 4);
    if (e == hipSuccess) e = hipMalloc((void**)&s->ctl, 8 * 4);
    if (e == hipSuccess) e = hipMemcpy(s->seeds, soa.data(), soa.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->pow, pw.data(), pw.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(s->sk, 0, s->sk_words * 8);
    if (e == hipSuccess) e = hipMemset(s->ctl, 0, 8 * 4);
    if (e == hipSuccess) e = hipEventCreate(&s->ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&s->ev[1]);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        gz_status st2 = hip_fail(e, "l0 sketch init");
        gz_l0_free(s);
        return st2;
    }
    *out = s;
    return GZ_OK;
}

gz_status gz_l0_free(gz_l0* s) {
    if (!s) return GZ_OK;
    hipDeviceSynchronize();
    hipFree(s->sk); hipFree(s->seeds); hipFree(s->pow); hipFree(s->cnt); hipFree(s->off);
    hipFree(s->cursor); hipFree(s->ctl); hipFree(s->grouped); hipFree(s->items);
    hipFree(s->staging);
    for (hipEvent_t e : s->ev)
        if (e) hipEventDestroy(e);
    delete s;
    return GZ_OK;
}

gz_status gz_l0_reset(gz_l0* s, hipStream_t stream) {
    if (!s) return fail(GZ_EINVAL, "null sketch");
    GZ_HIP(hipMemsetAsync(s->sk, 0, s->sk_words * 8, stream));
    return GZ_OK;
}

gz_status gz_l0_ingest(gz_l0* s, const uint32_t* src, const uint32_t* dst, const uint8_t* op,
                       uint64_t N, uint32_t flags, hipStream_t stream) {
    if (!s) return fail(GZ_EINVAL, "null sketch");
    if (N == 0) return GZ_OK;
    if (!src || !dst) return fail(GZ_EINVAL, "null stream arrays");
    if (N >= (1ull << 31)) return fail(GZ_EINVAL, "at most 2^31-1 updates per call");
    const bool host = !(flags & GZ_DEVICE_PTR);
    if (host) {
        const uint64_t words = 2 * N + (op ? (N + 3) / 4 : 0);
        GZ_TRY(grow_buf(&s->staging, words, &s->cap_staging, "input staging"));
        GZ_HIP(hipMemcpyAsync(s->staging, src, N * 4, hipMemcpyHostToDevice, stream));
        GZ_HIP(hipMemcpyAsync(s->staging + N, dst, N * 4, hipMemcpyHostToDevice, stream));
        if (op)
            GZ_HIP(hipMemcpyAsync(s->staging + 2 * N, op, N, hipMemcpyHostToDevice, stream));
        src = s->staging;
        dst = s->staging + N;
        if (op) op = reinterpret_cast<const uint8_t*>(s->staging + 2 * N);
    }
    GZ_TRY(grow_buf(&s->grouped, 2 * N, &s->cap_entries, "grouped entries"));
    GZ_TRY(grow_buf(&s->items, (uint64_t)s->V + 2 * N / kL0Chunk + 1, &s->cap_items, "work items"));
    const int cus = device_cu_count();
    GZ_HIP(hipMemsetAsync(s->cnt, 0, (size_t)s->V * 4, stream));
    GZ_HIP(hipMemsetAsync(s->ctl, 0, 8 * 4, stream));
    const uint32_t gblocks = (uint32_t)std::min<uint64_t>((N + 255) / 256, (uint64_t)cus * 8);
    k_l0_count<<<gblocks, 256, 0, stream>>>(src, dst, N, s->V, s->cnt, s->ctl + 2);
    k_l0_scan<<<1, kL0ScanThreads, 0, stream>>>(s->cnt, s->V, s->off, s->cursor, s->items, s->ctl);
    k_l0_scatter<<<gblocks, 256, 0, stream>>>(src, dst, op, N, s->cursor, s->grouped, s->ctl);
    L0Desc d{s->sk, s->seeds, s->pow, s->V, s->R, s->B, s->P};
    const uint32_t GW = (s->P + 63) & ~63u;
    const uint32_t DL = std::min(s->B, kL0Rows);
    const size_t smem = ((size_t)kL0Bits * s->P + (size_t)DL * s->P * kL0Words) * 8;
    GZ_TRY(set_smem_limit((const void*)k_l0_update, smem));
    const uint32_t wgs_cu = std::max<uint32_t>(1, (uint32_t)((160 * 1024) / smem));
    GZ_HIP(hipEventRecord(s->ev[0], stream));
    k_l0_update<<<cus * wgs_cu, GW * kL0Groups, smem, stream>>>(s->items, s->ctl, s->grouped, d,
                                                                 GW);
    GZ_HIP(hipEventRecord(s->ev[1], stream));
    GZ_HIP(hipGetLastError());
    s->timed = true;
    uint32_t err = 0;
    GZ_HIP(hipMemcpyAsync(&err, s->ctl + 2, 4, hipMemcpyDeviceToHost, stream));
    GZ_HIP(hipStreamSynchronize(stream));
    if (err) return fail(GZ_EINVAL, "invalid update (self-loop or node id out of range)");
    GZ_HIP(hipEventElapsedTime(&s->last_update_ms, s->ev[0], s->ev[1]));
    return GZ_OK;
}

gz_status gz_l0_last_update_ms(gz_l0* s, float* ms) {
    if (!s || !ms) return fail(GZ_EINVAL, "null argument");
    if (!s->timed) return fail(GZ_ESTATE, "no ingest yet");
    *ms = s->last_update_ms;
    return GZ_OK;
}

gz_status gz_l0_shape(const gz_l0* s, uint32_t* V, uint32_t* R, uint32_t* C, uint32_t* B,
                      uint64_t* n) {
    if (!s) return fail(GZ_EINVAL, "null sketch");
    if (V) *V = s->V;
    if (R) *R = s->R;
    if (C) *C = kC;
    if (B) *B = s->B;
    if (n) *n = s->n;
    return GZ_OK;
}

gz_status gz_l0_export(gz_l0* s, uint32_t lo, uint32_t hi, int64_t* a, int64_t* b, uint64_t* c) {
    if (!s || !a || !b || !c) return fail(GZ_EINVAL, "null argument");
    if (lo > hi || hi > s->V) return fail(GZ_EINVAL, "bad node range");
    const uint64_t cells = (uint64_t)(hi - lo) * s->P * s->B;
    if (!cells) return GZ_OK;
    GZ_HIP(hipDeviceSynchronize());
    void* buf = nullptr;
    GZ_HIP(hipMalloc(&buf, cells * 24));
    int64_t* da = (int64_t*)buf;
    int64_t* db = da + cells;
    uint64_t* dc = (uint64_t*)(db + cells);
    const uint64_t total = (uint64_t)(hi - lo) * s->P;
    k_l0_export<<<(uint32_t)std::min<uint64_t>((total + 255) / 256, 65535), 256>>>(
        s->sk, lo, hi, s->R, s->B, da, db, dc);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(a, da, cells * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(b, db, cells * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(c, dc, cells * 8, hipMemcpyDeviceToHost);
    hipFree(buf);
    if (e != hipSuccess) return hip_fail(e, "l0 export");
    return GZ_OK;
}

gz_status gz_l0_sample(gz_l0* s, uint32_t round, int32_t* kind, uint64_t* idx, int64_t* mult) {
    if (!s || !kind || !idx || !mult) return fail(GZ_EINVAL, "null argument");
    if (round >= s->R) return fail(GZ_EINVAL, "round out of range");
    GZ_HIP(hipDeviceSynchronize());
    void* buf = nullptr;
    GZ_HIP(hipMalloc(&buf, (size_t)s->V * 20));
    uint64_t* di = (uint64_t*)buf;
    int64_t* dm = (int64_t*)(di + s->V);
    int32_t* dk = (int32_t*)(dm + s->V);
    L0Desc d{s->sk, s->seeds, s->pow, s->V, s->R, s->B, s->P};
    k_l0_sample<<<(s->V * 8 + 255) / 256, 256>>>(s->sk, d, s->n, round, dk, di, dm);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(kind, dk, (size_t)s->V * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(idx, di, (size_t)s->V * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(mult, dm, (size_t)s->V * 8, hipMemcpyDeviceToHost);
    hipFree(buf);
    if (e != hipSuccess) return hip_fail(e, "l0 sample");
    return GZ_OK;
}

}  // extern "C"
