// Device-side arithmetic of the hash contract (see include/gz.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gz_internal.h"

namespace gz {

// multiply-add-shift: ((m * x + i) mod 2^64) >> 32 for a 32-bit key x, with the
// 64-bit multiplier split into words.  (m*x) mod 2^64 = mlo*x + (mhi*x mod 2^32)*2^32,
// so the high word is hi32(mlo*x + i) + mhi*x (mod 2^32): two v_mad_u64_u32.
__device__ __forceinline__ uint32_t mas_hash(uint32_t mlo, uint32_t mhi, uint64_t incr,
                                             uint32_t x) {
    uint64_t t = (uint64_t)mlo * x + incr;
    return (uint32_t)(t >> 32) + mhi * x;
}

// Seeds of one (round, column) pair held in registers.
struct PairSeeds {
    uint32_t row_mlo, row_mhi, chi_mlo, chi_mhi, clo_mlo, clo_mhi;
    uint64_t row_inc, chi_inc, clo_inc;
};

__device__ __forceinline__ PairSeeds load_pair_seeds(const uint32_t* __restrict__ seeds,
                                                     uint32_t P, uint32_t p) {
    PairSeeds s;
    s.row_mlo = seeds[S_ROW_MLO * P + p];
    s.row_mhi = seeds[S_ROW_MHI * P + p];
    s.row_inc = (uint64_t)seeds[S_ROW_ILO * P + p] | ((uint64_t)seeds[S_ROW_IHI * P + p] << 32);
    s.chi_mlo = seeds[S_CHI_MLO * P + p];
    s.chi_mhi = seeds[S_CHI_MHI * P + p];
    s.chi_inc = (uint64_t)seeds[S_CHI_ILO * P + p] | ((uint64_t)seeds[S_CHI_IHI * P + p] << 32);
    s.clo_mlo = seeds[S_CLO_MLO * P + p];
    s.clo_mhi = seeds[S_CLO_MHI * P + p];
    s.clo_inc = (uint64_t)seeds[S_CLO_ILO * P + p] | ((uint64_t)seeds[S_CLO_IHI * P + p] << 32);
    return s;
}

// depth = min(count of trailing zeros of the row hash, B-1); a zero hash counts 32
__device__ __forceinline__ uint32_t row_depth(const PairSeeds& s, uint32_t x, uint32_t Bm1) {
    uint32_t h = mas_hash(s.row_mlo, s.row_mhi, s.row_inc, x);
    uint32_t tz = __builtin_ctzg(h, 32);
    return tz < Bm1 ? tz : Bm1;
}

__device__ __forceinline__ uint32_t chk_hi(const PairSeeds& s, uint32_t x) {
    return mas_hash(s.chi_mlo, s.chi_mhi, s.chi_inc, x);
}

__device__ __forceinline__ uint32_t chk_lo(const PairSeeds& s, uint32_t x) {
    return mas_hash(s.clo_mlo, s.clo_mhi, s.clo_inc, x);
}

// Wide graphs (V > 2^16) hash the node pair (u < v) with the vector form of
// the family: h(u, v) = ((a*u + a2*v + b) mod 2^64) >> 32.  Per hash the seeds
// a, a2, b are 64-bit; on the device, word w = (k*3 + j)*2 + half of pair p
// (k: row low word / checksum-high / checksum-low / row high word, j: a / a2 / b)
// sits at seeds[w*P + p].  The row hash is 64 bits, high word * 2^32 + low
// word; the high word only matters when the low word is zero (depth >= 32).
// (a*u + a2*v + b) mod 2^64 has high word hi32(alo*u + a2lo*v + b) + ahi*u + a2hi*v
// (mod 2^32): two 64-bit multiply-adds in a chain plus two low multiplies.
struct WideHashSeeds {
    uint32_t alo, ahi, a2lo, a2hi;
    uint64_t b;
};
struct WideSeeds {
    WideHashSeeds h[3];  // row, checksum high word, checksum low word
};

__device__ __forceinline__ WideSeeds load_wide_seeds(const uint32_t* __restrict__ seeds,
                                                     uint32_t P, uint32_t p) {
    WideSeeds s;
#pragma unroll
    for (uint32_t k = 0; k < 3; ++k) {
        const uint32_t w = k * 6;
        s.h[k].alo = seeds[(w + 0) * P + p];
        s.h[k].ahi = seeds[(w + 1) * P + p];
        s.h[k].a2lo = seeds[(w + 2) * P + p];
        s.h[k].a2hi = seeds[(w + 3) * P + p];
        s.h[k].b = (uint64_t)seeds[(w + 4) * P + p] | ((uint64_t)seeds[(w + 5) * P + p] << 32);
    }
    return s;
}

__device__ __forceinline__ uint32_t pair_hash(const WideHashSeeds& s, uint32_t u, uint32_t v) {
    uint64_t t = (uint64_t)s.alo * u + s.b;
    t = (uint64_t)s.a2lo * v + t;
    return (uint32_t)(t >> 32) + s.ahi * u + s.a2hi * v;
}

// the high word of a wide graph's row hash (hash 3 of pair p), read from the seed
// table.  It is needed for about one entry in 2^32, from inside the update loop:
// the word offset passes through an empty asm before each load, so that neither
// the six addresses nor the loads are hoisted out of that loop (they would hold
// a dozen registers for the whole kernel).  (alo*u + a2lo*v + b) is summed in
// another order than pair_hash's, with the same result mod 2^64.
__device__ __forceinline__ uint32_t wide_row_hash_high(const uint32_t* __restrict__ seeds,
                                                       uint32_t P, uint32_t p, uint32_t u,
                                                       uint32_t v) {
    uint32_t off = (kWideHashes - 1) * 6 * P + p;
    uint32_t w[6];
#pragma unroll
    for (uint32_t k = 0; k < 6; ++k) {
        asm volatile("" : "+v"(off));
        w[k] = seeds[off];
        off += P;
    }
    uint64_t t = (uint64_t)w[0] * u;
    t = (uint64_t)w[2] * v + t;
    t += (uint64_t)w[4] | ((uint64_t)w[5] << 32);
    return (uint32_t)(t >> 32) + w[1] * u + w[3] * v;
}

// 64-bit position of pair {u, v} (ids up to 2^24)
__device__ __forceinline__ uint64_t edge_index64(uint32_t u, uint32_t v) {
    const uint32_t lo = u < v ? u : v;
    const uint32_t hi = u < v ? v : u;
    return (((uint64_t)hi * (hi - 1u)) >> 1) + lo;
}

// inverse of edge_index64: hi = largest v with v(v-1)/2 <= i (i < 2^47)
__device__ __forceinline__ void edge_pair64(uint64_t i, uint32_t* u, uint32_t* v) {
    uint64_t hi = (uint64_t)((1.0 + sqrt(1.0 + 8.0 * (double)i)) * 0.5);
    while (hi * (hi - 1) / 2 > i) --hi;
    while ((hi + 1) * hi / 2 <= i) ++hi;
    *v = (uint32_t)hi;
    *u = (uint32_t)(i - hi * (hi - 1) / 2);
}

// position of pair {u, v} in the characteristic vector; ids < 2^16 keep it in 32 bits
__device__ __forceinline__ uint32_t edge_index(uint32_t u, uint32_t v) {
    uint32_t lo = u < v ? u : v;
    uint32_t hi = u < v ? v : u;
    return ((hi * (hi - 1u)) >> 1) + lo;
}

// inverse of edge_index: hi = largest v with v(v-1)/2 <= i
__device__ __forceinline__ void edge_pair(uint32_t i, uint32_t* u, uint32_t* v) {
    double di = (double)i;
    uint32_t hi = (uint32_t)((1.0 + sqrt(1.0 + 8.0 * di)) * 0.5);
    // correct a possible rounding step in either direction
    while ((uint64_t)hi * (hi - 1) / 2 > i) --hi;
    while ((uint64_t)(hi + 1) * hi / 2 <= i) ++hi;
    *v = hi;
    *u = i - (uint32_t)((uint64_t)hi * (hi - 1) / 2);
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) {
    return __builtin_amdgcn_readfirstlane(x);
}

}  // namespace gz
