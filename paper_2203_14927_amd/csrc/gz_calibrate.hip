// Peak figures of the device the roofline of the sketch kernels is read
// against: a plain device copy (HBM read + write bandwidth) and the issue
// rates of the integer VALU instructions the hash and the bucket XOR are made
// of, each measured with HIP events on the caller's stream.
#include <vector>

#include "gz_internal.h"

namespace gz {

namespace {

__global__ void k_copy16(const uint4* __restrict__ a, uint4* __restrict__ b, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        b[i] = a[i];
}

// Eight independent chains per lane, `iters` rounds of one instruction each:
// kind 0 v_mul_lo_u32, 1 v_mad_u64_u32, 2 v_xor_b32 (each chain XORs in its
// neighbour, so that no chain folds away), 3 v_mad_u32_u24, 4 v_add_u32 (the
// same neighbour pattern), 5 v_ffbl_b32 (count of trailing zeros, clamped,
// plus one and XORed back into the chain: four instructions per round).  The result is stored so that
// no chain is dead.
template <int kKind>
__global__ __launch_bounds__(256) void k_alu(uint32_t iters, uint32_t seed, uint32_t* __restrict__ out) {
    uint32_t x[8];
    uint64_t y[8];
    const uint32_t m = seed | 1u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        x[k] = threadIdx.x * 8u + k + seed;
        y[k] = x[k];
    }
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if constexpr (kKind == 0) x[k] = x[k] * m;
            else if constexpr (kKind == 1) y[k] = (uint64_t)(uint32_t)y[k] * m + y[k];
            else if constexpr (kKind == 2) x[k] ^= x[(k + 1) & 7];
            else if constexpr (kKind == 3) x[k] = __umul24(x[k], m) + x[k];
            else if constexpr (kKind == 4) x[k] += x[(k + 1) & 7];
            else x[k] ^= (uint32_t)__builtin_ctzg(x[k], 32) + 1u;
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) r ^= (kKind == 1) ? (uint32_t)(y[k] ^ (y[k] >> 32)) : x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

template <typename F>
gz_status time_ms(hipStream_t s, F launch, float* ms) {
    hipEvent_t a, b;
    GZ_HIP(hipEventCreate(&a));
    GZ_HIP(hipEventCreate(&b));
    launch();  // warm-up
    GZ_HIP(hipEventRecord(a, s));
    launch();
    GZ_HIP(hipEventRecord(b, s));
    GZ_HIP(hipEventSynchronize(b));
    GZ_HIP(hipGetLastError());
    GZ_HIP(hipEventElapsedTime(ms, a, b));
    hipEventDestroy(a);
    hipEventDestroy(b);
    return GZ_OK;
}

}  // namespace
}  // namespace gz

using namespace gz;

extern "C" gz_status gz_measure_peaks(gz_peaks* out, hipStream_t stream) {
    if (!out) return fail(GZ_EINVAL, "null output");
    *out = gz_peaks{};
    const uint64_t bytes = 1ull << 30;
    uint4 *a = nullptr, *b = nullptr;
    GZ_HIP(hipMalloc((void**)&a, bytes));
    if (hipMalloc((void**)&b, bytes) != hipSuccess) {
        hipFree(a);
        return fail(GZ_ENOMEM, "calibration buffers");
    }
    const int cus = device_cu_count();
    gz_status st = GZ_OK;
    float ms = 0;
    if (!st) st = GZ_HIP_STATUS(hipMemsetAsync(a, 1, bytes, stream));
    if (!st)
        st = time_ms(stream, [&] { k_copy16<<<cus * 16, 256, 0, stream>>>(a, b, bytes / 16); }, &ms);
    if (!st) out->copy_gbs = 2.0 * bytes / (ms * 1e-3) / 1e9;
    // ALU kernels: 32 workgroups of 256 lanes per CU, eight chains per lane
    const uint32_t blocks = (uint32_t)cus * 32, iters = 4096;
    const double lane_ops = (double)blocks * 256 * iters * 8;
    uint32_t* o = reinterpret_cast<uint32_t*>(b);
    double* dst[6] = {&out->mul_lo_u32_tops, &out->mad_u64_u32_tops, &out->xor_b32_tops,
                      &out->mad_u32_u24_tops, &out->add_u32_tops, &out->ctz_b32_tops};
    for (int kind = 0; kind < 6 && !st; ++kind) {
        st = time_ms(stream, [&] {
            if (kind == 0) k_alu<0><<<blocks, 256, 0, stream>>>(iters, 0x9E3779B9u, o);
            else if (kind == 1) k_alu<1><<<blocks, 256, 0, stream>>>(iters, 0x9E3779B9u, o);
            else if (kind == 2) k_alu<2><<<blocks, 256, 0, stream>>>(iters, 0x9E3779B9u, o);
            else if (kind == 3) k_alu<3><<<blocks, 256, 0, stream>>>(iters, 0x9E3779B9u, o);
            else if (kind == 4) k_alu<4><<<blocks, 256, 0, stream>>>(iters, 0x9E3779B9u, o);
            else k_alu<5><<<blocks, 256, 0, stream>>>(iters, 0x9E3779B9u, o);
        }, &ms);
        // kind 5 issues four instructions per round (count, clamp, add, XOR)
        if (!st) *dst[kind] = lane_ops * (kind == 5 ? 4 : 1) / (ms * 1e-3) / 1e12;
    }
    hipFree(a);
    hipFree(b);
    out->cus = (uint32_t)cus;
    return st;
}
