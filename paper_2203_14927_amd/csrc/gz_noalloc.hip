// Ingest without device allocation: gz_ingest_noalloc carves every buffer of
// the ingest launch sequence (grouping tables, grouped entries, work items,
// per-call tables) from one fixed array in device memory that the library
// holds on each GPU it runs on, so callers that cannot allocate (code under
// stream capture, tight serving loops) can ingest.
#include <mutex>

#include "gz_internal.h"

namespace gz {

// 64 MiB per device, from the code object's own device memory (held until the
// process ends).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex& noalloc_mutex() {
    static std::mutex* m = new std::mutex();  // never destroyed: no teardown at exit
    return *m;
}
uint8_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// The device address of `scratch` on the current device, found once per device
// with that device current (each GPU holds its own copy at its own address; in
// host code the array's name is only a host-side stand-in).
hipError_t noalloc_scratch(uint8_t** ptr, size_t* cap) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(noalloc_mutex());
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<uint8_t*>(p);
    }
    *ptr = g_scratch_ptr[dev];
    *cap = kNoAllocScratchBytes;
    return hipSuccess;
}

}  // namespace gz

using namespace gz;

extern "C" gz_status gz_ingest_noalloc(gz_graph* g, const uint32_t* src, const uint32_t* dst,
                                       uint64_t N, uint32_t flags, hipStream_t stream) {
    if (!g) return fail(GZ_EINVAL, "null graph");
    uint8_t* p = nullptr;
    size_t cap = 0;
    GZ_HIP(noalloc_scratch(&p, &cap));
    return ingest_noalloc(g, src, dst, N, flags, stream, p, cap);
}
