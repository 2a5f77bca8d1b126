// Random-access ceiling of the device: how many independent random reads of a
// given width per second the memory system serves from a buffer far larger than
// the caches.  The lookup kernels are bound by this rate (each needle makes one
// or two dependent random reads), not by bytes, so the benchmark measures it
// next to them.
#include <hip/hip_runtime.h>

#include "fks_internal.hpp"

namespace fks {

__device__ __forceinline__ uint64_t probe_mix(uint64_t x) {
    // any fixed odd multiplier and shifts scatter consecutive indices across the buffer
    x *= 0xD6E8FEB86659FD93ull;
    x ^= x >> 32;
    x *= 0xA0761D6478BD642Full;
    x ^= x >> 29;
    return x;
}

template <int VEC>
__global__ __launch_bounds__(256) void k_probe_random(const uint4* __restrict__ buf, uint64_t mask_blocks,
                                                        uint64_t nprobe, uint32_t* __restrict__ sink) {
    uint32_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nprobe;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4* p = buf + (probe_mix(i) & mask_blocks) * VEC;
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            const uint4 v = p[k];
            acc ^= v.x ^ v.w;
        }
    }
    if (acc == 0x9E3779B9u) sink[0] = acc;   // keeps the loads alive
}

}  // namespace fks

using namespace fks;

extern "C" int fks_probe_random_reads(uint64_t buffer_bytes, uint64_t probes, uint32_t width_bytes, void* stream,
                                      double* ms_out) {
    if (!ms_out || probes == 0) return FKS_EINVAL;
    if (width_bytes != 16 && width_bytes != 32 && width_bytes != 64 && width_bytes != 128) return FKS_EINVAL;
    uint64_t blocks = 1;
    while (blocks * 2 * width_bytes <= buffer_bytes) blocks *= 2;   // a power of two of width-sized blocks
    hipStream_t st = (hipStream_t)stream;
    uint4* buf = (uint4*)dev_alloc(blocks * width_bytes, st);
    uint32_t* sink = (uint32_t*)dev_alloc(64, st);
    if (!buf || !sink) {
        dev_free(buf, st);
        dev_free(sink, st);
        return FKS_ENOMEM;
    }
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipMemsetAsync(buf, 1, blocks * width_bytes, st);
    const uint64_t mask = blocks - 1;
    const unsigned grid = 16384;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // the first pass warms the translation caches
        e = hipEventRecord(a, st);
        if (e != hipSuccess) break;
        switch (width_bytes) {
            case 16: hipLaunchKernelGGL(k_probe_random<1>, grid, 256, 0, st, buf, mask, probes, sink); break;
            case 32: hipLaunchKernelGGL(k_probe_random<2>, grid, 256, 0, st, buf, mask, probes, sink); break;
            case 64: hipLaunchKernelGGL(k_probe_random<4>, grid, 256, 0, st, buf, mask, probes, sink); break;
            default: hipLaunchKernelGGL(k_probe_random<8>, grid, 256, 0, st, buf, mask, probes, sink); break;
        }
        e = hipEventRecord(b, st);
    }
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess) *ms_out = ms;
    // released on every path; the frees are ordered after the probe on the stream
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    dev_free(buf, st);
    dev_free(sink, st);
    const hipError_t e2 = hipStreamSynchronize(st);
    if (e == hipSuccess) e = e2;
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}
