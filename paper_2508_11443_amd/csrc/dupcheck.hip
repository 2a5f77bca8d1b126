// Whether a build's keys hold two equal entries: the precondition of
// from_array_nodup (Section 3.2).  Equal keys land in the same bucket under
// every level-one attempt and no level-two trial separates them, so a build
// whose every attempt was rejected asks this question once to tell
// FKS_EDUPKEY from FKS_EBUILD.  It never runs on a build that succeeds.
//
// Linear probing over a power-of-two table of at least 2n key indices with
// 32-bit compare-and-swap: a key either claims an empty slot or meets an
// occupied one, whose key it compares with its own (strings: fingerprint,
// length, then bytes), and moves on.  At most n of the slots fill, so every
// probe sequence ends at an empty slot or at an equal key.
#include <hip/hip_runtime.h>

#include "fks_internal.hpp"
#include "prof.hpp"

namespace fks {

constexpr uint32_t kNoKey = 0xFFFFFFFFu;

__global__ void k_eq_clear(uint32_t* __restrict__ table, uint64_t cap, uint32_t* __restrict__ found) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap;
         i += (uint64_t)gridDim.x * blockDim.x)
        table[i] = kNoKey;
    if (blockIdx.x == 0 && threadIdx.x == 0) *found = 0;
}

__device__ __forceinline__ bool equal_strings(const int64_t* off, const uint8_t* bytes, uint32_t a, uint32_t b) {
    const int64_t la = off[a + 1] - off[a], lb = off[b + 1] - off[b];
    if (la != lb) return false;
    const uint8_t* pa = bytes + off[a];
    const uint8_t* pb = bytes + off[b];
    for (int64_t i = 0; i < la; ++i)
        if (pa[i] != pb[i]) return false;
    return true;
}

// keys: the u64 keys, or the strings' fingerprints under one base (equal strings
// have equal fingerprints); off/bytes: the strings (STR only)
template <bool STR>
__global__ __launch_bounds__(256) void k_eq_probe(const uint64_t* __restrict__ keys, uint64_t n,
                                                    const int64_t* __restrict__ off, const uint8_t* __restrict__ bytes,
                                                    uint32_t* __restrict__ table, uint64_t mask,
                                                    uint32_t* __restrict__ found) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = keys[i];
        uint64_t h = sm_fin(x) & mask;
        for (uint64_t probe = 0; probe <= mask; ++probe) {
            const uint32_t old = atomicCAS(&table[h], kNoKey, (uint32_t)i);
            if (old == kNoKey) break;   // claimed
            if (keys[old] == x && (!STR || equal_strings(off, bytes, old, (uint32_t)i))) {
                atomicOr(found, 1u);
                break;
            }
            h = (h + 1) & mask;
        }
    }
}

// *equal = whether keys[0..n) (or the n strings of off/bytes, fingerprinted as keys)
// hold two equal entries.  Synchronises the stream once.
int has_equal_keys(const uint64_t* keys, uint64_t n, const int64_t* off, const uint8_t* bytes, hipStream_t st,
                   bool* equal) {
    *equal = false;
    if (n < 2) return FKS_OK;
    uint64_t cap = 1;
    while (cap < 2 * n) cap <<= 1;
    uint32_t* table = (uint32_t*)dev_alloc(4 * cap + 256, st);
    if (!table) return FKS_ENOMEM;
    uint32_t* found = table + cap;
    auto grid = [](uint64_t items) {
        const uint64_t g = (items + 255) / 256;
        return (unsigned)(g < 1 ? 1 : g > 65536 ? 65536 : g);
    };
    hipLaunchKernelGGL(k_eq_clear, grid(cap), 256, 0, st, table, cap, found);
    if (off)
        FKS_TIMED("fks_equal_keys", st,
                  hipLaunchKernelGGL(k_eq_probe<true>, grid(n), 256, 0, st, keys, n, off, bytes, table, cap - 1,
                                     found));
    else
        FKS_TIMED("fks_equal_keys", st,
                  hipLaunchKernelGGL(k_eq_probe<false>, grid(n), 256, 0, st, keys, n, nullptr, nullptr, table,
                                     cap - 1, found));
    uint32_t h_found = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&h_found, found, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dev_free(table, st);
    if (e != hipSuccess) return hip_fail(e);
    *equal = h_found != 0;
    return FKS_OK;
}

}  // namespace fks
