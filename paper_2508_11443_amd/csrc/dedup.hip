// from_array (Figure 2): the constructor that accepts repeated keys.
//
// The input's distinct keys are collected in a linear-probing table with
// 64-bit compare-and-swap (load factor at most 1/2); every occurrence also
// lowers the slot's smallest input index with an atomic minimum, so a
// repeated key keeps the value of its first occurrence whatever the order in
// which the threads arrive.  The occupied slots are compacted and handed to
// from_array_nodup, whose table does not depend on the order of its input.
#include <hip/hip_runtime.h>

#include "fks_internal.hpp"
#include "prof.hpp"

namespace fks {

constexpr uint64_t kEmpty = ~0ull;   // slot marker; the key ~0 itself is tracked on the side

__global__ void k_dd_init(unsigned long long* __restrict__ tkey, uint32_t* __restrict__ tidx, uint64_t cap,
                          uint32_t* __restrict__ side) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
        tkey[i] = kEmpty;
        tidx[i] = 0xFFFFFFFFu;
    }
    if (blockIdx.x == 0 && threadIdx.x < 2) side[threadIdx.x] = threadIdx.x == 0 ? 0xFFFFFFFFu : 0u;
}

__global__ __launch_bounds__(256) void k_dd_insert(const uint64_t* __restrict__ keys, uint64_t u,
                                                     unsigned long long* __restrict__ tkey, uint32_t* __restrict__ tidx,
                                                     uint64_t mask, uint32_t* __restrict__ side) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < u; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = keys[i];
        if (x == kEmpty) {
            atomicMin(&side[0], (uint32_t)i);
            continue;
        }
        uint64_t h = sm_fin(x) & mask;
        for (uint64_t probe = 0; probe <= mask; ++probe) {
            const unsigned long long old = atomicCAS(&tkey[h], (unsigned long long)kEmpty, (unsigned long long)x);
            if (old == kEmpty || old == x) {
                atomicMin(&tidx[h], (uint32_t)i);
                break;
            }
            h = (h + 1) & mask;
        }
    }
}

__global__ __launch_bounds__(256) void k_dd_compact(const unsigned long long* __restrict__ tkey,
                                                      const uint32_t* __restrict__ tidx, uint64_t cap,
                                                      const uint32_t* __restrict__ vals, uint64_t* __restrict__ out_keys,
                                                      uint32_t* __restrict__ out_vals, uint32_t* __restrict__ side) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = tkey[i];
        if (x != kEmpty) {
            const uint32_t pos = atomicAdd(&side[1], 1u);
            out_keys[pos] = x;
            out_vals[pos] = vals[tidx[i]];
        }
    }
}

__global__ void k_dd_sentinel(const uint32_t* __restrict__ vals, uint64_t* __restrict__ out_keys,
                              uint32_t* __restrict__ out_vals, uint32_t* __restrict__ side) {
    if (threadIdx.x == 0 && side[0] != 0xFFFFFFFFu) {
        const uint32_t pos = side[1]++;
        out_keys[pos] = kEmpty;
        out_vals[pos] = vals[side[0]];
    }
}

}  // namespace fks

using namespace fks;

extern "C" int fks_build_u64_from_array(const uint64_t* d_keys, const uint32_t* d_vals, uint64_t u, uint64_t seed,
                                        const fks_params* params, const fks_allocator* alloc, void* stream,
                                        fks_map** out) {
    if (!out || (u && (!d_keys || !d_vals)) || u >= (1ull << 30) || !allocator_ok(alloc)) return FKS_EINVAL;
    if (u == 0) return fks_build_u64(d_keys, d_vals, 0, seed, params, alloc, stream, out);
    AllocScope scope(alloc);
    hipStream_t st = (hipStream_t)stream;
    uint64_t cap = 1;
    while (cap < 2 * u) cap <<= 1;
    unsigned long long* tkey = (unsigned long long*)dev_alloc(8 * cap, st);
    uint32_t* tidx = (uint32_t*)dev_alloc(4 * cap, st);
    uint64_t* dk = (uint64_t*)dev_alloc(8 * u, st);
    uint32_t* dv = (uint32_t*)dev_alloc(4 * u, st);
    uint32_t* side = (uint32_t*)dev_alloc(64, st);
    auto cleanup = [&]() {
        dev_free(tkey, st);
        dev_free(tidx, st);
        dev_free(dk, st);
        dev_free(dv, st);
        dev_free(side, st);
    };
    if (!tkey || !tidx || !dk || !dv || !side) {
        cleanup();
        return FKS_ENOMEM;
    }
    auto grid = [](uint64_t items) {
        uint64_t g = (items + 255) / 256;
        return (unsigned)(g < 1 ? 1 : g > 65536 ? 65536 : g);
    };
    hipLaunchKernelGGL(k_dd_init, grid(cap), 256, 0, st, tkey, tidx, cap, side);
    FKS_TIMED("fks_dedup_insert", st,
              hipLaunchKernelGGL(k_dd_insert, grid(u), 256, 0, st, d_keys, u, tkey, tidx, cap - 1, side));
    FKS_TIMED("fks_dedup_compact", st,
              hipLaunchKernelGGL(k_dd_compact, grid(cap), 256, 0, st, tkey, tidx, cap, d_vals, dk, dv, side));
    hipLaunchKernelGGL(k_dd_sentinel, 1, 64, 0, st, d_vals, dk, dv, side);
    uint32_t n = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&n, side + 1, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e);
    }
    dev_free(tkey, st);
    dev_free(tidx, st);
    tkey = nullptr;
    tidx = nullptr;
    int rc = fks_build_u64(dk, dv, n, seed, params, alloc, stream, out);
    cleanup();
    return rc;
}
