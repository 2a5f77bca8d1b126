// Batched lookup and membership (Figure 2 lookup; Section 4 operations 2 and 3).
//
// Per needle: j = hash(A) q mod n selects a bucket; probe 1 reads the 16-byte
// record of the bucket's group (slot base, the eight 4-bit sizes, the eight
// trial indices); the bucket's cell is base + sum of the squared sizes before
// it + hash(C[t]) q mod s^2, with the level-two triples C staged in LDS; probe
// 2 reads that cell and compares keys (Section 2.2 membership test).  An empty
// bucket answers "absent" after one probe.  Each thread keeps several needles
// in flight so that their random probes overlap.
#include <hip/hip_runtime.h>

#include "fks_internal.hpp"
#include "prof.hpp"

namespace fks {

constexpr int kLBlock = 256;
constexpr int kQ = 4;   // needles in flight per thread

__global__ void k_fill_outputs(uint64_t m, uint32_t* __restrict__ vals, uint64_t* __restrict__ vals64,
                               uint8_t* __restrict__ found, uint32_t missing, uint64_t missing64) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (vals) vals[i] = missing;
        if (vals64) vals64[i] = missing64;
        if (found) found[i] = 0;
    }
}

// V64: 64-bit values, the high half in the cell's aux word
template <bool WANT_VALS, bool WANT_FOUND, bool V64 = false>
__global__ __launch_bounds__(kLBlock) void k_lookup_u64(const Group* __restrict__ header,
                                                          const Cell* __restrict__ slots, Triple A,
                                                          uint64_t magic, uint32_t n,
                                                          const Triple* __restrict__ Cg, uint32_t T,
                                                          const uint64_t* __restrict__ q, uint64_t m,
                                                          uint32_t* __restrict__ vals,
                                                          uint8_t* __restrict__ found, uint32_t missing,
                                                          uint64_t* __restrict__ vals64 = nullptr,
                                                          uint64_t missing64 = 0) {
    __shared__ Triple C[kTMax];
    for (uint32_t t = threadIdx.x; t < T; t += kLBlock) C[t] = Cg[t];
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * kLBlock * kQ;
    for (uint64_t base = (uint64_t)blockIdx.x * kLBlock * kQ; base < m; base += stride) {
        uint64_t x[kQ];
        Group h[kQ];
        uint32_t kk[kQ];
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
            const uint64_t i = base + threadIdx.x + (uint64_t)k * kLBlock;
            x[k] = i < m ? __builtin_nontemporal_load(q + i) : 0;   // needles and answers stream
        }
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
            const uint64_t i = base + threadIdx.x + (uint64_t)k * kLBlock;
            const uint32_t j = fastmod(mshash(A, x[k]), magic, n);
            kk[k] = j & 7u;
            if (i < m) h[k] = header[j >> 3];
            else h[k] = Group{0, 0, 0, 0};
        }
        Cell c[kQ];
        uint32_t s[kQ];
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
            uint32_t p;
            s[k] = cell_of(h[k], kk[k], C, x[k], p) ? 1u : 0u;
            // read once per needle: a streaming load, so that the cells do not push the group
            // records out of the caches
            c[k] = s[k] ? load_cell_once(slots + p) : Cell{~x[k], 0, 0};
        }
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
            const uint64_t i = base + threadIdx.x + (uint64_t)k * kLBlock;
            if (i < m) {
                const bool hit = s[k] && c[k].key == x[k];
                if (WANT_VALS && V64)
                    __builtin_nontemporal_store(hit ? ((uint64_t)c[k].aux << 32) | c[k].val : missing64, vals64 + i);
                if (WANT_VALS && !V64) __builtin_nontemporal_store(hit ? c[k].val : missing, vals + i);
                if (WANT_FOUND) __builtin_nontemporal_store((uint8_t)(hit ? 1 : 0), found + i);
            }
        }
    }
}

// String needles: fingerprint, probe, then compare the stored bytes on a fingerprint hit.
// The needle and the stored key are read 64 bytes at a time as aligned dwords, so each
// costs one memory round trip; a needle of at most 64 bytes stays in registers for the
// comparison.
template <bool WANT_VALS>
__global__ __launch_bounds__(kLBlock) void k_lookup_bytes(
    const Group* __restrict__ header, const Cell* __restrict__ slots, Triple A, uint64_t beta,
    uint64_t magic, uint32_t n, const Triple* __restrict__ Cg, uint32_t T,
    const int64_t* __restrict__ koff, const uint8_t* __restrict__ kbytes,
    const int64_t* __restrict__ qoff, const uint8_t* __restrict__ qbytes, uint64_t qn, uint64_t m,
    uint32_t* __restrict__ vals, uint8_t* __restrict__ found, uint32_t missing) {
    __shared__ Triple C[kTMax];
    for (uint32_t t = threadIdx.x; t < T; t += kLBlock) C[t] = Cg[t];
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * kLBlock + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * kLBlock) {
        const int64_t a = qoff[i], b = qoff[i + 1];
        if (a < 0 || b < a || (uint64_t)b > qn) {
            // not a range of the needle buffer: nothing is read through it
            if (WANT_VALS) vals[i] = missing;
            if (found) found[i] = 0;
            continue;
        }
        const uint64_t len = (uint64_t)(b - a);
        const uint8_t* s = qbytes + a;
        uint32_t w[kChunkWords];
        const uint64_t y = fingerprint_words(s, len, beta, w);
        const uint32_t j = fastmod(mshash(A, y), magic, n);
        const Group h = header[j >> 3];
        const uint32_t k = j & 7u;
        bool hit = false;
        uint32_t v = missing;
        uint32_t p;
        if (cell_of(h, k, C, y, p)) {
            const Cell c = load_cell_once(slots + p);
            if (c.key == y) {
                const int64_t ka = koff[c.aux], kb = koff[c.aux + 1];
                if ((uint64_t)(kb - ka) == len) {
                    bool eq;
                    if (len <= 4 * kChunkWords) {
                        uint32_t u[kChunkWords];
                        load_words<kChunkWords>(kbytes + ka, (uint32_t)len, u);
                        uint32_t diff = 0;
#pragma unroll
                        for (int q = 0; q < kChunkWords; ++q) diff |= u[q] ^ w[q];
                        eq = diff == 0;
                    } else {
                        eq = bytes_equal(kbytes + ka, s, len);
                    }
                    if (eq) {
                        hit = true;
                        v = c.val;
                    }
                }
            }
        }
        if (WANT_VALS) vals[i] = v;
        if (found) found[i] = hit ? 1 : 0;
    }
}

static unsigned lookup_grid(uint64_t m, uint64_t per_block) {
    uint64_t g = (m + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

}  // namespace fks

using namespace fks;

extern "C" int fks_lookup_u64(const fks_map* map, const uint64_t* d_queries, uint64_t m, uint32_t* d_vals_out,
                              uint8_t* d_found_out, uint32_t missing, void* stream) {
    // 32-bit values from a map with 32-bit values; membership from any integer-key map
    if (!map || (m && !d_queries)) return FKS_EINVAL;
    if (map->kind != 0 && !(map->kind == 2 && !d_vals_out)) return FKS_EINVAL;
    if (m == 0 || (!d_vals_out && !d_found_out)) return FKS_OK;
    hipStream_t st = (hipStream_t)stream;
    if (map->n == 0) {
        FKS_TIMED("fks_fill_outputs", st, hipLaunchKernelGGL(k_fill_outputs, lookup_grid(m, kLBlock), kLBlock, 0, st, m, d_vals_out, nullptr, d_found_out,
                           missing, 0ull));
    } else {
        const unsigned grid = lookup_grid(m, (uint64_t)kLBlock * kQ);
        if (d_vals_out && d_found_out)
            FKS_TIMED("fks_lookup_u64", st, hipLaunchKernelGGL((k_lookup_u64<true, true>), grid, kLBlock, 0, st, map->header, map->slots, map->A,
                               map->magic_n, (uint32_t)map->n, map->C, map->T, d_queries, m, d_vals_out,
                               d_found_out, missing));
        else if (d_vals_out)
            FKS_TIMED("fks_lookup_u64", st, hipLaunchKernelGGL((k_lookup_u64<true, false>), grid, kLBlock, 0, st, map->header, map->slots, map->A,
                               map->magic_n, (uint32_t)map->n, map->C, map->T, d_queries, m, d_vals_out,
                               d_found_out, missing));
        else
            FKS_TIMED("fks_contains_u64", st, hipLaunchKernelGGL((k_lookup_u64<false, true>), grid, kLBlock, 0, st, map->header, map->slots, map->A,
                               map->magic_n, (uint32_t)map->n, map->C, map->T, d_queries, m, d_vals_out,
                               d_found_out, missing));
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

extern "C" int fks_contains_u64(const fks_map* map, const uint64_t* d_queries, uint64_t m, uint8_t* d_found_out,
                                void* stream) {
    if (!d_found_out && m) return FKS_EINVAL;
    return fks_lookup_u64(map, d_queries, m, nullptr, d_found_out, 0, stream);
}

extern "C" int fks_lookup_u64_v64(const fks_map* map, const uint64_t* d_queries, uint64_t m, uint64_t* d_vals_out,
                                  uint8_t* d_found_out, uint64_t missing, void* stream) {
    if (!map || map->kind != 2 || (m && (!d_queries || !d_vals_out))) return FKS_EINVAL;
    if (m == 0) return FKS_OK;
    hipStream_t st = (hipStream_t)stream;
    if (map->n == 0) {
        FKS_TIMED("fks_fill_outputs", st,
                  hipLaunchKernelGGL(k_fill_outputs, lookup_grid(m, kLBlock), kLBlock, 0, st, m, nullptr, d_vals_out,
                                     d_found_out, 0u, missing));
    } else {
        const unsigned grid = lookup_grid(m, (uint64_t)kLBlock * kQ);
        if (d_found_out)
            FKS_TIMED("fks_lookup_u64_v64", st,
                      hipLaunchKernelGGL((k_lookup_u64<true, true, true>), grid, kLBlock, 0, st, map->header,
                                         map->slots, map->A, map->magic_n, (uint32_t)map->n, map->C, map->T,
                                         d_queries, m, nullptr, d_found_out, 0u, d_vals_out, missing));
        else
            FKS_TIMED("fks_lookup_u64_v64", st,
                      hipLaunchKernelGGL((k_lookup_u64<true, false, true>), grid, kLBlock, 0, st, map->header,
                                         map->slots, map->A, map->magic_n, (uint32_t)map->n, map->C, map->T,
                                         d_queries, m, nullptr, nullptr, 0u, d_vals_out, missing));
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

static int lookup_bytes_impl(const fks_map* map, const int64_t* d_q_offsets, const uint8_t* d_q_bytes,
                             uint64_t q_nbytes, uint64_t m, uint32_t* d_vals_out, uint8_t* d_found_out,
                             uint32_t missing, void* stream) {
    if (!map || map->kind != 1 || (m && !d_q_offsets) || (q_nbytes && !d_q_bytes)) return FKS_EINVAL;
    if (m == 0 || (!d_vals_out && !d_found_out)) return FKS_OK;
    hipStream_t st = (hipStream_t)stream;
    if (map->n == 0) {
        FKS_TIMED("fks_fill_outputs", st, hipLaunchKernelGGL(k_fill_outputs, lookup_grid(m, kLBlock), kLBlock, 0, st, m, d_vals_out, nullptr, d_found_out,
                           missing, 0ull));
    } else {
        const unsigned grid = lookup_grid(m, (uint64_t)kLBlock * 2);
        if (d_vals_out)
            FKS_TIMED("fks_lookup_bytes", st, hipLaunchKernelGGL(k_lookup_bytes<true>, grid, kLBlock, 0, st, map->header, map->slots, map->A,
                               map->beta, map->magic_n, (uint32_t)map->n, map->C, map->T, map->ctx_off,
                               map->ctx_bytes, d_q_offsets, d_q_bytes, q_nbytes, m, d_vals_out, d_found_out,
                               missing));
        else
            FKS_TIMED("fks_contains_bytes", st, hipLaunchKernelGGL(k_lookup_bytes<false>, grid, kLBlock, 0, st, map->header, map->slots, map->A,
                               map->beta, map->magic_n, (uint32_t)map->n, map->C, map->T, map->ctx_off,
                               map->ctx_bytes, d_q_offsets, d_q_bytes, q_nbytes, m, d_vals_out, d_found_out,
                               missing));
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

extern "C" int fks_lookup_bytes(const fks_map* map, const int64_t* d_q_offsets, const uint8_t* d_q_bytes,
                                uint64_t q_nbytes, uint64_t m, uint32_t* d_vals_out, uint8_t* d_found_out,
                                uint32_t missing, void* stream) {
    return lookup_bytes_impl(map, d_q_offsets, d_q_bytes, q_nbytes, m, d_vals_out, d_found_out, missing, stream);
}

extern "C" int fks_contains_bytes(const fks_map* map, const int64_t* d_q_offsets, const uint8_t* d_q_bytes,
                                  uint64_t q_nbytes, uint64_t m, uint8_t* d_found_out, void* stream) {
    return lookup_bytes_impl(map, d_q_offsets, d_q_bytes, q_nbytes, m, nullptr, d_found_out, 0, stream);
}
