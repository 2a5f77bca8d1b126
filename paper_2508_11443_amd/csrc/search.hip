// The comparison maps of Section 4: the same (key, value) pairs as a sorted
// array searched by binary search, or in Eytzinger (level-order) layout.
//
// Build: a least-significant-digit radix sort of the pairs, eight passes of
// 8-bit digits.  Each pass is a per-worker digit count, an exclusive scan of the
// (digit, worker) count matrix, and a stable scatter: inside a 4096-record tile
// every wave owns a contiguous stretch and ranks its records round by round
// with a ballot match of the digit bits, so equal digits keep their input
// order, and the tile is staged in LDS sorted by digit so every digit's run is
// written to consecutive addresses.  A check of neighbours then rejects equal
// keys.  The Eytzinger layout gathers the sorted pairs into the level order of
// the complete binary search tree, computing each node's in-order rank in
// closed form.
// Lookup: the branch-free binary search (a fixed ceil(log2 n) steps for every
// needle, four needles per lane in lockstep), or the Eytzinger descent with the
// tree's top levels staged in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fks_internal.hpp"
#include "partition.hpp"
#include "prof.hpp"

struct fks_sorted {
    uint64_t n;
    uint32_t layout;
    int device;
    uint64_t* keys;   // n keys in layout order
    uint32_t* vals;   // their values
    fks_allocator alloc;   // where keys and vals came from (has_alloc == 0: the default pool)
    int has_alloc;
};

namespace fks {

constexpr uint32_t kRB = 256;                 // threads per block
constexpr uint32_t kRItems = 16;              // records per thread per tile
constexpr uint32_t kRTile = kRB * kRItems;    // 4096 records per tile
constexpr uint32_t kWaveSpan = 64 * kRItems;  // records of one wave inside a tile
constexpr uint32_t kTopLevels = 12;           // Eytzinger levels staged in LDS
constexpr uint32_t kTopNodes = (1u << kTopLevels) - 1;

__device__ __forceinline__ void chunk_of(uint64_t n, uint32_t W, uint64_t& a, uint64_t& b) {
    const uint64_t chunk = (n + W - 1) / W;
    a = min(n, (uint64_t)blockIdx.x * chunk);
    b = min(n, a + chunk);
}

// counts of one worker per digit: cnt[digit * W + worker]
__global__ __launch_bounds__(kRB) void k_rs_count(const uint64_t* __restrict__ keys, uint64_t n, uint32_t W,
                                                    uint32_t shift, uint32_t* __restrict__ cnt) {
    __shared__ uint32_t hist[256];
    uint64_t a, b;
    chunk_of(n, W, a, b);
    hist[threadIdx.x] = 0;
    __syncthreads();
    for (uint64_t ts = a; ts < b; ts += kRTile) {
        uint64_t x[kRItems];
#pragma unroll
        for (uint32_t k = 0; k < kRItems; ++k) {
            const uint64_t i = ts + threadIdx.x + (uint64_t)k * kRB;
            x[k] = i < b ? keys[i] : 0;
        }
#pragma unroll
        for (uint32_t k = 0; k < kRItems; ++k)
            if (ts + threadIdx.x + (uint64_t)k * kRB < b) atomicAdd(&hist[(x[k] >> shift) & 255u], 1u);
    }
    __syncthreads();
    cnt[(uint64_t)threadIdx.x * W + blockIdx.x] = hist[threadIdx.x];
}

// exclusive scan of one value per thread across the 256-thread block
__device__ __forceinline__ uint32_t rs_block_exscan(uint32_t v, uint32_t* wsum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t u = __shfl_up(inc, d, 64);
        if (lane >= d) inc += u;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) pre += q < w ? wsum[q] : 0u;
    __syncthreads();
    return pre + inc - v;
}

// Stable scatter of one worker's chunk by the digit at `shift`.
__global__ __launch_bounds__(kRB) void k_rs_scatter(const uint64_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals, uint64_t n, uint32_t W,
                                                      uint32_t shift, const uint32_t* __restrict__ off,
                                                      uint64_t* __restrict__ keys_out,
                                                      uint32_t* __restrict__ vals_out) {
    __shared__ uint64_t skey[kRTile];
    __shared__ uint32_t sval[kRTile];
    __shared__ uint32_t wcnt[4][256];   // per wave and digit: records ranked so far, then the wave's prefix
    __shared__ uint32_t toff[256], run[256];
    __shared__ uint32_t wsum[4];
    uint64_t a, b;
    chunk_of(n, W, a, b);
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    run[tid] = off[(uint64_t)tid * W + blockIdx.x];
    // wave wv reads records ts + wv*1024 + k*64 + lane: coalesced rounds, and the
    // (wave, round, lane) order is the input order
    uint64_t x[kRItems];
    uint32_t v[kRItems];
    auto load = [&](uint64_t ts) {
#pragma unroll
        for (uint32_t k = 0; k < kRItems; ++k) {
            const uint64_t i = ts + wv * kWaveSpan + k * 64 + lane;
            x[k] = i < b ? keys[i] : 0;
            v[k] = i < b ? vals[i] : 0;
        }
    };
    if (a < b) load(a);
    for (uint64_t ts = a; ts < b; ts += kRTile) {
#pragma unroll
        for (uint32_t w = 0; w < 4; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        uint32_t rank[kRItems];
#pragma unroll
        for (uint32_t k = 0; k < kRItems; ++k) {
            const bool valid = ts + wv * kWaveSpan + k * 64 + lane < b;
            const uint32_t d = (uint32_t)(x[k] >> shift) & 255u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (uint32_t bit = 0; bit < 8; ++bit) {
                const uint64_t m = __ballot((d >> bit) & 1u);
                peers &= ((d >> bit) & 1u) ? m : ~m;
            }
            if (valid) {
                const uint32_t before = wcnt[wv][d];
                rank[k] = before + (uint32_t)__popcll(peers & lt);
                if ((peers & lt) == 0) wcnt[wv][d] = before + (uint32_t)__popcll(peers);
            }
        }
        __syncthreads();
        // per digit: the tile's count, every wave's prefix, the digit's place in the tile
        uint32_t c = 0;
#pragma unroll
        for (uint32_t w = 0; w < 4; ++w) {
            const uint32_t cw = wcnt[w][tid];
            wcnt[w][tid] = c;
            c += cw;
        }
        toff[tid] = rs_block_exscan(c, wsum);
        __syncthreads();
#pragma unroll
        for (uint32_t k = 0; k < kRItems; ++k) {
            if (ts + wv * kWaveSpan + k * 64 + lane < b) {
                const uint32_t d = (uint32_t)(x[k] >> shift) & 255u;
                const uint32_t e = toff[d] + wcnt[wv][d] + rank[k];
                skey[e] = x[k];
                sval[e] = v[k];
            }
        }
        if (ts + kRTile < b) load(ts + kRTile);   // the next tile is in flight during the writes
        __syncthreads();
        const uint32_t cnt = (uint32_t)min((uint64_t)kRTile, b - ts);
        for (uint32_t e = tid; e < cnt; e += kRB) {
            const uint64_t key = skey[e];
            const uint32_t d = (uint32_t)(key >> shift) & 255u;
            const uint64_t dest = (uint64_t)run[d] + (e - toff[d]);
            keys_out[dest] = key;
            vals_out[dest] = sval[e];
        }
        __syncthreads();
        run[tid] += c;
    }
}

__global__ void k_rs_adjacent_equal(const uint64_t* __restrict__ k, uint64_t n, uint32_t* __restrict__ flag) {
    bool dup = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dup |= k[i] == k[i - 1];
    if (dup) atomicOr(flag, 1u);
}

// Level order of the complete binary search tree on n sorted records.  Node i
// (1-based) at depth d = floor(log2 i) would have in-order position
// r = (2(i - 2^d) + 1) 2^(H-d) - 1 in the perfect tree of depth H = floor(log2 n);
// the last level holds only its first L = n - 2^H + 1 leaves, whose perfect
// positions are the even numbers below 2L, so r drops by the missing leaves
// (even positions in [2L, r)).
__global__ void k_eytzinger(const uint64_t* __restrict__ sk, const uint32_t* __restrict__ sv, uint64_t n,
                            uint32_t H, uint64_t L, uint64_t* __restrict__ ek, uint32_t* __restrict__ ev) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i <= n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t d = 63u - (uint32_t)__clzll(i);
        const int64_t r = (int64_t)((((i - (1ull << d)) << 1) + 1) << (H - d)) - 1;
        const int64_t gone = r > (int64_t)(2 * L) ? (r - (int64_t)(2 * L) + 1) >> 1 : 0;
        const uint64_t rank = (uint64_t)(r - gone);
        ek[i - 1] = sk[rank];
        ev[i - 1] = sv[rank];
    }
}

constexpr uint32_t kQ = 4;   // needles per lane in lockstep

template <bool WANT_VALS>
__global__ __launch_bounds__(256) void k_bsearch(const uint64_t* __restrict__ sk, const uint32_t* __restrict__ sv,
                                                   uint64_t n, const uint64_t* __restrict__ q, uint64_t m,
                                                   uint32_t* __restrict__ out_vals, uint8_t* __restrict__ out_found,
                                                   uint32_t missing) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * kQ;
    for (uint64_t j0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kQ; j0 < m; j0 += stride) {
        uint64_t x[kQ], lo[kQ];
#pragma unroll
        for (uint32_t u = 0; u < kQ; ++u) {
            x[u] = j0 + u < m ? q[j0 + u] : 0;
            lo[u] = 0;
        }
        // the lower bound stays in [lo, lo + len]; len shrinks the same way for every needle
        uint64_t len = n;
        while (len > 1) {
            const uint64_t half = len >> 1;
#pragma unroll
            for (uint32_t u = 0; u < kQ; ++u) lo[u] = sk[lo[u] + half] < x[u] ? lo[u] + half : lo[u];
            len -= half;
        }
#pragma unroll
        for (uint32_t u = 0; u < kQ; ++u) {
            if (j0 + u >= m) break;
            // the lower bound is lo or lo + 1
            uint64_t pos = lo[u];
            bool hit = false;
            if (n) {
                const uint64_t kk = sk[pos];
                if (kk < x[u]) {
                    ++pos;
                    hit = pos < n && sk[pos] == x[u];
                } else {
                    hit = kk == x[u];
                }
            }
            out_found[j0 + u] = hit;
            if (WANT_VALS) out_vals[j0 + u] = hit ? sv[pos] : missing;
        }
    }
}

template <bool WANT_VALS>
__global__ __launch_bounds__(256) void k_eytz_search(const uint64_t* __restrict__ ek,
                                                       const uint32_t* __restrict__ ev, uint64_t n,
                                                       const uint64_t* __restrict__ q, uint64_t m,
                                                       uint32_t* __restrict__ out_vals,
                                                       uint8_t* __restrict__ out_found, uint32_t missing) {
    __shared__ uint64_t top[kTopNodes];
    const uint64_t ntop = min(n, (uint64_t)kTopNodes);
    for (uint32_t i = threadIdx.x; i < ntop; i += blockDim.x) top[i] = ek[i];
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * kQ;
    for (uint64_t j0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kQ; j0 < m; j0 += stride) {
        uint64_t x[kQ], i[kQ];
#pragma unroll
        for (uint32_t u = 0; u < kQ; ++u) {
            x[u] = j0 + u < m ? q[j0 + u] : 0;
            i[u] = 1;
        }
        // descend: a right turn appends a 1 to the node number, a left turn a 0
        for (uint32_t lvl = 0; lvl < kTopLevels; ++lvl) {
#pragma unroll
            for (uint32_t u = 0; u < kQ; ++u)
                if (i[u] <= ntop) i[u] = 2 * i[u] + (top[i[u] - 1] < x[u] ? 1 : 0);
        }
        bool more = true;
        while (more) {
            more = false;
#pragma unroll
            for (uint32_t u = 0; u < kQ; ++u)
                if (i[u] <= n) {
                    i[u] = 2 * i[u] + (ek[i[u] - 1] < x[u] ? 1 : 0);
                    more = true;
                }
        }
#pragma unroll
        for (uint32_t u = 0; u < kQ; ++u) {
            if (j0 + u >= m) break;
            // the lower bound is the node of the last left turn (0: none)
            const uint64_t lb = i[u] >> (__ffsll((long long)~i[u]));
            const bool hit = lb != 0 && ek[lb - 1] == x[u];
            out_found[j0 + u] = hit;
            if (WANT_VALS) out_vals[j0 + u] = hit ? ev[lb - 1] : missing;
        }
    }
}

static unsigned sgrid(uint64_t items, uint64_t per_block, unsigned cap) {
    uint64_t g = (items + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g > cap ? cap : g);
}

}  // namespace fks

using namespace fks;

extern "C" int fks_sorted_build_u64(const uint64_t* d_keys, const uint32_t* d_vals, uint64_t n, uint32_t layout,
                                    const fks_allocator* alloc, void* stream, fks_sorted** out) {
    if (!out || (n && (!d_keys || !d_vals)) || n >= (1ull << 32) || layout > 1 || !allocator_ok(alloc))
        return FKS_EINVAL;
    AllocScope scope(alloc);
    hipStream_t st = (hipStream_t)stream;
    fks_sorted* S = new fks_sorted{};
    keep_allocator(alloc, S->alloc, S->has_alloc);
    S->n = n;
    S->layout = layout;
    (void)hipGetDevice(&S->device);
    if (n == 0) {
        *out = S;
        return FKS_OK;
    }
    const uint32_t W = (uint32_t)std::min<uint64_t>(4096, std::max<uint64_t>(1, n / (4 * (uint64_t)kRTile)));
    const uint64_t N = 256ull * W;
    uint64_t* kb[2] = {(uint64_t*)dev_alloc(8 * n, st), (uint64_t*)dev_alloc(8 * n, st)};
    uint32_t* vb[2] = {(uint32_t*)dev_alloc(4 * n, st), (uint32_t*)dev_alloc(4 * n, st)};
    uint32_t* cnt = (uint32_t*)dev_alloc(4 * N, st);
    uint32_t* off = (uint32_t*)dev_alloc(4 * N, st);
    uint32_t* tsum = (uint32_t*)dev_alloc(4 * exscan_tiles(N), st);
    uint64_t* tpre = (uint64_t*)dev_alloc(8 * (exscan_tiles(N) + 1), st);
    uint32_t* flag = (uint32_t*)dev_alloc(64, st);
    uint32_t* hflag = nullptr;
    auto cleanup = [&]() {
        for (int z = 0; z < 2; ++z) {
            dev_free(kb[z], st);
            dev_free(vb[z], st);
        }
        dev_free(cnt, st);
        dev_free(off, st);
        dev_free(tsum, st);
        dev_free(tpre, st);
        dev_free(flag, st);
        if (hflag) (void)hipHostFree(hflag);
    };
    if (!kb[0] || !kb[1] || !vb[0] || !vb[1] || !cnt || !off || !tsum || !tpre || !flag ||
        hipHostMalloc((void**)&hflag, 4, hipHostMallocDefault) != hipSuccess) {
        cleanup();
        delete S;
        return FKS_ENOMEM;
    }
    const uint64_t* kin = d_keys;
    const uint32_t* vin = d_vals;
    int cur = 0;
    for (uint32_t pass = 0; pass < 8; ++pass) {
        const uint32_t shift = 8 * pass;
        FKS_TIMED("fks_sort_count", st, hipLaunchKernelGGL(k_rs_count, W, kRB, 0, st, kin, n, W, shift, cnt));
        exscan_u32(cnt, N, tsum, tpre, off, st);
        FKS_TIMED("fks_sort_scatter", st,
                  hipLaunchKernelGGL(k_rs_scatter, W, kRB, 0, st, kin, vin, n, W, shift, off, kb[cur], vb[cur]));
        kin = kb[cur];
        vin = vb[cur];
        cur ^= 1;
    }
    // kin/vin: the sorted pairs; the other buffer pair is free
    int rc = FKS_OK;
    hipError_t e = hipMemsetAsync(flag, 0, 4, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_rs_adjacent_equal, sgrid(n, 256, 8192), 256, 0, st, kin, n, flag);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(hflag, flag, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = hip_fail(e);
    else if (*hflag) rc = FKS_EDUPKEY;
    if (rc == FKS_OK && layout == 1) {
        uint32_t H = 0;
        while ((2ull << H) <= n) ++H;   // floor(log2 n)
        const uint64_t L = n - ((1ull << H) - 1);
        FKS_TIMED("fks_eytzinger", st,
                  hipLaunchKernelGGL(k_eytzinger, sgrid(n, 256, 65536), 256, 0, st, kin, vin, n, H, L, kb[cur],
                                     vb[cur]));
        kin = kb[cur];
        vin = vb[cur];
        cur ^= 1;
        e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(e);
    }
    if (rc != FKS_OK) {
        cleanup();
        delete S;
        return rc;
    }
    // keep the final pair of arrays, release the rest
    S->keys = const_cast<uint64_t*>(kin);
    S->vals = const_cast<uint32_t*>(vin);
    kb[cur ^ 1] = nullptr;
    vb[cur ^ 1] = nullptr;
    cleanup();
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        dev_free(S->keys, st);
        dev_free(S->vals, st);
        delete S;
        return hip_fail(e);
    }
    *out = S;
    return FKS_OK;
}

extern "C" int fks_sorted_lookup_u64(const fks_sorted* S, const uint64_t* d_q, uint64_t m, uint32_t* d_vals_out,
                                     uint8_t* d_found_out, uint32_t missing_value, void* stream) {
    if (!S || (m && (!d_q || !d_found_out))) return FKS_EINVAL;
    if (m == 0) return FKS_OK;
    hipStream_t st = (hipStream_t)stream;
    const unsigned grid = sgrid(m, 256 * kQ, 16384);
    if (S->layout == 0) {
        if (d_vals_out)
            FKS_TIMED("fks_bsearch_u64", st,
                      hipLaunchKernelGGL(k_bsearch<true>, grid, 256, 0, st, S->keys, S->vals, S->n, d_q, m,
                                         d_vals_out, d_found_out, missing_value));
        else
            FKS_TIMED("fks_bsearch_u64", st,
                      hipLaunchKernelGGL(k_bsearch<false>, grid, 256, 0, st, S->keys, S->vals, S->n, d_q, m,
                                         nullptr, d_found_out, missing_value));
    } else {
        if (d_vals_out)
            FKS_TIMED("fks_eytzinger_u64", st,
                      hipLaunchKernelGGL(k_eytz_search<true>, grid, 256, 0, st, S->keys, S->vals, S->n, d_q, m,
                                         d_vals_out, d_found_out, missing_value));
        else
            FKS_TIMED("fks_eytzinger_u64", st,
                      hipLaunchKernelGGL(k_eytz_search<false>, grid, 256, 0, st, S->keys, S->vals, S->n, d_q, m,
                                         nullptr, d_found_out, missing_value));
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

extern "C" int fks_sorted_export(const fks_sorted* S, uint64_t* h_keys, uint32_t* h_vals) {
    if (!S || (S->n && (!h_keys || !h_vals))) return FKS_EINVAL;
    if (S->n == 0) return FKS_OK;
    hipError_t e = hipMemcpy(h_keys, S->keys, 8 * S->n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(h_vals, S->vals, 4 * S->n, hipMemcpyDeviceToHost);
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

extern "C" int fks_sorted_info(const fks_sorted* S, uint64_t* n, uint32_t* layout) {
    if (!S) return FKS_EINVAL;
    if (n) *n = S->n;
    if (layout) *layout = S->layout;
    return FKS_OK;
}

extern "C" void fks_sorted_destroy(fks_sorted* S) {
    if (!S) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->device);
    {
        // back where the build took them from; frees are ordered on the null stream,
        // after all work already queued on it
        AllocScope scope(S->has_alloc ? &S->alloc : nullptr);
        dev_free(S->keys, nullptr);
        dev_free(S->vals, nullptr);
    }
    (void)hipSetDevice(prev);
    delete S;
}
