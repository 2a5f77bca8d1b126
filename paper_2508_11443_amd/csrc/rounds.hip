// The paper's own level-two schedule: the sortless flattened rounds of
// Section 2.5, one round per trial index, each a handful of data-parallel
// passes over the keys that are still unplaced.
//
// Round t, for the keys (o, key) of the remaining buckets (o indexes the
// compacted list of remaining buckets, as okeys does):
//   seghashes      cell = presum(s^2)[o] + hash(C[t]) key mod s[o]^2
//   segcollisions  counts = hist flat cells; a bucket collides when one of its
//                  cells counts more than one key (segor of counts > 1)
//   segresult      buckets without a collision are done and keep t
//   filter, presum the colliding buckets and their keys go on, re-indexed by
//                  the exclusive prefix sum of the collision flags
// Under the shared-triple reading (round t uses level-two triple t for every
// bucket) the trial a bucket keeps equals make_2's first success, so the table
// written from these trials is byte for byte the per-bucket schedule's.  The
// histogram over the flat cell space uses device atomics, as the paper's hist
// does; this schedule exists to measure that formulation on the same GPU.
#include <hip/hip_runtime.h>

#include <vector>

#include "fks_internal.hpp"
#include "prof.hpp"
#include "rounds.hpp"

namespace fks {

constexpr int kRB = 256;

static unsigned rgrid(uint64_t items) {
    uint64_t g = (items + kRB - 1) / kRB;
    return (unsigned)(g < 1 ? 1 : g > 65536 ? 65536 : g);
}

#define GRID_STRIDE(i, count) \
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (count); i += (uint64_t)gridDim.x * blockDim.x)

__global__ void k_r_fill(uint32_t* p, uint64_t count, uint32_t v) {
    GRID_STRIDE(i, count) p[i] = v;
}

// zero the first *count entries (the flat cell space of this round)
__global__ void k_r_zero_flat(uint32_t* p, const uint32_t* __restrict__ count) {
    const uint64_t c = *count;
    GRID_STRIDE(i, c) p[i] = 0;
}

// shape and the non-empty flags of every bucket
__global__ void k_r_shape(const uint32_t* __restrict__ words, uint64_t n, uint32_t* __restrict__ nz) {
    GRID_STRIDE(j, n) nz[j] = nib(words[j >> 3], (uint32_t)(j & 7)) != 0;
}

// ishape: the compacted list of non-empty buckets (index, size)
__global__ void k_r_ishape(const uint32_t* __restrict__ words, uint64_t n, const uint32_t* __restrict__ nz,
                           const uint32_t* __restrict__ pos, uint32_t* __restrict__ bj, uint32_t* __restrict__ bs) {
    GRID_STRIDE(j, n) {
        if (nz[j]) {
            bj[pos[j]] = (uint32_t)j;
            bs[pos[j]] = nib(words[j >> 3], (uint32_t)(j & 7));
        }
    }
}

// okeys: every key with the compacted index of its bucket
__global__ void k_r_okeys(const uint64_t* __restrict__ keys, uint64_t n, Triple A, uint64_t magic,
                          const uint32_t* __restrict__ pos, uint64_t* __restrict__ ok, uint32_t* __restrict__ oo) {
    GRID_STRIDE(i, n) {
        const uint64_t x = keys[i];
        ok[i] = x;
        oo[i] = pos[fastmod(mshash(A, x), magic, (uint32_t)n)];
    }
}

__global__ void k_r_squares(const uint32_t* __restrict__ bs, uint64_t m, uint32_t* __restrict__ sq) {
    GRID_STRIDE(o, m) sq[o] = bs[o] * bs[o];
}

// seghashes + hist
__global__ void k_r_hash(const uint64_t* __restrict__ ok, const uint32_t* __restrict__ oo, uint64_t K,
                         const uint32_t* __restrict__ bs, const uint32_t* __restrict__ sh, Triple c,
                         uint32_t* __restrict__ cell, uint32_t* __restrict__ counts) {
    GRID_STRIDE(i, K) {
        const uint32_t o = oo[i], s = bs[o];
        const uint32_t h = sh[o] + mshash(c, ok[i]) % (s * s);
        cell[i] = h;
        atomicAdd(&counts[h], 1u);
    }
}

// segor of (counts > 1) per bucket
__global__ void k_r_segor(const uint32_t* __restrict__ oo, uint64_t K, const uint32_t* __restrict__ cell,
                          const uint32_t* __restrict__ counts, uint32_t* __restrict__ coll) {
    GRID_STRIDE(i, K) {
        if (counts[cell[i]] > 1) coll[oo[i]] = 1;
    }
}

// segresult: buckets that are done keep this round's trial; the others are
// re-indexed by the prefix sum of the collision flags
__global__ void k_r_result(const uint32_t* __restrict__ bj, const uint32_t* __restrict__ bs, uint64_t m,
                           const uint32_t* __restrict__ coll, const uint32_t* __restrict__ npos, uint32_t t,
                           uint8_t* __restrict__ t_out, uint32_t* __restrict__ bj2, uint32_t* __restrict__ bs2) {
    GRID_STRIDE(o, m) {
        if (coll[o]) {
            bj2[npos[o]] = bj[o];
            bs2[npos[o]] = bs[o];
        } else {
            t_out[bj[o]] = (uint8_t)t;
        }
    }
}

// filter: keys of colliding buckets, re-indexed; order inside the output is
// not needed by the next round
__global__ __launch_bounds__(kRB) void k_r_filter(const uint64_t* __restrict__ ok, const uint32_t* __restrict__ oo,
                                                    uint64_t K, const uint32_t* __restrict__ coll,
                                                    const uint32_t* __restrict__ npos, uint64_t* __restrict__ ok2,
                                                    uint32_t* __restrict__ oo2, uint32_t* __restrict__ counter) {
    __shared__ uint32_t blk, base;
    GRID_STRIDE(i0, ((K + kRB - 1) / kRB) * kRB) {
        if (threadIdx.x == 0) blk = 0;
        __syncthreads();
        const uint64_t i = i0;
        bool keep = false;
        uint32_t mine = 0;
        if (i < K) {
            keep = coll[oo[i]] != 0;
            if (keep) mine = atomicAdd(&blk, 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) base = blk ? atomicAdd(counter, blk) : 0u;
        __syncthreads();
        if (keep) {
            ok2[base + mine] = ok[i];
            oo2[base + mine] = npos[oo[i]];
        }
        __syncthreads();
    }
}

// exclusive prefix of a u32 array (one block per 2048 entries, then the block
// totals), writing the total to *total
__global__ __launch_bounds__(kRB) void k_r_scan_tiles(const uint32_t* __restrict__ in, uint64_t N,
                                                        uint32_t* __restrict__ out, uint32_t* __restrict__ tsum) {
    __shared__ uint32_t ws[kRB / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kRB * 8 + (uint64_t)threadIdx.x * 8;
    uint32_t v[8], s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = base + k < N ? in[base + k] : 0u;
        s += v[k];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t u = __shfl_up(inc, d, 64);
        if (lane >= d) inc += u;
    }
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int q = 0; q < kRB / 64; ++q) {
        if (q < w) pre += ws[q];
        tot += ws[q];
    }
    uint32_t run = pre + inc - s;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (base + k < N) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_r_scan_top(uint32_t* __restrict__ tsum, uint32_t nt,
                                                       uint32_t* __restrict__ total) {
    __shared__ uint32_t part[1024];
    const uint32_t per = (nt + 1023) / 1024;
    const uint32_t a = threadIdx.x * per, b = min(nt, a + per);
    uint32_t s = 0;
    for (uint32_t i = a; i < b; ++i) s += tsum[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
        const uint32_t v = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (uint32_t i = a; i < b; ++i) {
        const uint32_t c = tsum[i];
        tsum[i] = run;
        run += c;
    }
    if (threadIdx.x == 1023) *total = part[1023];
}

__global__ __launch_bounds__(kRB) void k_r_scan_add(uint32_t* __restrict__ out, uint64_t N,
                                                      const uint32_t* __restrict__ tsum) {
    const uint64_t base = (uint64_t)blockIdx.x * kRB * 8 + (uint64_t)threadIdx.x * 8;
    const uint32_t add = tsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (base + k < N) out[base + k] += add;
}

struct RoundsScratch {
    uint32_t *nz, *pos, *tsum, *tot;
    uint32_t *bj[2], *bs[2], *sq, *sh, *coll, *npos, *counts, *cell;
    uint64_t* ok[2];
    uint32_t* oo[2];
    uint32_t* host;   // pinned: totals read back
};

static void presum(const uint32_t* in, uint64_t N, uint32_t* out, uint32_t* tsum, uint32_t* total, hipStream_t st) {
    const uint32_t nt = (uint32_t)((N + kRB * 8 - 1) / (kRB * 8));
    hipLaunchKernelGGL(k_r_scan_tiles, nt ? nt : 1, kRB, 0, st, in, N, out, tsum);
    hipLaunchKernelGGL(k_r_scan_top, 1, 1024, 0, st, tsum, nt ? nt : 1, total);
    hipLaunchKernelGGL(k_r_scan_add, nt ? nt : 1, kRB, 0, st, out, N, tsum);
}

int rounds_search(const uint64_t* keys, uint64_t n, uint64_t S, const Triple& A, uint64_t magic,
                  const uint32_t* words, const Triple* Ch, uint32_t T, uint8_t* t_out, bool* exhausted,
                  hipStream_t st) {
    RoundsScratch w{};
    std::vector<void*> owned;
    auto grab = [&](size_t bytes) {
        void* p = dev_alloc(bytes ? bytes : 16, st);
        owned.push_back(p);
        return p;
    };
    const uint64_t ntiles = (n + kRB * 8 - 1) / (kRB * 8) + 1;
    w.nz = (uint32_t*)grab(4 * n);
    w.pos = (uint32_t*)grab(4 * n);
    w.tsum = (uint32_t*)grab(4 * ntiles);
    w.tot = (uint32_t*)grab(64);
    for (int b = 0; b < 2; ++b) {
        w.bj[b] = (uint32_t*)grab(4 * n);
        w.bs[b] = (uint32_t*)grab(4 * n);
        w.ok[b] = (uint64_t*)grab(8 * n);
        w.oo[b] = (uint32_t*)grab(4 * n);
    }
    w.sq = (uint32_t*)grab(4 * n);
    w.sh = (uint32_t*)grab(4 * n);
    w.coll = (uint32_t*)grab(4 * n);
    w.npos = (uint32_t*)grab(4 * n);
    w.counts = (uint32_t*)grab(4 * (S ? S : 1));
    w.cell = (uint32_t*)grab(4 * n);
    auto release = [&]() {
        for (void* p : owned) dev_free(p, st);
    };
    for (void* p : owned)
        if (!p) {
            release();
            return FKS_ENOMEM;
        }
    static thread_local uint32_t* host = nullptr;
    if (!host && hipHostMalloc((void**)&host, 64, hipHostMallocDefault) != hipSuccess) host = nullptr;
    if (!host) {
        release();
        return FKS_ENOMEM;
    }
    // ishape and okeys
    hipLaunchKernelGGL(k_r_shape, rgrid(n), kRB, 0, st, words, n, w.nz);
    presum(w.nz, n, w.pos, w.tsum, w.tot, st);
    hipLaunchKernelGGL(k_r_ishape, rgrid(n), kRB, 0, st, words, n, w.nz, w.pos, w.bj[0], w.bs[0]);
    hipLaunchKernelGGL(k_r_okeys, rgrid(n), kRB, 0, st, keys, n, A, magic, w.pos, w.ok[0], w.oo[0]);
    hipError_t e = hipMemcpyAsync(host, w.tot, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        release();
        return hip_fail(e);
    }
    uint64_t m = host[0], K = n;
    int cur = 0;
    uint32_t t = 0;
    for (; t < T && K > 0; ++t) {
        const int nxt = cur ^ 1;
        {
            ProfScope timed("fks_rounds_round", st);
            hipLaunchKernelGGL(k_r_squares, rgrid(m), kRB, 0, st, w.bs[cur], m, w.sq);
            presum(w.sq, m, w.sh, w.tsum, w.tot, st);
            hipLaunchKernelGGL(k_r_zero_flat, rgrid(S), kRB, 0, st, w.counts, w.tot);
            hipLaunchKernelGGL(k_r_hash, rgrid(K), kRB, 0, st, w.ok[cur], w.oo[cur], K, w.bs[cur], w.sh, Ch[t],
                               w.cell, w.counts);
            hipLaunchKernelGGL(k_r_fill, rgrid(m), kRB, 0, st, w.coll, m, 0u);
            hipLaunchKernelGGL(k_r_segor, rgrid(K), kRB, 0, st, w.oo[cur], K, w.cell, w.counts, w.coll);
            presum(w.coll, m, w.npos, w.tsum, w.tot + 1, st);
            hipLaunchKernelGGL(k_r_result, rgrid(m), kRB, 0, st, w.bj[cur], w.bs[cur], m, w.coll, w.npos, t, t_out,
                               w.bj[nxt], w.bs[nxt]);
            hipLaunchKernelGGL(k_r_fill, 1, 64, 0, st, w.tot + 2, 1, 0u);
            hipLaunchKernelGGL(k_r_filter, rgrid(K), kRB, 0, st, w.ok[cur], w.oo[cur], K, w.coll, w.npos, w.ok[nxt],
                               w.oo[nxt], w.tot + 2);
        }
        e = hipMemcpyAsync(host, w.tot, 12, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            release();
            return hip_fail(e);
        }
        m = host[1];
        K = host[2];
        cur = nxt;
    }
    *exhausted = K > 0;
    release();
    e = hipGetLastError();
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

}  // namespace fks
