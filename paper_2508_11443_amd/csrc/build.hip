// Data-parallel construction of the two-level hash map (Sections 2.2-2.5).
//
// One level-one attempt r is five steps on the stream:
//   hist    g k = hash(A_r) k mod n for every key; 4-bit bucket counters packed
//           eight to a word (the histogram of Figure 1, with device atomics);
//           the value an atomic returns is the key's rank inside its bucket.
//   scan    exclusive prefix sums over groups of eight buckets of the bucket
//           sizes (where each bucket's keys start) and of their squares (where
//           each bucket's cells start) -- the offsets of Section 2.2 -- and the
//           table size S, read back to the host to check S <= c*n and size the
//           cell array.
//   group   counting-sort scatter: each key and its value go to the bucket's
//           key range at its rank (the groupby of make_1, without sorting).
//   search  per bucket, the smallest trial t whose level-two triple sends the
//           bucket's keys to distinct cells mod s^2 (make_2), with the keys of
//           256 consecutive buckets staged in LDS and one lane per bucket;
//   write   the same kernel fills the 256 buckets' contiguous cell range in LDS
//           (empty cells copy the bucket's lowest occupied cell) and streams
//           it out with coalesced 16-byte stores, then writes the 32 group
//           headers.
// String maps first fingerprint every key with the attempt's base and run the
// same steps on the fingerprints.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "fks_internal.hpp"
#include "partition.hpp"
#include "prof.hpp"
#include "rounds.hpp"

#include <cstdlib>

namespace fks {

constexpr int kBlock = 256;
constexpr int kHistItems = 4;
constexpr int kScanItems = 8;                         // groups per thread
constexpr int kScanTile = kBlock * kScanItems;        // groups per scan tile
constexpr int kScanTop = 1024;                        // threads of the tile-prefix kernel
constexpr uint32_t kKeyCap = 512;                     // keys staged per search block
constexpr uint32_t kCellCap = 2048;                   // cells staged per search block

// control words of one attempt (device), read back through Readback
struct Ctrl {
    uint64_t S;
    uint32_t oversize, bad_input, exhausted, dup, max_t, pad;   // same layout as Readback
};

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t count, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_ctrl(Ctrl* c) {
    if (threadIdx.x == 0) {
        c->S = 0;
        c->oversize = c->bad_input = c->exhausted = c->dup = c->max_t = c->pad = 0;
    }
}

// ---- string fingerprints -----------------------------------------------------

__device__ inline uint64_t fingerprint_dev(const uint8_t* __restrict__ s, uint64_t len, uint64_t beta) {
    uint64_t acc = len % kP61;
    uint64_t full = len / 4;
    for (uint64_t k = 0; k < full; ++k) {
        const uint8_t* p = s + 4 * k;
        uint32_t w = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
        acc = addmod61(mulmod61(acc, beta), w);
    }
    uint64_t rest = len - 4 * full;
    if (rest) {
        const uint8_t* p = s + 4 * full;
        uint32_t w = 0;
        for (uint64_t q = 0; q < rest; ++q) w |= (uint32_t)p[q] << (8 * q);
        acc = addmod61(mulmod61(acc, beta), w);
    }
    return acc;
}

__global__ __launch_bounds__(kBlock) void k_fingerprint(const int64_t* __restrict__ off,
                                                          const uint8_t* __restrict__ bytes,
                                                          uint64_t n, uint64_t beta,
                                                          uint64_t* __restrict__ y) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        int64_t a = off[i], b = off[i + 1];
        y[i] = fingerprint_dev(bytes + a, (uint64_t)(b - a), beta);
    }
}

__global__ void k_check_offsets(const int64_t* __restrict__ off, uint64_t n, uint64_t nbytes, Ctrl* ctrl) {
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        int64_t a = off[i];
        if (a < 0 || (uint64_t)a > nbytes) bad = true;
        if (i < n && off[i + 1] < a) bad = true;
    }
    if (bad) atomicOr(&ctrl->bad_input, 1u);
}

// ---- step 1: level-one histogram ------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_hist(const uint64_t* __restrict__ keys, uint64_t n,
                                                   Triple A, uint64_t magic,
                                                   uint32_t* __restrict__ sizes,
                                                   uint8_t* __restrict__ rank, Ctrl* ctrl) {
    const uint64_t i0 = (uint64_t)blockIdx.x * (kBlock * kHistItems) + threadIdx.x;
    uint64_t x[kHistItems];
#pragma unroll
    for (int k = 0; k < kHistItems; ++k) {
        uint64_t i = i0 + (uint64_t)k * kBlock;
        x[k] = i < n ? keys[i] : 0;
    }
    bool over = false;
#pragma unroll
    for (int k = 0; k < kHistItems; ++k) {
        uint64_t i = i0 + (uint64_t)k * kBlock;
        if (i < n) {
            uint32_t j = fastmod(mshash(A, x[k]), magic, (uint32_t)n);
            uint32_t sh = 4 * (j & 7u);
            uint32_t old = atomicAdd(&sizes[j >> 3], 1u << sh);
            uint32_t r = (old >> sh) & 15u;
            over |= (r == 15u);
            rank[i] = (uint8_t)r;
        }
    }
    if (over) atomicOr(&ctrl->oversize, 1u);
}

// ---- step 2: scans over groups ------------------------------------------------------

__device__ inline void group_stats(uint32_t sz, uint32_t& cnt, uint32_t& sq) {
    cnt = 0;
    sq = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        uint32_t s = nib(sz, k);
        cnt += s;
        sq += s * s;
    }
}

// inclusive scan of (a, b) across one wave of 64 lanes
__device__ inline void wave_scan2(uint32_t& a, uint32_t& b) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t ua = __shfl_up(a, d, 64);
        uint32_t ub = __shfl_up(b, d, 64);
        if (lane >= d) {
            a += ua;
            b += ub;
        }
    }
}

// block-wide exclusive scan of (a, b) for 256 threads; also returns the totals
__device__ inline void block_exscan2(uint32_t& a, uint32_t& b, uint32_t& tot_a, uint32_t& tot_b) {
    __shared__ uint32_t wa[kBlock / 64], wb[kBlock / 64];
    uint32_t ia = a, ib = b;
    wave_scan2(ia, ib);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 63) {
        wa[w] = ia;
        wb[w] = ib;
    }
    __syncthreads();
    uint32_t pa = 0, pb = 0;
    tot_a = 0;
    tot_b = 0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) {
        if (q < w) {
            pa += wa[q];
            pb += wb[q];
        }
        tot_a += wa[q];
        tot_b += wb[q];
    }
    a = pa + ia - a;
    b = pb + ib - b;
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ sizes, uint64_t G,
                                                          uint64_t* __restrict__ tile_cnt,
                                                          uint64_t* __restrict__ tile_sq) {
    const uint64_t g0 = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t cnt = 0, sq = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint64_t g = g0 + k;
        if (g < G) {
            uint32_t c, q;
            group_stats(sizes[g], c, q);
            cnt += c;
            sq += q;
        }
    }
    uint32_t ta, tb;
    block_exscan2(cnt, sq, ta, tb);
    if (threadIdx.x == 0) {
        tile_cnt[blockIdx.x] = ta;
        tile_sq[blockIdx.x] = tb;
    }
}

// one block: exclusive scan of the tile totals in place; total S to ctrl
__global__ __launch_bounds__(kScanTop) void k_scan_tiles(uint64_t* __restrict__ tile_cnt,
                                                           uint64_t* __restrict__ tile_sq,
                                                           uint64_t ntiles, Ctrl* ctrl) {
    __shared__ uint64_t sa[kScanTop], sb[kScanTop];
    const uint64_t per = (ntiles + kScanTop - 1) / kScanTop;
    const uint64_t lo = (uint64_t)threadIdx.x * per;
    uint64_t a = 0, b = 0;
    for (uint64_t i = lo; i < lo + per && i < ntiles; ++i) {
        a += tile_cnt[i];
        b += tile_sq[i];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 partial sums
    for (int d = 1; d < kScanTop; d <<= 1) {
        uint64_t va = 0, vb = 0;
        if ((int)threadIdx.x >= d) {
            va = sa[threadIdx.x - d];
            vb = sb[threadIdx.x - d];
        }
        __syncthreads();
        sa[threadIdx.x] += va;
        sb[threadIdx.x] += vb;
        __syncthreads();
    }
    uint64_t pa = sa[threadIdx.x] - a, pb = sb[threadIdx.x] - b;
    for (uint64_t i = lo; i < lo + per && i < ntiles; ++i) {
        uint64_t ca = tile_cnt[i], cb = tile_sq[i];
        tile_cnt[i] = pa;
        tile_sq[i] = pb;
        pa += ca;
        pb += cb;
    }
    if (threadIdx.x == kScanTop - 1) ctrl->S = sb[kScanTop - 1];
}

// per group: (where its keys start, where its cells start), both exclusive
__global__ __launch_bounds__(kBlock) void k_scan_down(const uint32_t* __restrict__ sizes, uint64_t G,
                                                        const uint64_t* __restrict__ tile_cnt,
                                                        const uint64_t* __restrict__ tile_sq,
                                                        uint2* __restrict__ gscan) {
    const uint64_t g0 = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t sz[kScanItems];
    uint32_t cnt = 0, sq = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint64_t g = g0 + k;
        sz[k] = g < G ? sizes[g] : 0u;
        uint32_t c, q;
        group_stats(sz[k], c, q);
        cnt += c;
        sq += q;
    }
    uint32_t ta, tb;
    block_exscan2(cnt, sq, ta, tb);
    uint32_t pc = (uint32_t)tile_cnt[blockIdx.x] + cnt;
    uint32_t pq = (uint32_t)tile_sq[blockIdx.x] + sq;   // meaningful only when S < 2^32
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint64_t g = g0 + k;
        if (g < G) gscan[g] = make_uint2(pc, pq);
        uint32_t c, q;
        group_stats(sz[k], c, q);
        pc += c;
        pq += q;
    }
}

// ---- step 3: group keys by bucket ---------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_group(const uint64_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ vals,
                                                    const uint8_t* __restrict__ rank, uint64_t n,
                                                    Triple A, uint64_t magic,
                                                    const uint32_t* __restrict__ sizes,
                                                    const uint2* __restrict__ gscan,
                                                    Cell* __restrict__ grouped, int aux_is_index) {
    const uint64_t i0 = (uint64_t)blockIdx.x * (kBlock * kHistItems) + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kHistItems; ++k) {
        uint64_t i = i0 + (uint64_t)k * kBlock;
        if (i < n) {
            uint64_t x = keys[i];
            uint32_t j = fastmod(mshash(A, x), magic, (uint32_t)n);
            uint32_t g = j >> 3, kk = j & 7u;
            uint32_t pos = gscan[g].x + prefix_cnt(sizes[g], kk) + rank[i];
            Cell c;
            c.key = x;
            c.val = vals[i];
            c.aux = aux_is_index ? (uint32_t)i : 0u;
            grouped[pos] = c;
        }
    }
}

// ---- steps 4+5: level-two search and table write ------------------------------------------

__device__ inline bool bit_test_set(uint64_t& m0, uint64_t& m1, uint64_t& m2, uint64_t& m3, uint32_t h) {
    uint64_t bit = 1ull << (h & 63u);
    uint32_t w = h >> 6;
    uint64_t cur = w == 0 ? m0 : w == 1 ? m1 : w == 2 ? m2 : m3;
    if (cur & bit) return true;
    if (w == 0) m0 |= bit;
    else if (w == 1) m1 |= bit;
    else if (w == 2) m2 |= bit;
    else m3 |= bit;
    return false;
}

// smallest trial whose hashes mod s^2 are distinct on the bucket; T if none
template <typename KeyAt>
__device__ inline uint32_t search_bucket(const Triple* C, uint32_t T, uint32_t s, KeyAt key_at) {
    const uint32_t s2 = s * s;
    for (uint32_t t = 0; t < T; ++t) {
        const Triple c = C[t];
        uint64_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
        bool collide = false;
        for (uint32_t i = 0; i < s; ++i) {
            uint32_t h = mshash(c, key_at(i)) % s2;
            if (bit_test_set(m0, m1, m2, m3, h)) {
                collide = true;
                break;
            }
        }
        if (!collide) return t;
    }
    return T;
}

__device__ inline bool strings_equal(const int64_t* off, const uint8_t* bytes, uint32_t a, uint32_t b) {
    int64_t la = off[a + 1] - off[a], lb = off[b + 1] - off[b];
    if (la != lb) return false;
    const uint8_t* pa = bytes + off[a];
    const uint8_t* pb = bytes + off[b];
    for (int64_t q = 0; q < la; ++q)
        if (pa[q] != pb[q]) return false;
    return true;
}

template <bool BYTES>
__global__ __launch_bounds__(kBlock) void k_search_write(
    const Cell* __restrict__ grouped, uint64_t n, uint64_t G, uint64_t S,
    const uint32_t* __restrict__ sizes, const uint2* __restrict__ gscan,
    const Triple* __restrict__ Cg, uint32_t T, Group* __restrict__ header,
    Cell* __restrict__ slots, Ctrl* ctrl, const int64_t* __restrict__ ctx_off,
    const uint8_t* __restrict__ ctx_bytes) {
    __shared__ Triple C[kTMax];
    __shared__ Cell ent[kKeyCap];
    __shared__ uint16_t smap[kCellCap];
    __shared__ uint32_t tsh[kBlock / 4];
    __shared__ uint32_t rng[4];
    __shared__ uint32_t blk_max_t;

    const uint32_t tid = threadIdx.x;
    for (uint32_t t = tid; t < T; t += kBlock) C[t] = Cg[t];
    if (tid == 0) blk_max_t = 0;

    const uint64_t j = (uint64_t)blockIdx.x * kBlock + tid;
    const uint64_t g = j >> 3;
    const uint32_t k = (uint32_t)(j & 7u);
    uint32_t s = 0, kst, off;
    if (g < G) {
        const uint32_t sz = sizes[g];
        const uint2 gs = gscan[g];
        s = nib(sz, k);
        kst = gs.x + prefix_cnt(sz, k);
        off = gs.y + prefix_sq(sz, k);
    } else {
        kst = (uint32_t)n;
        off = (uint32_t)S;
    }
    if (tid == 0) {
        rng[0] = kst;
        rng[2] = off;
    }
    if (tid == kBlock - 1) {
        rng[1] = kst + s;
        rng[3] = off + s * s;
    }
    __syncthreads();
    const uint32_t K0 = rng[0], K1 = rng[1], Z0 = rng[2], Z1 = rng[3];
    const bool fast = (K1 - K0 <= kKeyCap) && (Z1 - Z0 <= kCellCap);

    uint32_t t = 0;
    bool exhausted = false;
    if (fast) {
        for (uint32_t p = tid; p < K1 - K0; p += kBlock) ent[p] = grouped[K0 + p];
        __syncthreads();
        const uint32_t lk = kst - K0;
        if (s >= 2) {
            t = search_bucket(C, T, s, [&](uint32_t i) { return ent[lk + i].key; });
            exhausted = (t == T);
        }
        const uint32_t lz = off - Z0, s2 = s * s;
        if (s >= 1) {
            if (!exhausted) {
                for (uint32_t p = 0; p < s2; ++p) smap[lz + p] = 0xFFFFu;
                const Triple c = C[t];
                for (uint32_t i = 0; i < s; ++i) smap[lz + mshash(c, ent[lk + i].key) % s2] = (uint16_t)(lk + i);
                uint16_t first = 0;
                for (uint32_t p = 0; p < s2; ++p)
                    if (smap[lz + p] != 0xFFFFu) {
                        first = smap[lz + p];
                        break;
                    }
                for (uint32_t p = 0; p < s2; ++p)
                    if (smap[lz + p] == 0xFFFFu) smap[lz + p] = first;
            } else {
                for (uint32_t p = 0; p < s2; ++p) smap[lz + p] = (uint16_t)lk;
            }
        }
        if (exhausted) {
            bool dup = false;
            for (uint32_t a = 0; a < s; ++a)
                for (uint32_t b = a + 1; b < s; ++b) {
                    if (BYTES)
                        dup |= strings_equal(ctx_off, ctx_bytes, ent[lk + a].aux, ent[lk + b].aux);
                    else
                        dup |= ent[lk + a].key == ent[lk + b].key;
                }
            atomicOr(&ctrl->exhausted, 1u);
            if (dup) atomicOr(&ctrl->dup, 1u);
        }
        __syncthreads();
        for (uint32_t p = tid; p < Z1 - Z0; p += kBlock) slots[Z0 + p] = ent[smap[p]];
    } else {
        // rare: the block's keys or cells do not fit the LDS staging; work from HBM
        const Cell* bk = grouped + kst;
        if (s >= 2) {
            t = search_bucket(C, T, s, [&](uint32_t i) { return bk[i].key; });
            exhausted = (t == T);
        }
        const uint32_t s2 = s * s;
        if (s >= 1 && !exhausted) {
            const Triple c = C[t];
            uint32_t first_p = s2, first_i = 0;
            for (uint32_t i = 0; i < s; ++i) {
                uint32_t h = mshash(c, bk[i].key) % s2;
                if (h < first_p) {
                    first_p = h;
                    first_i = i;
                }
            }
            for (uint32_t p = 0; p < s2; ++p) {
                uint32_t who = first_i;
                for (uint32_t i = 0; i < s; ++i)
                    if (mshash(c, bk[i].key) % s2 == p) who = i;
                slots[off + p] = bk[who];
            }
        }
        if (exhausted) {
            bool dup = false;
            for (uint32_t a = 0; a < s; ++a)
                for (uint32_t b = a + 1; b < s; ++b) {
                    if (BYTES)
                        dup |= strings_equal(ctx_off, ctx_bytes, bk[a].aux, bk[b].aux);
                    else
                        dup |= bk[a].key == bk[b].key;
                }
            atomicOr(&ctrl->exhausted, 1u);
            if (dup) atomicOr(&ctrl->dup, 1u);
        }
    }
    // trial indices of the block's buckets, one byte each
    if (exhausted) t = 0;
    if (t) atomicMax(&blk_max_t, t);
    reinterpret_cast<uint8_t*>(tsh)[tid] = (uint8_t)t;
    __syncthreads();
    if (tid < kBlock / 8) {
        const uint64_t gg = (uint64_t)blockIdx.x * (kBlock / 8) + tid;
        if (gg < G) {
            Group h;
            h.base = gscan[gg].y;
            h.sizes = sizes[gg];
            h.t_lo = tsh[2 * tid];
            h.t_hi = tsh[2 * tid + 1];
            header[gg] = h;
        }
    }
    if (tid == 0 && blk_max_t) atomicMax(&ctrl->max_t, blk_max_t);
}

__global__ void k_rebase_offsets(const int64_t* __restrict__ in, int64_t* __restrict__ out, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

// ---- host driver ------------------------------------------------------------------------

static unsigned grid_for(uint64_t items, uint64_t per_block, unsigned cap = 1u << 30) {
    uint64_t g = (items + per_block - 1) / per_block;
    if (g == 0) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

struct Scratch {
    uint32_t* sizes = nullptr;
    uint8_t* rank = nullptr;
    uint2* gscan = nullptr;
    uint64_t* tiles = nullptr;   // 2 * ntiles
    Cell* grouped = nullptr;
    uint64_t* y = nullptr;       // fingerprints (string maps)
    Ctrl* ctrl = nullptr;
    Readback* host = nullptr;    // pinned
};

static void free_scratch(Scratch& w, hipStream_t st) {
    dev_free(w.sizes, st);
    dev_free(w.rank, st);
    dev_free(w.gscan, st);
    dev_free(w.tiles, st);
    dev_free(w.grouped, st);
    dev_free(w.y, st);
    dev_free(w.ctrl, st);
    w = Scratch{};
}

// one pinned readback buffer per host thread, kept for the life of the process
static Readback* pinned_readback() {
    static thread_local Readback* buf = nullptr;
    if (!buf) {
        if (hipHostMalloc((void**)&buf, sizeof(Readback), hipHostMallocDefault) != hipSuccess) buf = nullptr;
    }
    return buf;
}

static int check_params(uint64_t n, const fks_params* p, fks_params& out) {
    fks_params_default(&out);
    if (p) out = *p;
    if (n >= (1ull << 30)) return FKS_EINVAL;
    if (out.c < 1 || out.c > 16 || out.T < 1 || out.T > kTMax || out.R < 1 || out.R > 1024 ||
        out.schedule > 1)
        return FKS_EINVAL;
    if ((uint64_t)out.c * n >= (1ull << 32)) return FKS_EINVAL;
    return FKS_OK;
}

static int read_ctrl(Scratch& w, hipStream_t st) {
    FKS_HIP(hipMemcpyAsync(w.host, w.ctrl, sizeof(Readback), hipMemcpyDeviceToHost, st));
    FKS_HIP(hipStreamSynchronize(st));
    return FKS_OK;
}

static bool legacy_build() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("FKS_BUILD_LEGACY");
        v = (e && e[0] == '1') ? 1 : 0;
    }
    return v == 1;
}

// Level-one attempts with the partitioned passes (partition.hip).
static int attempts_partitioned(fks_map* M, const uint64_t* d_keys_in, const uint32_t* d_vals,
                                const fks_params& P, Ctrl* ctrl, Readback* host, uint64_t* y, hipStream_t st) {
    const uint64_t n = M->n;
    const uint64_t G = (n + 7) / 8;
    const bool bytes = M->kind == 1;
    const PartPlan plan = part_plan(n);
    const uint32_t Q = plan.Q;
    PartArgs a{};
    a.n = n;
    a.G = G;
    a.bytes = bytes;
    a.vals = d_vals;
    // scratch, freed when the attempts are over
    std::vector<void*> owned;
    auto grab = [&](size_t bytes_) {
        void* p = dev_alloc(bytes_, st);
        owned.push_back(p);
        return p;
    };
    auto release = [&]() {
        for (void* p : owned) dev_free(p, st);
        owned.clear();
    };
    if (plan.passes >= 2) {
        a.k1 = (uint64_t*)grab(8 * n);
        a.v1 = (uint32_t*)grab(4 * n);
        if (bytes) a.a1 = (uint32_t*)grab(4 * n);
    }
    if (plan.passes >= 1) {
        a.k2 = (uint64_t*)grab(8 * n);
        a.v2 = (uint32_t*)grab(4 * n);
        if (bytes) a.a2 = (uint32_t*)grab(4 * n);
    }
    a.cnt = (uint32_t*)grab(4 * plan.matrix);
    a.off = (uint32_t*)grab(4 * plan.matrix);
    a.tsum = (uint32_t*)grab(4 * part_scan_tiles(plan));
    a.tpre = (uint64_t*)grab(8 * (part_scan_tiles(plan) + 1));
    a.offA = (uint64_t*)grab(8 * 257);
    a.offQ = (uint64_t*)grab(8 * ((size_t)Q + 1));
    a.sqQ = (uint32_t*)grab(4 * (size_t)Q);
    a.cbase = (uint64_t*)grab(8 * ((size_t)Q + 1));
    a.sizes = (uint32_t*)grab(4 * (size_t)Q * (kPartBuckets / 8));
    a.S_dev = &ctrl->S;
    a.oversize = &ctrl->oversize;
    for (void* p : owned)
        if (!p) {
            release();
            return FKS_ENOMEM;
        }
    Triple Ch[kTMax];
    int rc = FKS_OK;
    for (uint32_t r = 0; r < P.R; ++r) {
        const Triple A = level1_triple(M->seed, r);
        const uint64_t beta = level1_beta(M->seed, r);
        a.A = A;
        a.magic = M->magic_n;
        a.keys = d_keys_in;
        if (bytes) {
            FKS_TIMED("fks_fingerprint", st,
                      hipLaunchKernelGGL(k_fingerprint, grid_for(n, kBlock, 65536), kBlock, 0, st, M->ctx_off,
                                         M->ctx_bytes, n, beta, y));
            a.keys = y;
        }
        hipLaunchKernelGGL(k_zero_ctrl, 1, 64, 0, st, ctrl);
        PartOut o;
        if ((rc = part_prepare(a, st, o))) break;
        FKS_HIP(hipMemcpyAsync(host, ctrl, sizeof(Readback), hipMemcpyDeviceToHost, st));
        FKS_HIP(hipStreamSynchronize(st));
        if (host->oversize) continue;
        const uint64_t S = host->S;
        if (S > (uint64_t)P.c * n) continue;
        for (uint32_t t = 0; t < P.T; ++t) Ch[t] = level2_triple(M->seed, r, t);
        FKS_HIP(hipMemcpyAsync(M->C, Ch, sizeof(Triple) * P.T, hipMemcpyHostToDevice, st));
        Cell* slots = (Cell*)dev_alloc(16 * (S ? S : 1), st);
        if (!slots) {
            rc = FKS_ENOMEM;
            break;
        }
        const uint8_t* given_t = nullptr;
        if (P.schedule == 1) {
            // the paper's flattened rounds decide every bucket's trial; the table
            // write below then only places the keys
            uint8_t* tb = (uint8_t*)dev_alloc(4 * ((n + 3) / 4), st);
            if (!tb) {
                dev_free(slots, st);
                rc = FKS_ENOMEM;
                break;
            }
            owned.push_back(tb);
            hipLaunchKernelGGL(k_fill_u32, grid_for((n + 3) / 4, kBlock, 8192), kBlock, 0, st, (uint32_t*)tb,
                               (n + 3) / 4, 0u);
            bool exhausted = false;
            rc = rounds_search(o.keys, n, S, A, M->magic_n, a.sizes, Ch, P.T, tb, &exhausted, st);
            if (rc) {
                dev_free(slots, st);
                break;
            }
            // a bucket left after T rounds goes through the per-bucket search, which
            // reports the exhaustion (and any duplicate keys) exactly as it would alone
            if (!exhausted) given_t = tb;
        }
        rc = part_finish(a, o, M->C, P.T, M->header, slots, &ctrl->exhausted, M->ctx_off, M->ctx_bytes, given_t, st);
        if (rc == FKS_OK) {
            hipError_t e = hipMemcpyAsync(host, ctrl, sizeof(Readback), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) rc = hip_fail(e);
        }
        if (rc) {
            dev_free(slots, st);
            break;
        }
        if (host->exhausted) {
            dev_free(slots, st);
            if (host->dup) {
                rc = FKS_EDUPKEY;
                break;
            }
            continue;
        }
        M->slots = slots;
        M->S = S;
        M->r = r;
        M->A = A;
        M->beta = beta;
        M->max_t = host->max_t;
        M->device_bytes += 16 * S;
        release();
        return FKS_OK;
    }
    release();
    return rc ? rc : FKS_EBUILD;
}

// keys: device u64 keys (or fingerprints); vals; aux_is_index for string maps
static int build_common(fks_map* M, const uint64_t* d_keys_in, const uint32_t* d_vals,
                        const int64_t* d_off, const uint8_t* d_bytes, uint64_t nbytes,
                        const fks_params& P, hipStream_t st) {
    const uint64_t n = M->n;
    const uint64_t G = (n + 7) / 8;
    const bool bytes = M->kind == 1;
    const uint64_t ntiles = (G + kScanTile - 1) / kScanTile;
    Scratch w;
    int rc = FKS_OK;
    auto fail = [&](int code) {
        free_scratch(w, st);
        return code;
    };
    const bool legacy = legacy_build();
    if (legacy) {
        w.sizes = (uint32_t*)dev_alloc(4 * G, st);
        w.rank = (uint8_t*)dev_alloc(n, st);
        w.gscan = (uint2*)dev_alloc(8 * G, st);
        w.tiles = (uint64_t*)dev_alloc(16 * ntiles, st);
        w.grouped = (Cell*)dev_alloc(16 * n, st);
        if (!w.sizes || !w.rank || !w.gscan || !w.tiles || !w.grouped) return fail(FKS_ENOMEM);
    }
    w.ctrl = (Ctrl*)dev_alloc(sizeof(Ctrl), st);
    if (bytes) w.y = (uint64_t*)dev_alloc(8 * n, st);
    if (!w.ctrl || (bytes && !w.y)) return fail(FKS_ENOMEM);
    w.host = pinned_readback();
    if (!w.host) return fail(FKS_ENOMEM);
    M->header = (Group*)dev_alloc(16 * G, st);
    M->C = (Triple*)dev_alloc(sizeof(Triple) * P.T, st);
    if (!M->header || !M->C) return fail(FKS_ENOMEM);
    M->device_bytes = 16 * G + sizeof(Triple) * P.T;

    if (bytes) {
        // the map keeps its own copy of the context (Section 3.1)
        M->ctx_off = (int64_t*)dev_alloc(8 * (n + 1), st);
        M->ctx_bytes = (uint8_t*)dev_alloc(nbytes ? nbytes : 1, st);
        if (!M->ctx_off || !M->ctx_bytes) return fail(FKS_ENOMEM);
        M->ctx_nbytes = nbytes;
        M->device_bytes += 8 * (n + 1) + nbytes;
        hipLaunchKernelGGL(k_zero_ctrl, 1, 64, 0, st, w.ctrl);
        hipLaunchKernelGGL(k_check_offsets, grid_for(n + 1, kBlock, 4096), kBlock, 0, st, d_off, n, nbytes, w.ctrl);
        if ((rc = read_ctrl(w, st))) return fail(rc);
        if (w.host->bad_input) return fail(FKS_EINVAL);
        FKS_HIP(hipMemcpyAsync(M->ctx_off, d_off, 8 * (n + 1), hipMemcpyDeviceToDevice, st));
        if (nbytes) FKS_HIP(hipMemcpyAsync(M->ctx_bytes, d_bytes, nbytes, hipMemcpyDeviceToDevice, st));
    }

    Triple Ch[kTMax];
    const uint64_t magic = fastmod_magic((uint32_t)n);
    M->magic_n = magic;
    if (!legacy_build()) {
        rc = attempts_partitioned(M, d_keys_in, d_vals, P, w.ctrl, w.host, w.y, st);
        free_scratch(w, st);
        return rc;
    }
    for (uint32_t r = 0; r < P.R; ++r) {
        const Triple A = level1_triple(M->seed, r);
        const uint64_t beta = level1_beta(M->seed, r);
        const uint64_t* keys = d_keys_in;
        if (bytes) {
            FKS_TIMED("fks_fingerprint", st, hipLaunchKernelGGL(k_fingerprint, grid_for(n, kBlock, 65536), kBlock, 0, st, M->ctx_off,
                               M->ctx_bytes, n, beta, w.y));
            keys = w.y;
        }
        hipLaunchKernelGGL(k_zero_ctrl, 1, 64, 0, st, w.ctrl);
        FKS_TIMED("fks_zero_counts", st, hipLaunchKernelGGL(k_fill_u32, grid_for(G, kBlock, 8192), kBlock, 0, st, w.sizes, G, 0u));
        FKS_TIMED("fks_hist", st, hipLaunchKernelGGL(k_hist, grid_for(n, kBlock * kHistItems), kBlock, 0, st, keys, n, A, magic,
                           w.sizes, w.rank, w.ctrl));
        FKS_TIMED("fks_scan_reduce", st, hipLaunchKernelGGL(k_scan_reduce, (unsigned)ntiles, kBlock, 0, st, w.sizes, G, w.tiles, w.tiles + ntiles));
        FKS_TIMED("fks_scan_tiles", st, hipLaunchKernelGGL(k_scan_tiles, 1, kScanTop, 0, st, w.tiles, w.tiles + ntiles, ntiles, w.ctrl));
        FKS_TIMED("fks_scan_down", st, hipLaunchKernelGGL(k_scan_down, (unsigned)ntiles, kBlock, 0, st, w.sizes, G, w.tiles, w.tiles + ntiles,
                           w.gscan));
        FKS_HIP(hipGetLastError());
        if ((rc = read_ctrl(w, st))) return fail(rc);
        if (w.host->oversize) continue;
        const uint64_t S = w.host->S;
        if (S > (uint64_t)P.c * n) continue;

        for (uint32_t t = 0; t < P.T; ++t) Ch[t] = level2_triple(M->seed, r, t);
        FKS_HIP(hipMemcpyAsync(M->C, Ch, sizeof(Triple) * P.T, hipMemcpyHostToDevice, st));
        Cell* slots = (Cell*)dev_alloc(16 * S, st);
        if (!slots) return fail(FKS_ENOMEM);
        FKS_TIMED("fks_group", st, hipLaunchKernelGGL(k_group, grid_for(n, kBlock * kHistItems), kBlock, 0, st, keys, d_vals, w.rank, n, A,
                           magic, w.sizes, w.gscan, w.grouped, bytes ? 1 : 0));
        if (bytes)
            FKS_TIMED("fks_search_write", st, hipLaunchKernelGGL(k_search_write<true>, grid_for(n, kBlock), kBlock, 0, st, w.grouped, n, G, S,
                               w.sizes, w.gscan, M->C, P.T, M->header, slots, w.ctrl, M->ctx_off,
                               M->ctx_bytes));
        else
            FKS_TIMED("fks_search_write", st, hipLaunchKernelGGL(k_search_write<false>, grid_for(n, kBlock), kBlock, 0, st, w.grouped, n, G, S,
                               w.sizes, w.gscan, M->C, P.T, M->header, slots, w.ctrl, nullptr, nullptr));
        {
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) {
                dev_free(slots, st);
                return fail(hip_fail(e));
            }
        }
        if ((rc = read_ctrl(w, st))) {
            dev_free(slots, st);
            return fail(rc);
        }
        if (w.host->exhausted) {
            dev_free(slots, st);
            if (w.host->dup) return fail(FKS_EDUPKEY);
            continue;
        }
        M->slots = slots;
        M->S = S;
        M->r = r;
        M->A = A;
        M->beta = beta;
        M->max_t = w.host->max_t;
        M->device_bytes += 16 * S;
        free_scratch(w, st);
        return FKS_OK;
    }
    return fail(FKS_EBUILD);
}

static void release_partial(fks_map* M, hipStream_t st) {
    dev_free(M->header, st);
    dev_free(M->slots, st);
    dev_free(M->C, st);
    dev_free(M->ctx_off, st);
    dev_free(M->ctx_bytes, st);
    delete M;
}

static fks_map* new_map(uint32_t kind, uint64_t n, uint64_t seed, const fks_params& P) {
    fks_map* M = new fks_map;
    std::memset(M, 0, sizeof(*M));
    M->kind = kind;
    M->n = n;
    M->seed = seed;
    M->c = P.c;
    M->T = P.T;
    M->R = P.R;
    (void)hipGetDevice(&M->device);
    return M;
}

static int build_empty(fks_map* M, const fks_params& P, hipStream_t st) {
    // n = 0: no buckets and no cells; every lookup is absent
    Triple Ch[kTMax];
    M->A = level1_triple(M->seed, 0);
    M->beta = level1_beta(M->seed, 0);
    M->C = (Triple*)dev_alloc(sizeof(Triple) * P.T, st);
    if (!M->C) return FKS_ENOMEM;
    for (uint32_t t = 0; t < P.T; ++t) Ch[t] = level2_triple(M->seed, 0, t);
    FKS_HIP(hipMemcpyAsync(M->C, Ch, sizeof(Triple) * P.T, hipMemcpyHostToDevice, st));
    FKS_HIP(hipStreamSynchronize(st));
    M->device_bytes = sizeof(Triple) * P.T;
    return FKS_OK;
}

}  // namespace fks

extern "C" int fks_build_u64(const uint64_t* d_keys, const uint32_t* d_vals, uint64_t n, uint64_t seed,
                             const fks_params* params, void* stream, fks_map** out) {
    using namespace fks;
    if (!out || (n && (!d_keys || !d_vals))) return FKS_EINVAL;
    fks_params P;
    int rc = check_params(n, params, P);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    fks_map* M = new_map(0, n, seed, P);
    rc = n ? build_common(M, d_keys, d_vals, nullptr, nullptr, 0, P, st) : build_empty(M, P, st);
    if (rc) {
        release_partial(M, st);
        return rc;
    }
    *out = M;
    return FKS_OK;
}

extern "C" int fks_build_bytes(const int64_t* d_offsets, const uint8_t* d_bytes, uint64_t nbytes,
                               const uint32_t* d_vals, uint64_t n, uint64_t seed, const fks_params* params,
                               void* stream, fks_map** out) {
    using namespace fks;
    if (!out || !d_offsets || (n && !d_vals) || (nbytes && !d_bytes)) return FKS_EINVAL;
    fks_params P;
    int rc = check_params(n, params, P);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    fks_map* M = new_map(1, n, seed, P);
    if (n) {
        rc = build_common(M, nullptr, d_vals, d_offsets, d_bytes, nbytes, P, st);
    } else {
        // keep a copy of the (empty) context too
        rc = build_empty(M, P, st);
        if (!rc) {
            M->ctx_off = (int64_t*)dev_alloc(8, st);
            M->ctx_bytes = (uint8_t*)dev_alloc(nbytes ? nbytes : 1, st);
            if (!M->ctx_off || !M->ctx_bytes) rc = FKS_ENOMEM;
            else {
                hipError_t e = hipMemcpyAsync(M->ctx_off, d_offsets, 8, hipMemcpyDeviceToDevice, st);
                if (e == hipSuccess && nbytes) e = hipMemcpyAsync(M->ctx_bytes, d_bytes, nbytes, hipMemcpyDeviceToDevice, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e != hipSuccess) rc = hip_fail(e);
                M->ctx_nbytes = nbytes;
            }
        }
    }
    if (rc) {
        release_partial(M, st);
        return rc;
    }
    *out = M;
    return FKS_OK;
}
