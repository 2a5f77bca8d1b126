// Partitioned construction: the level-one attempt as a few streaming passes.
//
// Buckets are cut into partitions of 1024 consecutive buckets (q = j >> 10).  Keys are
// moved into partition order by one to three coalescing radix passes over q (at most 8
// bits, 256 bins, per pass, so every 12288-record tile writes runs of about 48 records per
// bin); each worker's runs go to offsets from a scanned count matrix, or are reserved with
// one atomic add per (tile, bin) on a cursor into a fixed-capacity region.  Then every
// partition is finished by one workgroup that holds its ~1024 keys in LDS: ranks from an
// LDS histogram, scan of the 128 group statistics, grouping, the per-bucket level-two
// search of make_2, and the coalesced write of the partition's contiguous cells and group
// headers.  Only the partition totals of squared sizes (the offsets of Section 2.2, at
// partition granularity) cross partitions: either a size pass and a scan turn them into
// cell bases and the table size S, or the final pass publishes each total and finds its
// own base by a look-back over its predecessors'.  Device-scope atomics serve only the
// cursors, the final pass's tickets and look-back words, and an attempt's outcome flags;
// every per-key access is a coalesced stream or LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fks_internal.hpp"
#include "partition.hpp"
#include "prof.hpp"

namespace fks {

constexpr uint32_t kPB = 256;                 // threads per block, partition passes
constexpr uint32_t kPItems = 16;              // keys per thread per tile
constexpr uint32_t kPTile = kPB * kPItems;    // 4096 keys per tile
// scatter tiles of the single-map passes: 1024 threads x 12 records (12288 records, runs of ~48
// per bin, 149 KB of LDS: one workgroup and four waves per SIMD on a CU), or x 8 when an aux
// word travels (16-byte records, 8192-record tiles, 133 KB)
constexpr uint32_t kPScatterThreads = 1024, kPScatterItems = 12, kPScatterItemsAux = 8;
constexpr uint64_t kWorkerKeys = 2ull * kPScatterThreads * kPScatterItems;   // keys per scatter worker: two tiles
constexpr uint32_t kBins = 256;               // bins per scatter pass
constexpr uint32_t kFinalKeyCap = 1248;       // keys of one partition held in LDS (mean 1024, sd 32)
constexpr uint32_t kLdsTrials = 16;          // level-two triples held in the final pass's LDS (larger trials are rare)
constexpr uint32_t kFinalCellCap = 3072;      // cells of one partition staged in LDS (mean <= 2048, sd ~106)
constexpr uint32_t kGroupsPerPart = kPartBuckets / 8;

__global__ void k_zero_words(uint32_t* __restrict__ p, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_set_range(uint64_t* off, uint64_t n) {
    if (threadIdx.x == 0) {
        off[0] = 0;
        off[1] = n;
    }
}

__device__ __forceinline__ uint32_t bucket_of(const Triple& A, uint64_t magic, uint32_t n, uint64_t x) {
    return fastmod(mshash(A, x), magic, n);
}

// Worker blockIdx.x of W in segment blockIdx.y: segment = the whole input
// (ranges == nullptr) or [ranges[s], ranges[s+1]); the worker owns one
// contiguous chunk of it and walks the chunk in tiles, so that counting and
// scattering see the keys in the same order.
__device__ __forceinline__ void worker_range(const uint64_t* ranges, uint64_t n, uint32_t W, uint64_t& a,
                                             uint64_t& b, const WideSeg* segs = nullptr,
                                             const uint64_t* ranges_hi = nullptr, uint64_t hi_cap = 0) {
    uint64_t lo = 0, hi = n;
    if (segs) {
        lo = segs[blockIdx.y].in_lo;
        hi = segs[blockIdx.y].in_hi;
    } else if (ranges) {
        lo = ranges[blockIdx.y];
        // a cursor that ran past its region's end (overflow raised) stops at the end
        hi = ranges_hi ? min(ranges_hi[blockIdx.y], lo + hi_cap) : ranges[blockIdx.y + 1];
    }
    const uint64_t chunk = (hi - lo + W - 1) / W;
    a = min(hi, lo + (uint64_t)blockIdx.x * chunk);
    b = min(hi, a + chunk);
}

// counts of one worker per bin: cnt[(segment * 256 + bin) * W + worker]
// (segs: segment blockIdx.y is a wide map of a batch, with its own keys and hash)
__global__ __launch_bounds__(kPB) void k_dcount(const uint64_t* __restrict__ keys, uint64_t n, Triple A,
                                                  uint64_t magic, const uint64_t* __restrict__ ranges, uint32_t W,
                                                  uint32_t shift, uint32_t mask, uint32_t* __restrict__ cnt,
                                                  const WideSeg* __restrict__ segs = nullptr) {
    __shared__ uint32_t bins[kBins];
    uint64_t a, b;
    worker_range(ranges, n, W, a, b, segs);
    if (segs) {
        A = segs[blockIdx.y].A;
        magic = segs[blockIdx.y].magic;
        n = segs[blockIdx.y].n;
    }
    for (uint32_t k = threadIdx.x; k < kBins; k += kPB) bins[k] = 0;
    __syncthreads();
    for (uint64_t ts = a; ts < b; ts += kPTile) {
        uint64_t x[kPItems];
#pragma unroll
        for (uint32_t k = 0; k < kPItems; ++k) {
            const uint64_t i = ts + threadIdx.x + (uint64_t)k * kPB;
            x[k] = i < b ? keys[i] : 0;
        }
#pragma unroll
        for (uint32_t k = 0; k < kPItems; ++k) {
            const uint64_t i = ts + threadIdx.x + (uint64_t)k * kPB;
            if (i < b) {
                const uint32_t q = bucket_of(A, magic, (uint32_t)n, x[k]) >> kPartBits;
                atomicAdd(&bins[(q >> shift) & mask], 1u);
            }
        }
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < kBins; k += kPB)
        cnt[((uint64_t)blockIdx.y * kBins + k) * W + blockIdx.x] = bins[k];
}

// exclusive scan of 256 per-thread values across the block (one value per thread)
__device__ __forceinline__ uint32_t block_exscan256(uint32_t v, uint32_t* wsum) {
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
    for (int q = 0; q < w; ++q) pre += wsum[q];
    __syncthreads();
    return pre + inc - v;
}

// Scatter of one worker's chunk: every tile is sorted by bin in LDS, then each
// bin's run is written to consecutive addresses from the worker's scanned
// offset (no device atomics; the output order is a function of the input).
// BT threads per block (at least one per bin), ITEMS records per thread per tile
// CURSOR: instead of offsets from a count matrix, every tile reserves each bin's run with
// one atomic add on the bin's cursor (bins are fixed-capacity regions: bin i of segment s
// owns [(s * (mask + 1) + i) * cap, ... + cap)); records that would land beyond their
// region are dropped and *overflow is raised, so the attempt can be redone with counts.
// Segment s reads [ranges[s], ranges_hi[s]).  The order of records inside a bin then
// depends on timing, which the final pass does not see: its table depends only on which
// records each partition holds.
template <bool AUX, uint32_t ITEMS, uint32_t BT = kPB, bool CURSOR = false>
__global__ __launch_bounds__(BT) void k_dscatter(const uint64_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ vals,
                                                    const uint32_t* __restrict__ aux, uint64_t n, Triple A,
                                                    uint64_t magic, const uint64_t* __restrict__ ranges, uint32_t W,
                                                    uint32_t shift, uint32_t mask, const uint32_t* __restrict__ off,
                                                    uint64_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                                                    uint32_t* __restrict__ aux_out,
                                                    const WideSeg* __restrict__ segs = nullptr,
                                                    unsigned long long* __restrict__ cursor = nullptr,
                                                    const uint64_t* __restrict__ ranges_hi = nullptr,
                                                    uint64_t cap = 0, uint32_t* __restrict__ overflow = nullptr,
                                                    uint64_t in_cap = 0) {
    __shared__ uint64_t skey[(BT * ITEMS)];
    __shared__ uint32_t sval[(BT * ITEMS)];
    __shared__ uint32_t saux[AUX ? (BT * ITEMS) : 1];
    __shared__ uint32_t run[kBins], tcnt[kBins], toff[kBins];
    __shared__ uint32_t wsum[BT / 64];
    static_assert(BT >= kBins && BT % 64 == 0, "one bin per thread");
    __shared__ uint64_t lim[CURSOR ? kBins : 1];
    uint64_t a, b;
    worker_range(ranges, n, W, a, b, segs, ranges_hi, in_cap);
    if (segs) {
        A = segs[blockIdx.y].A;
        magic = segs[blockIdx.y].magic;
        n = segs[blockIdx.y].n;
    }
    const uint32_t tid = threadIdx.x;
    if (!CURSOR && tid < kBins) run[tid] = off[((uint64_t)blockIdx.y * kBins + tid) * W + blockIdx.x];
    if (CURSOR && tid < kBins) lim[tid] = ((uint64_t)blockIdx.y * (mask + 1) + tid + 1) * cap;
    // a tile's records are loaded into registers one tile ahead: the loads of
    // tile i+1 are in flight while tile i is written out
    uint64_t x[ITEMS];
    uint32_t v[ITEMS], u[AUX ? ITEMS : 1];
    auto load = [&](uint64_t ts) {
#pragma unroll
        for (uint32_t k = 0; k < ITEMS; ++k) {
            const uint64_t i = ts + tid + (uint64_t)k * BT;
            x[k] = i < b ? keys[i] : 0;
            v[k] = i < b ? vals[i] : 0;
            if (AUX) u[AUX ? k : 0] = i < b ? (aux ? aux[i] : (uint32_t)i) : 0;
        }
    };
    if (a < b) load(a);
    for (uint64_t ts = a; ts < b; ts += (BT * ITEMS)) {
        if (tid < kBins) tcnt[tid] = 0;
        __syncthreads();
        uint32_t bin[ITEMS], rank[ITEMS];
#pragma unroll
        for (uint32_t k = 0; k < ITEMS; ++k) {
            const uint64_t i = ts + tid + (uint64_t)k * BT;
            if (i < b) {
                const uint32_t q = bucket_of(A, magic, (uint32_t)n, x[k]) >> kPartBits;
                bin[k] = (q >> shift) & mask;
                rank[k] = atomicAdd(&tcnt[bin[k]], 1u);
            }
        }
        __syncthreads();
        if (CURSOR && tid <= mask && tcnt[tid]) {
            // this tile's run of bin tid: reserved now, written after the tile is sorted
            const unsigned long long at =
                atomicAdd(&cursor[(uint64_t)blockIdx.y * (mask + 1) + tid], (unsigned long long)tcnt[tid]);
            run[tid] = (uint32_t)at;
            if (at + tcnt[tid] > lim[tid]) atomicOr(overflow, 1u);
        }
        {
            const uint32_t e = block_exscan256(tid < kBins ? tcnt[tid] : 0u, wsum);
            if (tid < kBins) toff[tid] = e;
        }
        __syncthreads();
#pragma unroll
        for (uint32_t k = 0; k < ITEMS; ++k) {
            const uint64_t i = ts + tid + (uint64_t)k * BT;
            if (i < b) {
                const uint32_t e = toff[bin[k]] + rank[k];
                skey[e] = x[k];
                sval[e] = v[k];
                if (AUX) saux[e] = u[AUX ? k : 0];
            }
        }
        if (ts + (BT * ITEMS) < b) load(ts + (BT * ITEMS));
        __syncthreads();
        const uint32_t cnt = (uint32_t)min((uint64_t)(BT * ITEMS), b - ts);
        for (uint32_t e = tid; e < cnt; e += BT) {
            // the bin is hashed again rather than staged in LDS: the pass waits on memory,
            // and a staged byte per record measured the same
            const uint32_t bb = ((bucket_of(A, magic, (uint32_t)n, skey[e]) >> kPartBits) >> shift) & mask;
            const uint64_t dest = (uint64_t)run[bb] + (e - toff[bb]);
            if (CURSOR && dest >= lim[bb]) continue;   // beyond the bin's region: dropped, overflow raised
            keys_out[dest] = skey[e];
            vals_out[dest] = sval[e];
            if (AUX) aux_out[dest] = saux[e];
        }
        __syncthreads();
        if (!CURSOR && tid < kBins) run[tid] += tcnt[tid];
    }
}

// the set-up of the cursor passes in one launch: the cursor of fixed-capacity region i of
// either pass starts at i * cap (begin[i] keeps that start), and the fused final pass's
// look-back words and ticket (zw words) start at zero
__global__ void k_init_cursors(unsigned long long* __restrict__ cur1, uint64_t* __restrict__ beg1, uint64_t count1,
                               uint64_t cap1, unsigned long long* __restrict__ cur2, uint64_t* __restrict__ beg2,
                               uint64_t count2, uint64_t cap2, uint32_t* __restrict__ zw, uint64_t nzw,
                               uint32_t* __restrict__ ticket) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count1 + count2 + nzw; i += stride) {
        if (i < count1) {
            cur1[i] = i * cap1;
            beg1[i] = i * cap1;
        } else if (i < count1 + count2) {
            const uint64_t j = i - count1;
            cur2[j] = j * cap2;
            beg2[j] = j * cap2;
        } else {
            zw[i - count1 - count2] = 0;
        }
    }
    if (ticket && blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0;
}


// ---- exclusive scan of a u32 array across blocks (values sum below 2^32) --------------------

constexpr uint32_t kXItems = 8;
constexpr uint32_t kXTile = kPB * kXItems;

__global__ __launch_bounds__(kPB) void k_xscan_reduce(const uint32_t* __restrict__ in, uint64_t N,
                                                        uint32_t* __restrict__ tsum) {
    __shared__ uint32_t wsum[kPB / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kXTile + (uint64_t)threadIdx.x * kXItems;
    uint32_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kXItems; ++k)
        if (base + k < N) s += in[base + k];
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t w = 0; w < kPB / 64; ++w) t += wsum[w];
        tsum[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kPB) void k_xscan_down(const uint32_t* __restrict__ in, uint64_t N,
                                                      const uint64_t* __restrict__ tpre, uint32_t* __restrict__ out) {
    __shared__ uint32_t wsum[kPB / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kXTile + (uint64_t)threadIdx.x * kXItems;
    uint32_t v[kXItems];
    uint32_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kXItems; ++k) {
        v[k] = base + k < N ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t run = (uint32_t)tpre[blockIdx.x] + block_exscan256(s, wsum);
#pragma unroll
    for (uint32_t k = 0; k < kXItems; ++k) {
        if (base + k < N) out[base + k] = run;
        run += v[k];
    }
}

// the same downsweep with 64-bit outputs; out[N] = the total (tpre[tiles])
__global__ __launch_bounds__(kPB) void k_xscan_down64(const uint32_t* __restrict__ in, uint64_t N,
                                                        const uint64_t* __restrict__ tpre,
                                                        uint64_t* __restrict__ out) {
    __shared__ uint32_t wsum[kPB / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kXTile + (uint64_t)threadIdx.x * kXItems;
    uint32_t v[kXItems];
    uint32_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kXItems; ++k) {
        v[k] = base + k < N ? in[base + k] : 0u;
        s += v[k];
    }
    uint64_t run = tpre[blockIdx.x] + block_exscan256(s, wsum);
#pragma unroll
    for (uint32_t k = 0; k < kXItems; ++k) {
        if (base + k < N) out[base + k] = run;
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[N] = tpre[gridDim.x];
}

// offsets of bins from a scanned count matrix: out[i] = off[((i >> bits) * 256 + (i & mask)) * W]
// for i < count, out[count] = total
__global__ void k_extract_offsets(const uint32_t* __restrict__ off, uint32_t W, uint32_t bits, uint32_t count,
                                  uint64_t total, uint64_t* __restrict__ out) {
    const uint32_t mask = (1u << bits) - 1;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= count; i += gridDim.x * blockDim.x)
        out[i] = i < count ? (uint64_t)off[((uint64_t)(i >> bits) * kBins + (i & mask)) * W] : total;
}

// single block: exclusive prefix of cnt[0..N) into off (u64), copy into cursor,
// off[N] = total; the total also into *total when given
__global__ __launch_bounds__(1024) void k_scan_counts(const uint32_t* __restrict__ cnt, uint32_t N,
                                                        uint64_t* __restrict__ off, uint64_t* __restrict__ cursor,
                                                        uint64_t* __restrict__ total) {
    __shared__ uint64_t part[1024];
    const uint32_t per = (N + 1023) / 1024;
    const uint32_t a = threadIdx.x * per, b = min(N, a + per);
    uint64_t s = 0;
    for (uint32_t i = a; i < b; ++i) s += cnt[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
        const uint64_t v = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t run = part[threadIdx.x] - s;
    for (uint32_t i = a; i < b; ++i) {
        off[i] = run;
        if (cursor) cursor[i] = run;
        run += cnt[i];
    }
    if (threadIdx.x == 1023) {
        off[N] = part[1023];
        if (total) *total = part[1023];
    }
}

// per partition: 4-bit bucket sizes (written to the global size words) and the
// partition's sum of squared sizes
// (segs: partition q is partition q % kSegParts of wide map q / kSegParts; its
// size words are stored at q * 128 all the same, and an oversize bucket rejects
// only that map: oversize points to the maps' outcome words, four per map)
__global__ __launch_bounds__(kPB) void k_psizes(const uint64_t* __restrict__ keys, uint64_t n, Triple A,
                                                  uint64_t magic, const uint64_t* __restrict__ offQ,
                                                  uint32_t* __restrict__ sizes, uint64_t G,
                                                  uint32_t* __restrict__ sq_out, uint32_t* __restrict__ oversize,
                                                  const WideSeg* __restrict__ segs = nullptr) {
    __shared__ uint32_t words[kGroupsPerPart];
    __shared__ uint32_t red[kPB / 64];
    const uint32_t q = blockIdx.x;
    uint32_t qh = q;   // the partition's place among its map's partitions
    if (segs) {
        const WideSeg& sg = segs[q / kSegParts];
        A = sg.A;
        magic = sg.magic;
        n = sg.n;
        G = sg.G;
        qh = q % kSegParts;
        oversize += 4 * (q / kSegParts);
    }
    for (uint32_t g = threadIdx.x; g < kGroupsPerPart; g += kPB) words[g] = 0;
    __syncthreads();
    const uint64_t lo = offQ[q], hi = offQ[q + 1];
    bool over = false;
    auto count = [&](uint64_t x) {
        const uint32_t lb = bucket_of(A, magic, (uint32_t)n, x) & (kPartBuckets - 1);
        const uint32_t sh = 4 * (lb & 7u);
        const uint32_t old = atomicAdd(&words[lb >> 3], 1u << sh);
        over |= ((old >> sh) & 15u) == 15u;
    };
    // a typical partition's keys are all loaded before the first is hashed
    constexpr uint32_t KPT = 5;
    uint64_t x[KPT];
#pragma unroll
    for (uint32_t k = 0; k < KPT; ++k) {
        const uint64_t i = lo + threadIdx.x + (uint64_t)k * kPB;
        x[k] = i < hi ? keys[i] : 0;
    }
#pragma unroll
    for (uint32_t k = 0; k < KPT; ++k)
        if (lo + threadIdx.x + (uint64_t)k * kPB < hi) count(x[k]);
    for (uint64_t i = lo + threadIdx.x + (uint64_t)KPT * kPB; i < hi; i += kPB) count(keys[i]);
    if (over) atomicOr(oversize, 1u);
    __syncthreads();
    uint32_t sq = 0;
    for (uint32_t g = threadIdx.x; g < kGroupsPerPart; g += kPB) {
        const uint32_t w = words[g];
        if ((uint64_t)qh * kGroupsPerPart + g < G) sizes[(uint64_t)q * kGroupsPerPart + g] = w;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t s = nib(w, k);
            sq += s * s;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) sq += __shfl_xor(sq, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t w = 0; w < kPB / 64; ++w) t += red[w];
        sq_out[q] = t;
    }
}

__device__ __forceinline__ bool test_set4(uint64_t& m0, uint64_t& m1, uint64_t& m2, uint64_t& m3, uint32_t h) {
    const uint64_t bit = 1ull << (h & 63u);
    const uint32_t w = h >> 6;
    const uint64_t cur = w == 0 ? m0 : w == 1 ? m1 : w == 2 ? m2 : m3;
    if (cur & bit) return true;
    if (w == 0) m0 |= bit;
    else if (w == 1) m1 |= bit;
    else if (w == 2) m2 |= bit;
    else m3 |= bit;
    return false;
}

template <typename KeyAt>
__device__ __forceinline__ uint32_t min_trial(const Triple* C, uint32_t T, uint32_t s, KeyAt key_at,
                                              uint32_t t0 = 0) {
    const uint32_t s2 = s * s;
    for (uint32_t t = t0; t < T; ++t) {
        const Triple c = C[t];
        uint64_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
        bool collide = false;
        for (uint32_t i = 0; i < s && !collide; ++i) collide = test_set4(m0, m1, m2, m3, mshash(c, key_at(i)) % s2);
        if (!collide) return t;
    }
    return T;
}

__device__ __forceinline__ bool same_string(const int64_t* off, const uint8_t* bytes, uint32_t a, uint32_t b) {
    const int64_t la = off[a + 1] - off[a], lb = off[b + 1] - off[b];
    if (la != lb) return false;
    const uint8_t* pa = bytes + off[a];
    const uint8_t* pb = bytes + off[b];
    for (int64_t i = 0; i < la; ++i)
        if (pa[i] != pb[i]) return false;
    return true;
}

template <bool AUX>
struct FinalLds {
    uint64_t key[kFinalKeyCap];
    uint32_t val[kFinalKeyCap];
    uint32_t aux[AUX ? kFinalKeyCap : 1];
    uint16_t smap[kFinalCellCap];
    uint32_t words[kGroupsPerPart];
    uint32_t cnt2[kGroupsPerPart];
    uint32_t gks[kGroupsPerPart];
    uint32_t gbase[kGroupsPerPart];
    uint8_t tb[kPartBuckets];
    uint32_t occ[kFinalCellCap / 32];   // cells taken by trial 0
    uint32_t fl[kPartBuckets / 32];     // buckets where trial 0 collides
    uint16_t hard[kFinalKeyCap / 2];   // buckets of two or more keys that trial 0 does not place
    uint64_t mag[16];             // remainder magic of s^2, s = 0..15
    Triple tri[kLdsTrials];       // the first level-two triples (larger trials are rare)
    uint32_t nhard;
    uint32_t wsum[2][kPB / 64];
    uint32_t flags[3];   // exhausted, dup, max_t
    uint64_t c0;         // fused form: the partition's first cell, from the look-back
    uint32_t sqtot;      // the partition's sum of squared sizes
    uint32_t ticket;     // fused form: the partition this workgroup works on
    uint32_t over;       // fused form: a bucket above 15 keys
};

// look-back polls of one predecessor's word before the fused pass gives up (far beyond any
// real wait: every predecessor publishes its sum without waiting on anything)
constexpr uint32_t kSpinLimit = 1u << 24;

// The fused final pass (single map, level-two search in partition order): each partition
// takes a ticket, sizes its buckets itself, publishes its sum of squared sizes, and finds
// its first cell by a look-back over its predecessors' published sums (a decoupled
// look-back scan: the nearest predecessor that already published its inclusive prefix
// ends it).  state holds one word per partition: value << 2 | 1 (the partition's own sum)
// or value << 2 | 2 (the inclusive prefix); zero means not yet published.
struct FuseArgs {
    uint64_t* state;      // Q words, zero before the launch
    uint32_t* ticket;     // zero before the launch
    uint64_t* S_out;      // the table's S, written by the last partition
    uint32_t* oversize;   // set when some bucket holds more than 15 keys
    uint32_t* stalled;    // set when a look-back gave up
    uint32_t Q;
    const uint64_t* qend; // partition q's records are [offQ[q], min(qend[q], offQ[q] + qcap))
    uint64_t qcap;        // 0: no cap
};

// largest of a small value (below 16) over the wave's active lanes
__device__ __forceinline__ uint32_t wave_max16(uint32_t v) {
    uint32_t m = 0;
#pragma unroll
    for (int b = 3; b >= 0; --b) {
        const uint32_t c = m | (1u << b);
        if (__any(v >= c)) m = c;
    }
    return m;
}

// smallest trial from t0 on for a bucket of 2..8 keys held in registers: one 64-bit
// occupancy mask, remainders by multiplication.  smax: the largest bucket among the
// wave's active lanes; key slots beyond it are skipped by the whole wave
// (tri(t): triple t)
template <typename TriAt>
__device__ __forceinline__ uint32_t min_trial_small(TriAt tri, uint32_t T, uint32_t s, const uint64_t (&kx)[8],
                                                    uint64_t M, uint32_t t0 = 0, uint32_t smax = 8) {
    const uint32_t s2 = s * s;
    for (uint32_t t = t0; t < T; ++t) {
        const Triple c = tri(t);
        uint64_t m = 0;
        bool collide = false;
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i) {
            if (i >= smax) break;
            if (i < s && !collide) {
                const uint64_t bit = 1ull << fastmod(mshash(c, kx[i]), M, s2);
                collide = (m & bit) != 0;
                m |= bit;
            }
        }
        if (!collide) return t;
    }
    return T;
}

// waves per SIMD the final pass is compiled for (registers within 80, or 96 with an aux
// word): the LDS of six workgroups (26.5 KB each), or five with an aux word (31.5 KB),
// fits a CU
template <bool AUX>
constexpr unsigned kFinalWaves = AUX ? 5u : 6u;

// AUX: an aux word travels with every key (a string key's index, or the high
// half of a 64-bit value); STR: keys are string fingerprints, so equal keys
// are told apart by their bytes
// MULTI: partition q is partition q % kSegParts of wide map q / kSegParts of a batch
// (segs); the map's hash, triples (Cg + map*T), header and cells (pool offsets) come
// from its descriptor, cbase holds kSegParts+1 map-relative cell offsets per map,
// and ctrl_flags points to four outcome words per map (a map whose word 0 is set was
// rejected before this kernel and is skipped)
// FUSED: the single map's final pass sizes its own partition and finds its first cell by
// the look-back above (no separate size pass and scan; grid = Q)
template <bool AUX, bool STR, bool MULTI = false, bool FUSED = false>
__global__ __launch_bounds__(kPB) __attribute__((amdgpu_waves_per_eu(kFinalWaves<AUX>))) void k_pfinal(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                                  const uint32_t* __restrict__ aux, int aux_is_pos, uint64_t n,
                                                  Triple A, uint64_t magic, const uint64_t* __restrict__ offQ,
                                                  const uint64_t* __restrict__ cbase, const uint32_t* __restrict__ sizes,
                                                  uint64_t G, const Triple* __restrict__ Cg, uint32_t T,
                                                  Group* __restrict__ header, Cell* __restrict__ slots,
                                                  uint32_t* __restrict__ ctrl_flags, const int64_t* __restrict__ ctx_off,
                                                  const uint8_t* __restrict__ ctx_bytes,
                                                  const uint8_t* __restrict__ given_t,
                                                  const WideSeg* __restrict__ segs = nullptr,
                                                  const uint32_t* __restrict__ reject = nullptr,
                                                  uint64_t cap = ~0ull, FuseArgs fa = FuseArgs{}) {
    static_assert(!(MULTI && FUSED), "the fused pass builds one map");
    __shared__ FinalLds<AUX> L;
    const uint32_t tid = threadIdx.x;
    // an attempt already rejected by the size pass (a bucket above 15 keys) or by bad
    // string offsets is skipped (both flags are set before this kernel starts)
    if (reject && (reject[0] | reject[1])) return;   // the whole block
    uint32_t q = blockIdx.x;
    if (FUSED) {
        // partitions go in ticket order: every partition a look-back below waits for was
        // taken by a workgroup that is already running
        if (tid == 0) L.ticket = atomicAdd(fa.ticket, 1u);
        __syncthreads();
        q = L.ticket;
    }
    uint32_t qh = q;   // the partition's place among its map's partitions
    uint64_t cq = q;   // its entry in cbase
    if (MULTI) {
        const uint32_t mseg = q / kSegParts;
        const WideSeg& sg = segs[mseg];
        qh = q % kSegParts;
        if (ctrl_flags[4 * mseg] != 0 || (uint64_t)qh * kPartBuckets >= sg.n) return;   // the whole block
        A = sg.A;
        magic = sg.magic;
        n = sg.n;
        G = sg.G;
        Cg += (uint64_t)sg.map * T;
        header += sg.hdr_off;
        slots += sg.slot_off;
        ctrl_flags += 4 * mseg + 1;
        cq = (uint64_t)mseg * (kSegParts + 1) + qh;
    }
    const uint64_t k0 = offQ[q];
    const uint64_t k1 = !FUSED ? offQ[q + 1] : fa.qcap ? min(fa.qend[q], k0 + fa.qcap) : fa.qend[q];
    const uint32_t nq = (uint32_t)(k1 - k0);
    const bool keys_fit = nq <= kFinalKeyCap;
    // a partition whose cells would end beyond the cells allocated is skipped (the attempt
    // then runs this pass again into an exact allocation); the fused form learns its cells
    // below
    uint64_t c0 = 0;
    uint32_t Sq = 0;
    if (!FUSED) {
        c0 = cbase[cq];
        Sq = (uint32_t)(cbase[cq + 1] - c0);
        if (c0 + Sq > cap) return;   // the whole block
    }
    bool fast = FUSED ? keys_fit : keys_fit && Sq <= kFinalCellCap;
    // the partition's records go in flight first; the set-up below overlaps their latency
    constexpr uint32_t KPT = (kFinalKeyCap + kPB - 1) / kPB;   // record slots per thread
    uint64_t xk[KPT];
    uint32_t vk[KPT], ak[KPT];
    if (fast) {
#pragma unroll
        for (uint32_t k = 0; k < KPT; ++k) {
            const uint32_t i = tid + k * kPB;
            if (i < nq) {
                // streaming loads: each record is read once here (and each cell and group
                // record below written once), so none of them displaces the caches' other data
                xk[k] = __builtin_nontemporal_load(keys + k0 + i);
                vk[k] = __builtin_nontemporal_load(vals + k0 + i);
                if (AUX) ak[k] = aux_is_pos ? (uint32_t)(k0 + i) : aux[k0 + i];
            }
        }
    }
    // the first kLdsTrials level-two triples are staged in LDS; larger trials read theirs
    // from global memory
    const Triple* const LC = Cg;
    for (uint32_t t = tid; t < kLdsTrials && t < T; t += kPB) L.tri[t] = Cg[t];
    auto tri = [&](uint32_t t) { return t < kLdsTrials ? L.tri[t] : Cg[t]; };
    if (!FUSED) {
        for (uint32_t g = tid; g < kGroupsPerPart; g += kPB)
            L.words[g] = (uint64_t)qh * kGroupsPerPart + g < G ? sizes[(uint64_t)q * kGroupsPerPart + g] : 0u;
    }
    if (tid < 3) L.flags[tid] = 0;
    if (FUSED && tid == 0) L.over = 0;
    if (FUSED || fast) {
        for (uint32_t g = tid; g < kGroupsPerPart; g += kPB) L.cnt2[g] = 0;
        for (uint32_t b = tid; b < kPartBuckets; b += kPB) L.tb[b] = 0;
        for (uint32_t w = tid; w < kFinalCellCap / 32; w += kPB) L.occ[w] = 0;
        if (tid < kPartBuckets / 32) L.fl[tid] = 0;
        if (tid < 16) L.mag[tid] = tid ? fastmod_magic(tid * tid) : 0;
        if (tid == 0) L.nhard = 0;
    }
    __syncthreads();
    uint32_t lbk[KPT], rk[KPT], c0k[KPT];
    // rank the partition's records (when they fit) in their buckets: ranks come from an LDS
    // histogram of the 4-bit bucket sizes, which the fused form also takes as the
    // partition's sizes.  The records stay in registers until they are grouped.
    auto stage = [&]() {
        bool over = false;
#pragma unroll
        for (uint32_t k = 0; k < KPT; ++k) {
            const uint32_t i = tid + k * kPB;
            if (i < nq) {
                const uint32_t lb = bucket_of(A, magic, (uint32_t)n, xk[k]) & (kPartBuckets - 1);
                lbk[k] = lb;
                const uint32_t sh = 4 * (lb & 7u);
                rk[k] = (atomicAdd(&L.cnt2[lb >> 3], 1u << sh) >> sh) & 15u;
                over |= rk[k] == 15u;   // this key is the bucket's sixteenth
            }
        }
        return over;
    };
    if (FUSED) {
        bool over = false;
        if (keys_fit) {
            over = stage();
        } else {
            // too many keys to stage: their sizes from one pass over them
            for (uint32_t i = tid; i < nq; i += kPB) {
                const uint32_t lb = bucket_of(A, magic, (uint32_t)n, keys[k0 + i]) & (kPartBuckets - 1);
                const uint32_t sh = 4 * (lb & 7u);
                over |= ((atomicAdd(&L.cnt2[lb >> 3], 1u << sh) >> sh) & 15u) == 15u;
            }
        }
        if (over) atomicOr(&L.over, 1u);
        __syncthreads();
        for (uint32_t g = tid; g < kGroupsPerPart; g += kPB) L.words[g] = L.cnt2[g];
        __syncthreads();
    }
    // group statistics: where each group's keys and cells start inside the partition
    {
        uint32_t c = 0, s2 = 0;
        if (tid < kGroupsPerPart) {
            const uint32_t w = L.words[tid];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t s = nib(w, k);
                c += s;
                s2 += s * s;
            }
        }
        uint32_t ic = c, is = s2;
        const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t uc = __shfl_up(ic, d, 64), us = __shfl_up(is, d, 64);
            if (lane >= d) {
                ic += uc;
                is += us;
            }
        }
        if (lane == 63) {
            L.wsum[0][wv] = ic;
            L.wsum[1][wv] = is;
        }
        __syncthreads();
        uint32_t pc = 0, ps = 0;
        for (int w = 0; w < wv; ++w) {
            pc += L.wsum[0][w];
            ps += L.wsum[1][w];
        }
        if (tid < kGroupsPerPart) {
            L.gks[tid] = pc + ic - c;
            L.gbase[tid] = ps + is - s2;
        }
        if (tid == kGroupsPerPart - 1) L.sqtot = ps + is;
    }
    // fused form: the partition's first cell, from the predecessors' published sums back to
    // the nearest published inclusive prefix (64 per round: lane l reads partition
    // end - 1 - l); then this partition's inclusive prefix is published.  Called by the
    // whole workgroup just before the cells are written, when the predecessors' sums, which
    // each publishes as soon as it has sized its buckets, are there to read.
    auto lookback = [&]() {
        if (tid < 64) {
            const uint32_t lane = tid;
            uint64_t excl = 0;
            int64_t end = (int64_t)q;
            for (;;) {
                const int64_t idx = end - 1 - (int64_t)lane;
                uint64_t v = 2;   // before the first partition: an inclusive prefix of 0
                if (idx >= 0) {
                    uint32_t spins = 0;
                    for (;;) {
                        v = __hip_atomic_load(&fa.state[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (v & 3u) break;
                        if (++spins > kSpinLimit) {
                            atomicOr(fa.stalled, 1u);
                            v = 2;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                const uint64_t incl = __ballot((v & 3u) == 2u);
                uint64_t take = v >> 2;
                const bool last = incl != 0;
                if (last && lane > (uint32_t)(__ffsll((long long)incl) - 1)) take = 0;
                for (int d = 32; d >= 1; d >>= 1) take += __shfl_xor(take, d, 64);
                excl += take;
                if (last) break;
                end -= 64;
            }
            if (lane == 0) {
                L.c0 = excl;
                __hip_atomic_store(&fa.state[q], ((excl + Sq) << 2) | 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (q + 1 == fa.Q) *fa.S_out = excl + Sq;
            }
        }
        __syncthreads();
        c0 = L.c0;
    };
    if (FUSED) {
        __syncthreads();
        Sq = L.sqtot;
        // publish this partition's sum at once: the look-backs of later partitions read it
        if (tid == 0)
            __hip_atomic_store(&fa.state[q], ((uint64_t)Sq << 2) | 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (L.over) {
            lookback();
            if (tid == 0) atomicOr(fa.oversize, 1u);
            return;   // the whole block: the attempt is rejected
        }
        fast = keys_fit && Sq <= kFinalCellCap;
    }
    if (fast) {
        if (!FUSED) (void)stage();
        __syncthreads();
        // group by bucket: each record goes to the LDS slot of its rank in its bucket, so a
        // bucket's keys lie together (from here on a record is named by its slot).  A lone
        // key owns its bucket's single cell.  Every key of a larger bucket tries trial 0 at
        // once: the second key to claim a cell marks its bucket as colliding, and only those
        // buckets are searched below.
        const Triple c0t = L.tri[0];
#pragma unroll
        for (uint32_t k = 0; k < KPT; ++k) {
            const uint32_t i = tid + k * kPB;
            if (i < nq) {
                const uint32_t lb = lbk[k], g = lb >> 3, kk = lb & 7u, w = L.words[g];
                const uint32_t s = nib(w, kk);
                const uint32_t off = L.gbase[g] + prefix_sq(w, kk);
                const uint32_t slot = L.gks[g] + prefix_cnt(w, kk) + rk[k];
                if (s >= 2) {
                    // the key of rank r marks cells [r*s, r*s + s) of its bucket with the
                    // bucket's first cell; placement below overwrites the cells keys take, and
                    // the write-out resolves a cell still marked to the bucket's lowest
                    // occupied cell (the fill rule)
                    const uint32_t from = off + rk[k] * s;
                    for (uint32_t u = 0; u < s; ++u) L.smap[from + u] = (uint16_t)(0x8000u | off);
                }
                rk[k] = slot;
                L.key[slot] = xk[k];
                L.val[slot] = vk[k];
                if (AUX) L.aux[slot] = ak[k];
                c0k[k] = off;
                const uint32_t h0 = mshash(c0t, xk[k]);   // trial 0
                if (s == 1) {
                    L.smap[off] = (uint16_t)slot;
                    L.tb[lb] = (uint8_t)tag_of(h0);   // trial 0; the byte holds the key's tag
                } else {
                    if (!given_t) {
                        const uint32_t cell = off + fastmod(h0, L.mag[s], s * s);
                        c0k[k] = cell;
                        const uint32_t bit = 1u << (cell & 31u), bb = 1u << (lb & 31u);
                        if ((atomicOr(&L.occ[cell >> 5], bit) & bit) && !(atomicOr(&L.fl[lb >> 5], bb) & bb))
                            L.hard[atomicAdd(&L.nhard, 1u)] = (uint16_t)lb;
                    }
                }
            }
        }
        __syncthreads();
        // Trials: a bucket that trial 0 places keeps t = 0 (tb is zero); given trials (the
        // rounds schedule) are taken as they are
        if (given_t) {
            for (uint32_t b = tid; b < kPartBuckets; b += kPB) {
                if (nib(L.words[b >> 3], b & 7u) < 2) continue;
                const uint32_t t = given_t[(uint64_t)q * kPartBuckets + b];
                L.tb[b] = (uint8_t)t;
                if (t) atomicMax(&L.flags[2], t);
            }
        }
        // the colliding buckets, one lane each, trials from 1 on with the keys in registers;
        // bucket j goes to lane j / 4 of wave j % 4, so that all four SIMDs search (a packed
        // list of ~80 buckets would otherwise occupy one and a half waves)
        const uint32_t nh = given_t ? 0u : L.nhard;
        for (uint32_t j = (tid & 63u) * (kPB / 64) + (tid >> 6); j < nh; j += kPB) {
            const uint32_t b = L.hard[j];
            const uint32_t w = L.words[b >> 3];
            const uint32_t sb = nib(w, b & 7u);
            const uint32_t kst = L.gks[b >> 3] + prefix_cnt(w, b & 7u);
            uint32_t t;
            if (sb <= 8) {
                const uint32_t smax = wave_max16(sb);
                uint64_t kx[8];
#pragma unroll
                for (uint32_t i = 0; i < 8; ++i) kx[i] = i < sb ? L.key[kst + i] : 0;
                t = min_trial_small(tri, T, sb, kx, L.mag[sb], 1, smax);
            } else {
                t = min_trial(LC, T, sb, [&](uint32_t i) { return L.key[kst + i]; }, 1);
            }
            if (t < T) {
                L.tb[b] = (uint8_t)t;
                atomicMax(&L.flags[2], t);
            } else {
                // no trial separates the bucket: the attempt fails, or the build when
                // two keys are equal; the cells get any in-range content
                bool dup = false;
                for (uint32_t a2 = 0; a2 < sb; ++a2)
                    for (uint32_t b2 = a2 + 1; b2 < sb; ++b2) {
                        const uint32_t ia = kst + a2, ib = kst + b2;
                        if (STR) dup |= same_string(ctx_off, ctx_bytes, L.aux[ia], L.aux[ib]);
                        else dup |= L.key[ia] == L.key[ib];
                    }
                atomicOr(&L.flags[0], 1u);
                if (dup) atomicOr(&L.flags[1], 1u);
            }
        }
        __syncthreads();
        // every key of a larger bucket writes its own cell
#pragma unroll
        for (uint32_t k = 0; k < KPT; ++k) {
            const uint32_t i = tid + k * kPB;
            if (i < nq) {
                const uint32_t lb = lbk[k], g = lb >> 3, kk = lb & 7u, w = L.words[g];
                const uint32_t sb = nib(w, kk);
                if (sb >= 2) {
                    const uint32_t t = L.tb[lb];
                    const uint32_t cell = (t || given_t) ? L.gbase[g] + prefix_sq(w, kk) +
                                                               fastmod(mshash(tri(t), L.key[rk[k]]), L.mag[sb], sb * sb)
                                                         : c0k[k];
                    L.smap[cell] = (uint16_t)rk[k];
                }
            }
        }
        __syncthreads();
        if (FUSED) {
            lookback();
            if (c0 + Sq > cap) return;   // the whole block
        }
        // write-out: indices first (a marked cell resolves to the bucket's lowest
        // occupied cell; every bucket holds a key), then the records
        constexpr uint32_t CPT = kFinalCellCap / kPB;
        static_assert(kFinalCellCap % kPB == 0, "whole cells per thread");
        uint32_t idx[CPT];
#pragma unroll
        for (uint32_t k = 0; k < CPT; ++k) {
            const uint32_t p = tid + k * kPB;
            idx[k] = p < Sq ? L.smap[p] : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < CPT; ++k) {
            if (idx[k] & 0x8000u) {
                uint32_t i;
                for (uint32_t p2 = idx[k] & 0x7FFFu; (i = L.smap[p2]) & 0x8000u; ++p2) {}
                idx[k] = i;
            }
        }
#pragma unroll
        for (uint32_t k = 0; k < CPT; ++k) {
            const uint32_t p = tid + k * kPB;
            if (p < Sq) {
                const uint32_t i = idx[k];
                Cell c;
                c.key = L.key[i];
                c.val = L.val[i];
                c.aux = AUX ? L.aux[i] : 0u;
                store_cell_once(slots + c0 + p, c);
            }
        }
    } else {
        // rare: the partition does not fit the LDS staging; every bucket gathers its
        // own keys from HBM (a scan of the partition), searches and writes its cells
        __syncthreads();
        if (FUSED) {
            lookback();
            if (c0 + Sq > cap) return;   // the whole block
        }
        for (uint32_t b = tid; b < kPartBuckets; b += kPB) {
            const uint32_t g = b >> 3, kk = b & 7u, w = L.words[g];
            const uint32_t s = nib(w, kk);
            const uint32_t off = L.gbase[g] + prefix_sq(w, kk);
            uint64_t mine[kSMax];
            uint32_t pos[kSMax];
            uint32_t got = 0;
            if (s) {
                for (uint32_t i = 0; i < nq && got < s; ++i) {
                    const uint64_t x = keys[k0 + i];
                    if ((bucket_of(A, magic, (uint32_t)n, x) & (kPartBuckets - 1)) == b) {
                        mine[got] = x;
                        pos[got] = i;
                        ++got;
                    }
                }
            }
            uint32_t t = 0;
            bool exhausted = false;
            if (s >= 2) {
                t = given_t ? given_t[(uint64_t)q * kPartBuckets + b]
                            : min_trial(LC, T, s, [&](uint32_t i) { return mine[i]; });
                exhausted = t == T;
            }
            const uint32_t s2 = s * s;
            if (s >= 1 && !exhausted) {
                const Triple c = LC[t];
                uint32_t first_p = s2, first_i = 0;
                for (uint32_t i = 0; i < s; ++i) {
                    const uint32_t h = mshash(c, mine[i]) % s2;
                    if (h < first_p) {
                        first_p = h;
                        first_i = i;
                    }
                }
                for (uint32_t p = 0; p < s2; ++p) {
                    uint32_t who = first_i;
                    for (uint32_t i = 0; i < s; ++i)
                        if (mshash(c, mine[i]) % s2 == p) who = i;
                    Cell cl;
                    cl.key = mine[who];
                    cl.val = vals[k0 + pos[who]];
                    cl.aux = AUX ? (aux_is_pos ? (uint32_t)(k0 + pos[who]) : aux[k0 + pos[who]]) : 0u;
                    slots[c0 + off + p] = cl;
                }
            }
            if (exhausted) {
                bool dup = false;
                for (uint32_t a = 0; a < s; ++a)
                    for (uint32_t b2 = a + 1; b2 < s; ++b2) {
                        if (STR) {
                            const uint32_t xa = aux_is_pos ? (uint32_t)(k0 + pos[a]) : aux[k0 + pos[a]];
                            const uint32_t xb = aux_is_pos ? (uint32_t)(k0 + pos[b2]) : aux[k0 + pos[b2]];
                            dup |= same_string(ctx_off, ctx_bytes, xa, xb);
                        } else {
                            dup |= mine[a] == mine[b2];
                        }
                    }
                atomicOr(&L.flags[0], 1u);
                if (dup) atomicOr(&L.flags[1], 1u);
                t = 0;
            }
            if (t) atomicMax(&L.flags[2], t);
            L.tb[b] = (uint8_t)(s == 1 ? key_tag(LC[0], mine[0]) : t);
        }
        __syncthreads();
    }
    for (uint32_t g = tid; g < kGroupsPerPart; g += kPB) {
        const uint64_t gg = (uint64_t)qh * kGroupsPerPart + g;
        if (gg < G) {
            Group h;
            h.base = (uint32_t)(c0 + L.gbase[g]);
            h.sizes = L.words[g];
            h.t_lo = (uint32_t)L.tb[8 * g] | ((uint32_t)L.tb[8 * g + 1] << 8) | ((uint32_t)L.tb[8 * g + 2] << 16) |
                     ((uint32_t)L.tb[8 * g + 3] << 24);
            h.t_hi = (uint32_t)L.tb[8 * g + 4] | ((uint32_t)L.tb[8 * g + 5] << 8) |
                     ((uint32_t)L.tb[8 * g + 6] << 16) | ((uint32_t)L.tb[8 * g + 7] << 24);
            const u32x4 hw = {h.base, h.sizes, h.t_lo, h.t_hi};
            __builtin_nontemporal_store(hw, reinterpret_cast<u32x4*>(header) + gg);
        }
    }
    if (tid == 0) {
        if (L.flags[0]) atomicOr(&ctrl_flags[0], 1u);
        if (L.flags[1]) atomicOr(&ctrl_flags[1], 1u);
        if (L.flags[2]) atomicMax(&ctrl_flags[2], L.flags[2]);
    }
}

// cell offsets of every wide map's partitions (map-relative) and the map's S; a map
// whose S exceeds c*n is rejected (outcome word 0)
__global__ void k_wbases(const uint32_t* __restrict__ sqQ, const WideSeg* __restrict__ segs, uint32_t nseg,
                         uint64_t* __restrict__ cbase, uint32_t* __restrict__ flags) {
    for (uint32_t m = blockIdx.x * blockDim.x + threadIdx.x; m < nseg; m += gridDim.x * blockDim.x) {
        uint64_t acc = 0;
        for (uint32_t j = 0; j < kSegParts; ++j) {
            cbase[(uint64_t)m * (kSegParts + 1) + j] = acc;
            acc += sqQ[(uint64_t)m * kSegParts + j];
        }
        cbase[(uint64_t)m * (kSegParts + 1) + kSegParts] = acc;
        if (acc > (uint64_t)segs[m].c * segs[m].n) flags[4 * m] |= 2u;
    }
}

// ---- host planning and launches ------------------------------------------------------

PartPlan part_plan(uint64_t n) {
    PartPlan P{};
    P.Q = (uint32_t)((n + kPartBuckets - 1) / kPartBuckets);
    uint32_t bits = 0;
    while ((1ull << bits) < P.Q) ++bits;
    P.bits_q = bits;
    auto clampu = [](uint64_t v, uint64_t lo, uint64_t hi) { return (uint32_t)(v < lo ? lo : v > hi ? hi : v); };
    P.W1 = clampu((n + kWorkerKeys - 1) / (kWorkerKeys), 1, 4096);
    // regions of the cursor form: a first-level bin covers 2^shiftA partitions of 1024
    // buckets and a partition 1024 buckets; with n keys in n buckets the keys of B buckets
    // number B on average with a standard deviation of about sqrt(B), and the regions hold
    // 12 deviations more (an overflow only sends the attempt back to the counted passes)
    auto region = [](uint64_t B) {
        const uint64_t sd = (uint64_t)std::ceil(std::sqrt((double)B));
        return (B + 12 * sd + 64 + 255) & ~(uint64_t)255;
    };
    if (P.Q <= 1) {
        P.passes = 0;
    } else if (bits <= 8) {
        P.passes = 1;
        P.binsA = P.Q;
        P.capQ = region(kPartBuckets);
    } else if (bits <= 16) {
        P.passes = 2;
        P.shiftA = bits - 8;
        P.binsA = (uint32_t)((P.Q + (1u << P.shiftA) - 1) >> P.shiftA);
        P.bitsB = P.shiftA;
        P.W2 = clampu((n / P.binsA + kWorkerKeys - 1) / (kWorkerKeys), 1, 64);
        P.cap1 = region((uint64_t)kPartBuckets << P.shiftA);
        P.capQ = region(kPartBuckets);
    } else {
        P.passes = 3;
        P.shiftA = bits - 8;
        P.binsA = (uint32_t)((P.Q + (1u << P.shiftA) - 1) >> P.shiftA);
        P.bitsC = bits - 16;
        P.bitsB = 8;
        P.binsAB = (uint32_t)((P.Q + (1u << P.bitsC) - 1) >> P.bitsC);
        P.W2 = clampu((n / P.binsA + kWorkerKeys - 1) / (kWorkerKeys), 1, 64);
        P.W3 = clampu((n / P.binsAB + kWorkerKeys - 1) / (kWorkerKeys), 1, 64);
    }
    uint64_t m1 = (uint64_t)kBins * P.W1;
    uint64_t m2 = P.passes >= 2 ? (uint64_t)P.binsA * kBins * P.W2 : 0;
    uint64_t m3 = P.passes == 3 ? (uint64_t)P.binsAB * kBins * P.W3 : 0;
    P.matrix = std::max(m1, std::max(m2, m3));
    return P;
}

uint64_t exscan_tiles(uint64_t N) { return (N + kXTile - 1) / kXTile; }
uint64_t part_scan_tiles(const PartPlan& P) { return exscan_tiles(std::max<uint64_t>(P.matrix, P.Q)); }

void exscan_u32(const uint32_t* in, uint64_t N, uint32_t* tsum, uint64_t* tpre, uint32_t* out, hipStream_t st) {
    const uint32_t nt = (uint32_t)exscan_tiles(N);
    hipLaunchKernelGGL(k_xscan_reduce, nt, kPB, 0, st, in, N, tsum);
    hipLaunchKernelGGL(k_scan_counts, 1, 1024, 0, st, tsum, nt, tpre, nullptr, nullptr);
    hipLaunchKernelGGL(k_xscan_down, nt, kPB, 0, st, in, N, tpre, out);
}

static void scan_matrix(const PartArgs& a, uint64_t N, hipStream_t st) { exscan_u32(a.cnt, N, a.tsum, a.tpre, a.off, st); }

template <bool AUX>
static void scatter(const PartArgs& a, const uint64_t* kin, const uint32_t* vin, const uint32_t* ain,
                    const uint64_t* ranges, dim3 grid, uint32_t W, uint32_t shift, uint32_t mask, uint64_t* kout,
                    uint32_t* vout, uint32_t* aout, hipStream_t st) {
    FKS_TIMED("fks_part_scatter", st,
              hipLaunchKernelGGL((k_dscatter<AUX, AUX ? kPScatterItemsAux : kPScatterItems, kPScatterThreads>), grid,
                                 kPScatterThreads, 0, st, kin, vin, ain, a.n, a.A, a.magic, ranges, W,
                                 shift, mask, a.off, kout, vout, aout));
}

template <bool AUX>
static void scatter_cursor(const PartArgs& a, const uint64_t* kin, const uint32_t* vin, const uint32_t* ain,
                           const uint64_t* ranges, const uint64_t* ranges_hi, uint64_t in_cap, dim3 grid, uint32_t W,
                           uint32_t shift, uint32_t mask, uint64_t* kout, uint32_t* vout, uint32_t* aout,
                           unsigned long long* cursor, uint64_t cap, hipStream_t st) {
    FKS_TIMED("fks_part_scatter", st,
              hipLaunchKernelGGL((k_dscatter<AUX, AUX ? kPScatterItemsAux : kPScatterItems, kPScatterThreads, true>),
                                 grid, kPScatterThreads, 0, st, kin, vin, ain, a.n, a.A, a.magic, ranges, W, shift,
                                 mask, nullptr, kout, vout, aout, nullptr, cursor, ranges_hi, cap, a.overflow,
                                 in_cap));
}

static unsigned grid_for_count(uint64_t count) { return (unsigned)std::min<uint64_t>((count + 255) / 256, 4096); }

// Runs the partition passes of one attempt; stream-ordered outputs: offQ, the
// records in partition order (o.keys/vals/aux), the size words, the partition
// sums of squares, their scan (cbase) and the total S (*S_dev).
int part_prepare(const PartArgs& a, hipStream_t st, PartOut& o) {
    const PartPlan P = part_plan(a.n);
    const uint64_t n = a.n;
    const bool aux = a.aux;
    o.plan = P;
    o.keys = a.keys;
    o.vals = a.vals;
    o.aux = a.aux_in;
    o.aux_is_pos = a.aux_in ? 0 : 1;
    o.qbeg = a.offQ;
    o.qend = a.offQ + 1;
    o.qcap = 0;   // no cap: the counted passes fill their ranges exactly
    o.prezeroed = false;
    auto count = [&](const uint64_t* kin, const uint64_t* ranges, dim3 grid, uint32_t W, uint32_t shift,
                     uint32_t mask) {
        FKS_TIMED("fks_part_count", st,
                  hipLaunchKernelGGL(k_dcount, grid, kPB, 0, st, kin, n, a.A, a.magic, ranges, W, shift, mask,
                                     a.cnt));
    };
    if (P.passes == 0) {
        hipLaunchKernelGGL(k_set_range, 1, 64, 0, st, a.offQ, n);
    } else if (P.passes == 1 && a.cursor) {
        // one pass straight into the partitions' regions, each run reserved on its partition's
        // cursor; the fused final pass's look-back words and ticket are cleared in the same launch
        const uint64_t nzw = a.fused ? 2 * (uint64_t)P.Q : 0;
        hipLaunchKernelGGL(k_init_cursors, grid_for_count(P.Q + nzw), 256, 0, st, a.cur1, a.begA, (uint64_t)0,
                           (uint64_t)0, a.cur2, a.begQ, (uint64_t)P.Q, P.capQ, reinterpret_cast<uint32_t*>(a.cbase),
                           nzw, a.fused ? a.sqQ : nullptr);
        o.prezeroed = a.fused;
        if (aux)
            scatter_cursor<true>(a, a.keys, a.vals, a.aux_in, nullptr, nullptr, 0, dim3(P.W1, 1), P.W1, 0, 255, a.k2,
                                 a.v2, a.a2, a.cur2, P.capQ, st);
        else
            scatter_cursor<false>(a, a.keys, a.vals, nullptr, nullptr, nullptr, 0, dim3(P.W1, 1), P.W1, 0, 255,
                                  a.k2, a.v2, a.a2, a.cur2, P.capQ, st);
        o.keys = a.k2;
        o.vals = a.v2;
        o.aux = a.a2;
        o.aux_is_pos = aux ? 0 : 1;
        o.qbeg = a.begQ;
        o.qend = reinterpret_cast<const uint64_t*>(a.cur2);
        o.qcap = P.capQ;
    } else if (P.passes == 1) {
        count(a.keys, nullptr, dim3(P.W1, 1), P.W1, 0, 255);
        scan_matrix(a, (uint64_t)kBins * P.W1, st);
        if (aux)
            scatter<true>(a, a.keys, a.vals, a.aux_in, nullptr, dim3(P.W1, 1), P.W1, 0, 255, a.k2, a.v2, a.a2, st);
        else
            scatter<false>(a, a.keys, a.vals, nullptr, nullptr, dim3(P.W1, 1), P.W1, 0, 255, a.k2, a.v2, a.a2, st);
        hipLaunchKernelGGL(k_extract_offsets, (P.Q + 256) / 256, 256, 0, st, a.off, P.W1, 8u, P.Q, n, a.offQ);
        o.keys = a.k2;
        o.vals = a.v2;
        o.aux = a.a2;
        o.aux_is_pos = aux ? 0 : 1;
    } else if (P.passes == 2 && a.cursor) {
        // first-level bins, then partitions, each reserved run by run on the bin's cursor; the
        // fused final pass's look-back words and ticket are cleared in the same launch
        const uint64_t nzw = a.fused ? 2 * (uint64_t)P.Q : 0;
        hipLaunchKernelGGL(k_init_cursors, grid_for_count(P.binsA + P.Q + nzw), 256, 0, st, a.cur1, a.begA,
                           (uint64_t)P.binsA, P.cap1, a.cur2, a.begQ, (uint64_t)P.Q, P.capQ,
                           reinterpret_cast<uint32_t*>(a.cbase), nzw, a.fused ? a.sqQ : nullptr);
        o.prezeroed = a.fused;
        if (aux)
            scatter_cursor<true>(a, a.keys, a.vals, a.aux_in, nullptr, nullptr, 0, dim3(P.W1, 1), P.W1, P.shiftA,
                                 255, a.k1, a.v1, a.a1, a.cur1, P.cap1, st);
        else
            scatter_cursor<false>(a, a.keys, a.vals, nullptr, nullptr, nullptr, 0, dim3(P.W1, 1), P.W1, P.shiftA,
                                  255, a.k1, a.v1, a.a1, a.cur1, P.cap1, st);
        const uint32_t maskB = (1u << P.bitsB) - 1;
        const uint64_t* hi1 = reinterpret_cast<const uint64_t*>(a.cur1);
        if (aux)
            scatter_cursor<true>(a, a.k1, a.v1, a.a1, a.begA, hi1, P.cap1, dim3(P.W2, P.binsA), P.W2, 0, maskB, a.k2,
                                 a.v2, a.a2, a.cur2, P.capQ, st);
        else
            scatter_cursor<false>(a, a.k1, a.v1, nullptr, a.begA, hi1, P.cap1, dim3(P.W2, P.binsA), P.W2, 0, maskB,
                                  a.k2, a.v2, a.a2, a.cur2, P.capQ, st);
        o.keys = a.k2;
        o.vals = a.v2;
        o.aux = a.a2;
        o.aux_is_pos = aux ? 0 : 1;
        o.qbeg = a.begQ;
        o.qend = reinterpret_cast<const uint64_t*>(a.cur2);
        o.qcap = P.capQ;
    } else if (P.passes == 2) {
        count(a.keys, nullptr, dim3(P.W1, 1), P.W1, P.shiftA, 255);
        scan_matrix(a, (uint64_t)kBins * P.W1, st);
        if (aux)
            scatter<true>(a, a.keys, a.vals, a.aux_in, nullptr, dim3(P.W1, 1), P.W1, P.shiftA, 255, a.k1, a.v1,
                          a.a1, st);
        else
            scatter<false>(a, a.keys, a.vals, nullptr, nullptr, dim3(P.W1, 1), P.W1, P.shiftA, 255, a.k1, a.v1,
                           a.a1, st);
        hipLaunchKernelGGL(k_extract_offsets, (P.binsA + 256) / 256, 256, 0, st, a.off, P.W1, 8u, P.binsA, n, a.offA);
        const uint32_t maskB = (1u << P.bitsB) - 1;
        count(a.k1, a.offA, dim3(P.W2, P.binsA), P.W2, 0, maskB);
        scan_matrix(a, (uint64_t)P.binsA * kBins * P.W2, st);
        if (aux)
            scatter<true>(a, a.k1, a.v1, a.a1, a.offA, dim3(P.W2, P.binsA), P.W2, 0, maskB, a.k2, a.v2, a.a2, st);
        else
            scatter<false>(a, a.k1, a.v1, nullptr, a.offA, dim3(P.W2, P.binsA), P.W2, 0, maskB, a.k2, a.v2, a.a2, st);
        hipLaunchKernelGGL(k_extract_offsets, (P.Q + 256) / 256, 256, 0, st, a.off, P.W2, P.bitsB, P.Q, n, a.offQ);
        o.keys = a.k2;
        o.vals = a.v2;
        o.aux = a.a2;
        o.aux_is_pos = aux ? 0 : 1;
    } else {
        // top 8 bits into k1, the middle 8 bits within each first-level bin into k2, the
        // low bits within each second-level bin back into k1
        count(a.keys, nullptr, dim3(P.W1, 1), P.W1, P.shiftA, 255);
        scan_matrix(a, (uint64_t)kBins * P.W1, st);
        if (aux)
            scatter<true>(a, a.keys, a.vals, a.aux_in, nullptr, dim3(P.W1, 1), P.W1, P.shiftA, 255, a.k1, a.v1,
                          a.a1, st);
        else
            scatter<false>(a, a.keys, a.vals, nullptr, nullptr, dim3(P.W1, 1), P.W1, P.shiftA, 255, a.k1, a.v1,
                           a.a1, st);
        hipLaunchKernelGGL(k_extract_offsets, (P.binsA + 256) / 256, 256, 0, st, a.off, P.W1, 8u, P.binsA, n, a.offA);
        count(a.k1, a.offA, dim3(P.W2, P.binsA), P.W2, P.bitsC, 255);
        scan_matrix(a, (uint64_t)P.binsA * kBins * P.W2, st);
        if (aux)
            scatter<true>(a, a.k1, a.v1, a.a1, a.offA, dim3(P.W2, P.binsA), P.W2, P.bitsC, 255, a.k2, a.v2, a.a2, st);
        else
            scatter<false>(a, a.k1, a.v1, nullptr, a.offA, dim3(P.W2, P.binsA), P.W2, P.bitsC, 255, a.k2, a.v2,
                           a.a2, st);
        hipLaunchKernelGGL(k_extract_offsets, (P.binsAB + 256) / 256, 256, 0, st, a.off, P.W2, 8u, P.binsAB, n,
                           a.offAB);
        const uint32_t maskC = (1u << P.bitsC) - 1;
        count(a.k2, a.offAB, dim3(P.W3, P.binsAB), P.W3, 0, maskC);
        scan_matrix(a, (uint64_t)P.binsAB * kBins * P.W3, st);
        if (aux)
            scatter<true>(a, a.k2, a.v2, a.a2, a.offAB, dim3(P.W3, P.binsAB), P.W3, 0, maskC, a.k1, a.v1, a.a1, st);
        else
            scatter<false>(a, a.k2, a.v2, nullptr, a.offAB, dim3(P.W3, P.binsAB), P.W3, 0, maskC, a.k1, a.v1,
                           nullptr, st);
        hipLaunchKernelGGL(k_extract_offsets, (P.Q + 256) / 256, 256, 0, st, a.off, P.W3, P.bitsC, P.Q, n, a.offQ);
        o.keys = a.k1;
        o.vals = a.v1;
        o.aux = a.a1;
        o.aux_is_pos = aux ? 0 : 1;
    }
    if (a.fused) {
        // the fused final pass sizes the partitions and finds their cell bases itself
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? FKS_OK : hip_fail(e);
    }
    FKS_TIMED("fks_part_sizes", st,
              hipLaunchKernelGGL(k_psizes, P.Q, kPB, 0, st, o.keys, n, a.A, a.magic, a.offQ, a.sizes, a.G, a.sqQ,
                                 a.oversize));
    {
        // cell bases of the partitions (exclusive scan of their sums of squares) and S
        const uint32_t nt = (uint32_t)exscan_tiles(P.Q);
        hipLaunchKernelGGL(k_xscan_reduce, nt, kPB, 0, st, a.sqQ, (uint64_t)P.Q, a.tsum);
        hipLaunchKernelGGL(k_scan_counts, 1, 1024, 0, st, a.tsum, nt, a.tpre, nullptr, a.S_dev);
        hipLaunchKernelGGL(k_xscan_down64, nt, kPB, 0, st, a.sqQ, (uint64_t)P.Q, a.tpre, a.cbase);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

template <bool AUX, bool STR>
static void launch_fused(const PartArgs& a, const PartOut& o, const Triple* C, uint32_t T, Group* header, Cell* slots,
                         uint32_t* flags, const int64_t* ctx_off, const uint8_t* ctx_bytes, const uint32_t* reject,
                         uint64_t cap, hipStream_t st) {
    const uint32_t Q = o.plan.Q;
    // the look-back words (in the cell-base scratch) and the ticket (in the partition-sum
    // scratch) start at zero (the cursor passes' set-up has cleared them already)
    if (!o.prezeroed) {
        hipLaunchKernelGGL(k_zero_words, (2 * Q + 255) / 256, 256, 0, st, reinterpret_cast<uint32_t*>(a.cbase),
                           (uint64_t)2 * Q);
        hipLaunchKernelGGL(k_zero_words, 1, 64, 0, st, a.sqQ, (uint64_t)1);
    }
    const FuseArgs fa{a.cbase, a.sqQ, a.S_dev, a.oversize, a.stalled, Q, o.qend, o.qcap};
    FKS_TIMED("fks_part_final", st,
              hipLaunchKernelGGL((k_pfinal<AUX, STR, false, true>), Q, kPB, 0, st, o.keys, o.vals,
                                 AUX ? o.aux : nullptr, AUX ? o.aux_is_pos : 1, a.n, a.A, a.magic, o.qbeg, a.cbase,
                                 a.sizes, a.G, C, T, header, slots, flags, ctx_off, ctx_bytes, nullptr, nullptr,
                                 reject, cap, fa));
}

int part_finish(const PartArgs& a, PartOut& o, const Triple* C, uint32_t T, Group* header, Cell* slots,
                uint32_t* flags, const int64_t* ctx_off, const uint8_t* ctx_bytes, const uint8_t* given_t,
                const uint32_t* reject, uint64_t cap, hipStream_t st) {
    if (a.fused && !given_t) {
        if (a.aux && a.str)
            launch_fused<true, true>(a, o, C, T, header, slots, flags, ctx_off, ctx_bytes, reject, cap, st);
        else if (a.aux)
            launch_fused<true, false>(a, o, C, T, header, slots, flags, nullptr, nullptr, reject, cap, st);
        else
            launch_fused<false, false>(a, o, C, T, header, slots, flags, nullptr, nullptr, reject, cap, st);
        o.prezeroed = false;   // the look-back words are used up: a second run clears them again
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? FKS_OK : hip_fail(e);
    }
    if (a.aux && a.str)
        FKS_TIMED("fks_part_final", st,
                  hipLaunchKernelGGL((k_pfinal<true, true>), o.plan.Q, kPB, 0, st, o.keys, o.vals,
                                     o.aux, o.aux_is_pos, a.n, a.A, a.magic, a.offQ, a.cbase, a.sizes, a.G, C, T,
                                     header, slots, flags, ctx_off, ctx_bytes, given_t, nullptr, reject, cap));
    else if (a.aux)
        FKS_TIMED("fks_part_final", st,
                  hipLaunchKernelGGL((k_pfinal<true, false>), o.plan.Q, kPB, 0, st, o.keys, o.vals,
                                     o.aux, o.aux_is_pos, a.n, a.A, a.magic, a.offQ, a.cbase, a.sizes, a.G, C, T,
                                     header, slots, flags, nullptr, nullptr, given_t, nullptr, reject, cap));
    else
        FKS_TIMED("fks_part_final", st,
                  hipLaunchKernelGGL((k_pfinal<false, false>), o.plan.Q, kPB, 0, st, o.keys, o.vals,
                                     nullptr, 1, a.n, a.A, a.magic, a.offQ, a.cbase, a.sizes, a.G, C, T, header,
                                     slots, flags, nullptr, nullptr, given_t, nullptr, reject, cap));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

}  // namespace fks

namespace fks {

// scratch of wide_build: partitioned keys and values, count matrix and its scan,
// partition offsets, sums of squares and size words
static size_t wide_layout(uint64_t nkeys, uint32_t nseg, uint32_t W, size_t* at) {
    const uint64_t Q = (uint64_t)nseg * kSegParts, N = (uint64_t)nseg * kBins * W;
    const uint64_t tiles = exscan_tiles(std::max<uint64_t>(N, Q));
    const size_t sz[8] = {8 * nkeys, 4 * nkeys, 4 * N, 4 * N, 4 * tiles, 8 * (tiles + 1), 8 * (Q + 1),
                          4 * Q + 4 * Q * kGroupsPerPart};
    size_t total = 0;
    for (int i = 0; i < 8; ++i) {
        if (at) at[i] = total;
        total += (sz[i] + 255) & ~(size_t)255;
    }
    return total;
}

size_t wide_scratch_bytes(uint64_t nkeys, uint32_t nseg, uint32_t W) { return wide_layout(nkeys, nseg, W, nullptr); }

int wide_build(const uint64_t* d_keys, const uint32_t* d_vals, const WideSeg* segs, uint32_t nseg, uint64_t nkeys,
               uint32_t W, const Triple* Cpool, uint32_t T, Group* hdr_pool, Cell* slot_pool, uint32_t* flags,
               uint64_t* cbase, void* scratch, hipStream_t st) {
    if (nseg == 0) return FKS_OK;
    size_t at[8];
    wide_layout(nkeys, nseg, W, at);
    char* base = (char*)scratch;
    uint64_t* k2 = (uint64_t*)(base + at[0]);
    uint32_t* v2 = (uint32_t*)(base + at[1]);
    uint32_t* cnt = (uint32_t*)(base + at[2]);
    uint32_t* off = (uint32_t*)(base + at[3]);
    uint32_t* tsum = (uint32_t*)(base + at[4]);
    uint64_t* tpre = (uint64_t*)(base + at[5]);
    uint64_t* offQ = (uint64_t*)(base + at[6]);
    uint32_t* sqQ = (uint32_t*)(base + at[7]);
    uint32_t* sizes = sqQ + (uint64_t)nseg * kSegParts;
    const uint32_t Q = nseg * kSegParts;
    const uint64_t N = (uint64_t)nseg * kBins * W;
    const Triple A0{0, 0, 0};
    hipLaunchKernelGGL(k_zero_words, (4 * nseg + 255) / 256, 256, 0, st, flags, (uint64_t)4 * nseg);
    FKS_TIMED("fks_wide_count", st,
              hipLaunchKernelGGL(k_dcount, dim3(W, nseg), kPB, 0, st, d_keys, nkeys, A0, 0ull, nullptr, W, 0u,
                                 kSegParts - 1, cnt, segs));
    exscan_u32(cnt, N, tsum, tpre, off, st);
    FKS_TIMED("fks_wide_scatter", st,
              hipLaunchKernelGGL((k_dscatter<false, kPScatterItems, kPScatterThreads>), dim3(W, nseg),
                                 kPScatterThreads, 0, st, d_keys, d_vals,
                                 nullptr, nkeys, A0, 0ull, nullptr, W, 0u, kSegParts - 1, off, k2, v2, nullptr,
                                 segs));
    hipLaunchKernelGGL(k_extract_offsets, (Q + 256) / 256, 256, 0, st, off, W, 6u, Q, nkeys, offQ);
    FKS_TIMED("fks_wide_sizes", st,
              hipLaunchKernelGGL(k_psizes, Q, kPB, 0, st, k2, nkeys, A0, 0ull, offQ, sizes, 0ull, sqQ, flags,
                                 segs));
    hipLaunchKernelGGL(k_wbases, (nseg + 255) / 256, 256, 0, st, sqQ, segs, nseg, cbase, flags);
    FKS_TIMED("fks_wide_final", st,
              hipLaunchKernelGGL((k_pfinal<false, false, true>), Q, kPB, 0, st, k2, v2, nullptr, 1,
                                 nkeys, A0, 0ull, offQ, cbase, sizes, 0ull, Cpool, T, hdr_pool, slot_pool, flags,
                                 nullptr, nullptr, nullptr, segs));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

}  // namespace fks
