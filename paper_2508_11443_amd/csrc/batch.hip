// Batched construction of many independent maps in one persistent launch, and
// lookups of (map id, key) needles spread over them.
//
// Maps cannot be elements of arrays in the paper's setting (Section 3.2: that
// would make irregular arrays); here a batch is one more level of flattening
// above the buckets of Section 2.4: maps -> buckets -> keys.  Map m is built
// exactly as a single map would be with seed sigma_m = entry m of the batch
// seed's stream, so a map's table is the same whether it was built alone or
// in a batch.
//
// Schedule: a persistent grid of workgroups pulls maps from a queue ordered
// by decreasing size (largest first, so the long maps start early and the
// small ones fill the tail).  A workgroup runs the whole construction of its
// map: level-one histogram with LDS atomics on 4-bit counters, scan of the
// group statistics, counting-sort scatter into a global staging area (hot in
// L2/MALL for all but the largest maps), then chunks of BT buckets for the
// level-two search and the coalesced table write.  The workgroup size BT and
// the number of workgroups per CU are the tunable schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "fks_internal.hpp"
#include "partition.hpp"
#include "prof.hpp"

namespace fks {

constexpr uint32_t kBatchMaxN = 1u << 16;                  // keys per map in a batch
constexpr uint32_t kBatchMaxG = kBatchMaxN / 8;            // groups per map
constexpr uint32_t kBU = 4;                                // keys per thread in flight per pass

// What a lookup needs about map m (64 bytes, read per needle from L2).
struct alignas(64) LDesc {
    uint32_t n;          // 0 for failed maps: every needle is absent
    uint32_t T;
    uint64_t magic;
    Triple A;
    uint64_t hdr_off;    // first group record in the header pool
    uint64_t slot_off;   // first cell in the cell pool
};

// Build outcome of map m.
struct BDesc {
    uint64_t key_off;
    uint64_t hdr_off;
    uint64_t slot_off;
    uint64_t seed;
    uint32_t n;
    uint32_t S;
    uint32_t r;
    int32_t status;
    uint32_t max_t;
    uint32_t pad;
};

template <int BT>
struct BatchLds {
    uint32_t sizes[kBatchMaxG];
    Triple C[kTMax];
    Cell ent[2 * BT];
    uint16_t smap[8 * BT];
    uint32_t tsh[BT / 4];
    uint32_t wsum_a[BT / 64], wsum_b[BT / 64];
    uint32_t rng[4];
    uint64_t mag[16];   // remainder magic of s^2, s = 0..15
    uint32_t work, oversize, exhausted, dup, max_t, S;
};

// block-wide exclusive scan of two counters for BT threads
template <int BT>
__device__ inline void bexscan2(BatchLds<BT>& L, uint32_t& a, uint32_t& b, uint32_t& ta, uint32_t& tb) {
    uint32_t ia = a, ib = b;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t ua = __shfl_up(ia, d, 64), ub = __shfl_up(ib, d, 64);
        if (lane >= d) {
            ia += ua;
            ib += ub;
        }
    }
    if (lane == 63) {
        L.wsum_a[w] = ia;
        L.wsum_b[w] = ib;
    }
    __syncthreads();
    uint32_t pa = 0, pb = 0;
    ta = 0;
    tb = 0;
    for (int q = 0; q < BT / 64; ++q) {
        if (q < w) {
            pa += L.wsum_a[q];
            pb += L.wsum_b[q];
        }
        ta += L.wsum_a[q];
        tb += L.wsum_b[q];
    }
    a = pa + ia - a;
    b = pb + ib - b;
    __syncthreads();
}

__device__ inline bool bts4(uint64_t& m0, uint64_t& m1, uint64_t& m2, uint64_t& m3, uint32_t h) {
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

template <typename KeyAt>
__device__ inline uint32_t first_trial(const Triple* C, uint32_t T, uint32_t s, uint64_t M, KeyAt key_at) {
    const uint32_t s2 = s * s;
    if (s2 <= 64) {
        // up to 8 keys: one 64-bit occupancy mask in a register
        for (uint32_t t = 0; t < T; ++t) {
            const Triple c = C[t];
            uint64_t m = 0;
            bool collide = false;
            for (uint32_t i = 0; i < s; ++i) {
                const uint64_t bit = 1ull << fastmod(mshash(c, key_at(i)), M, s2);
                if (m & bit) {
                    collide = true;
                    break;
                }
                m |= bit;
            }
            if (!collide) return t;
        }
        return T;
    }
    for (uint32_t t = 0; t < T; ++t) {
        const Triple c = C[t];
        uint64_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
        bool collide = false;
        for (uint32_t i = 0; i < s; ++i) {
            if (bts4(m0, m1, m2, m3, fastmod(mshash(c, key_at(i)), M, s2))) {
                collide = true;
                break;
            }
        }
        if (!collide) return t;
    }
    return T;
}

template <int BT>
__global__ __launch_bounds__(BT) void k_batch_build(
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals, BDesc* __restrict__ bdesc,
    LDesc* __restrict__ ldesc, const uint32_t* __restrict__ order, uint32_t M, uint32_t* __restrict__ queue,
    uint32_t c, uint32_t T, uint32_t R, Triple* __restrict__ Cpool, Group* __restrict__ hdr_pool,
    Cell* __restrict__ slot_pool, uint8_t* __restrict__ rank_s, uint2* __restrict__ gscan_s,
    Cell* __restrict__ grouped_s) {
    __shared__ BatchLds<BT> L;
    const uint32_t tid = threadIdx.x;
    if (tid < 16) L.mag[tid] = tid ? fastmod_magic(tid * tid) : 0;   // published by the loop's first barrier
    for (;;) {
        if (tid == 0) L.work = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t w = L.work;
        __syncthreads();
        if (w >= M) break;
        const uint32_t mi = order[w];
        const BDesc D = bdesc[mi];
        const uint32_t n = D.n;
        const uint32_t G = (n + 7) / 8;
        const uint64_t ko = D.key_off, ho = D.hdr_off, so = D.slot_off;
        const uint64_t magic = n ? fastmod_magic(n) : 0;
        int32_t status = FKS_EBUILD;
        uint32_t acc_r = 0, acc_S = 0, acc_maxt = 0;
        Triple acc_A{0, 0, 0};
        if (n == 0) status = FKS_OK;
        for (uint32_t r = 0; r < R && n; ++r) {
            const Triple A = level1_triple(D.seed, r);
            for (uint32_t t = tid; t < T; t += BT) L.C[t] = level2_triple(D.seed, r, t);
            for (uint32_t g = tid; g < G; g += BT) L.sizes[g] = 0;
            if (tid == 0) {
                L.oversize = L.exhausted = L.dup = L.max_t = 0;
            }
            __syncthreads();
            // level-one histogram; the atomic's old value is the key's rank
            bool over = false;
            // kBU keys per thread are loaded before any is hashed, so their loads overlap
            for (uint32_t i0 = 0; i0 < n; i0 += kBU * BT) {
                uint64_t xs[kBU];
#pragma unroll
                for (uint32_t u = 0; u < kBU; ++u) {
                    const uint32_t i = i0 + u * BT + tid;
                    xs[u] = i < n ? keys[ko + i] : 0;
                }
#pragma unroll
                for (uint32_t u = 0; u < kBU; ++u) {
                    const uint32_t i = i0 + u * BT + tid;
                    if (i < n) {
                        const uint32_t j = fastmod(mshash(A, xs[u]), magic, n);
                        const uint32_t sh = 4 * (j & 7u);
                        const uint32_t old = atomicAdd(&L.sizes[j >> 3], 1u << sh);
                        const uint32_t rk = (old >> sh) & 15u;
                        over |= rk == 15u;
                        rank_s[ko + i] = (uint8_t)rk;
                    }
                }
            }
            if (over) atomicOr(&L.oversize, 1u);
            __syncthreads();
            const bool oversize = L.oversize != 0;
            __syncthreads();   // every thread has read the flag before anyone resets it
            if (oversize) continue;
            // scan of group statistics: each thread owns a run of consecutive groups
            const uint32_t per = (G + BT - 1) / BT;
            const uint32_t g0 = tid * per, g1 = min(G, g0 + per);
            uint32_t cnt = 0, sq = 0;
            for (uint32_t g = g0; g < g1; ++g) {
                const uint32_t sz = L.sizes[g];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint32_t s = nib(sz, k);
                    cnt += s;
                    sq += s * s;
                }
            }
            uint32_t tot_cnt, tot_sq;
            bexscan2<BT>(L, cnt, sq, tot_cnt, tot_sq);
            for (uint32_t g = g0; g < g1; ++g) {
                gscan_s[ho + g] = make_uint2(cnt, sq);
                const uint32_t sz = L.sizes[g];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint32_t s = nib(sz, k);
                    cnt += s;
                    sq += s * s;
                }
            }
            const uint32_t S = tot_sq;
            if ((uint64_t)S > (uint64_t)c * n) {
                __syncthreads();
                continue;
            }
            __syncthreads();
            // counting-sort scatter of the map's keys into its staging range
            for (uint32_t i0 = 0; i0 < n; i0 += kBU * BT) {
                uint64_t xs[kBU];
                uint32_t vs[kBU], rs[kBU];
#pragma unroll
                for (uint32_t u = 0; u < kBU; ++u) {
                    const uint32_t i = i0 + u * BT + tid;
                    xs[u] = i < n ? keys[ko + i] : 0;
                    vs[u] = i < n ? vals[ko + i] : 0;
                    rs[u] = i < n ? rank_s[ko + i] : 0;
                }
#pragma unroll
                for (uint32_t u = 0; u < kBU; ++u) {
                    const uint32_t i = i0 + u * BT + tid;
                    if (i < n) {
                        const uint32_t j = fastmod(mshash(A, xs[u]), magic, n);
                        const uint32_t g = j >> 3, kk = j & 7u;
                        const uint32_t pos = gscan_s[ho + g].x + prefix_cnt(L.sizes[g], kk) + rs[u];
                        Cell e;
                        e.key = xs[u];
                        e.val = vs[u];
                        e.aux = 0;
                        grouped_s[ko + pos] = e;
                    }
                }
            }
            __syncthreads();
            // level-two search and table write, BT buckets at a time.  The staged records
            // of consecutive chunks are contiguous, so the next chunk's 2*BT records (and
            // its group prefixes) are loaded while the current chunk is processed.
            Cell pre0{}, pre1{};
            auto prefetch = [&](uint32_t from) {
                const uint32_t a = from + tid, b = from + BT + tid;
                pre0 = a < n ? grouped_s[ko + a] : Cell{};
                pre1 = b < n ? grouped_s[ko + b] : Cell{};
            };
            prefetch(0);
            uint2 gs_next = (tid >> 3) < G ? gscan_s[ho + (tid >> 3)] : make_uint2(0, 0);
            for (uint32_t b0 = 0; b0 < n; b0 += BT) {
                const uint32_t j = b0 + tid;
                const uint32_t g = j >> 3, k = j & 7u;
                const uint2 gs = gs_next;
                {
                    const uint32_t gn = (b0 + BT + tid) >> 3;
                    gs_next = gn < G ? gscan_s[ho + gn] : make_uint2(0, 0);
                }
                uint32_t s = 0, kst, off;
                if (g < G) {
                    const uint32_t sz = L.sizes[g];
                    s = nib(sz, k);
                    kst = gs.x + prefix_cnt(sz, k);
                    off = gs.y + prefix_sq(sz, k);
                } else {
                    kst = n;
                    off = S;
                }
                if (tid == 0) {
                    L.rng[0] = kst;
                    L.rng[2] = off;
                }
                if (tid == BT - 1) {
                    L.rng[1] = kst + s;
                    L.rng[3] = off + s * s;
                }
                __syncthreads();
                const uint32_t K0 = L.rng[0], K1 = L.rng[1], Z0 = L.rng[2], Z1 = L.rng[3];
                const bool fast = (K1 - K0 <= 2u * BT) && (Z1 - Z0 <= 8u * BT);
                uint32_t t = 0;
                bool exhausted = false;
                const Cell* bk = grouped_s + ko + kst;
                uint64_t key0 = 0;   // the key of a one-key bucket
                if (fast) {
                    // this chunk's records come from the window prefetched at K0
                    if (tid < K1 - K0) L.ent[tid] = pre0;
                    if (BT + tid < K1 - K0) L.ent[BT + tid] = pre1;
                    prefetch(K1);
                    __syncthreads();
                    const uint32_t lk = kst - K0, lz = off - Z0, s2 = s * s;
                    if (s >= 2) {
                        t = first_trial(L.C, T, s, L.mag[s], [&](uint32_t i) { return L.ent[lk + i].key; });
                        exhausted = t == T;
                    }
                    if (s == 1) {
                        L.smap[lz] = (uint16_t)lk;   // a lone key owns its bucket's one cell
                        key0 = L.ent[lk].key;
                    } else if (s >= 2 && s <= 8 && !exhausted) {
                        // the cells of every key from registers; each cell is written once, the
                        // empty ones with the key of the lowest occupied cell (fill rule)
                        const Triple cc = L.C[t];
                        const uint64_t M = L.mag[s];
                        uint64_t occ = 0;
                        uint32_t lowest = s2, who = lk;
#pragma unroll
                        for (uint32_t i = 0; i < 8; ++i) {
                            if (i < s) {
                                const uint32_t h = fastmod(mshash(cc, L.ent[lk + i].key), M, s2);
                                occ |= 1ull << h;
                                L.smap[lz + h] = (uint16_t)(lk + i);
                                if (h < lowest) {
                                    lowest = h;
                                    who = lk + i;
                                }
                            }
                        }
                        for (uint32_t p = 0; p < s2; ++p)
                            if (!((occ >> p) & 1ull)) L.smap[lz + p] = (uint16_t)who;
                    } else if (s >= 1) {
                        if (!exhausted) {
                            for (uint32_t p = 0; p < s2; ++p) L.smap[lz + p] = 0xFFFFu;
                            const Triple cc = L.C[t];
                            for (uint32_t i = 0; i < s; ++i)
                                L.smap[lz + fastmod(mshash(cc, L.ent[lk + i].key), L.mag[s], s2)] = (uint16_t)(lk + i);
                            uint16_t first = 0;
                            for (uint32_t p = 0; p < s2; ++p)
                                if (L.smap[lz + p] != 0xFFFFu) {
                                    first = L.smap[lz + p];
                                    break;
                                }
                            for (uint32_t p = 0; p < s2; ++p)
                                if (L.smap[lz + p] == 0xFFFFu) L.smap[lz + p] = first;
                        } else {
                            for (uint32_t p = 0; p < s2; ++p) L.smap[lz + p] = (uint16_t)lk;
                        }
                    }
                    if (exhausted) {
                        bool dup = false;
                        for (uint32_t a = 0; a < s; ++a)
                            for (uint32_t b = a + 1; b < s; ++b) dup |= L.ent[lk + a].key == L.ent[lk + b].key;
                        atomicOr(&L.exhausted, 1u);
                        if (dup) atomicOr(&L.dup, 1u);
                    }
                    __syncthreads();
                    for (uint32_t p = tid; p < Z1 - Z0; p += BT) store_cell_once(slot_pool + so + Z0 + p, L.ent[L.smap[p]]);
                } else {
                    prefetch(K1);
                    if (s >= 2) {
                        t = first_trial(L.C, T, s, L.mag[s], [&](uint32_t i) { return bk[i].key; });
                        exhausted = t == T;
                    }
                    if (s == 1) key0 = bk[0].key;
                    const uint32_t s2 = s * s;
                    if (s >= 1 && !exhausted) {
                        const Triple cc = L.C[t];
                        uint32_t first_p = s2, first_i = 0;
                        for (uint32_t i = 0; i < s; ++i) {
                            const uint32_t h = mshash(cc, bk[i].key) % s2;
                            if (h < first_p) {
                                first_p = h;
                                first_i = i;
                            }
                        }
                        for (uint32_t p = 0; p < s2; ++p) {
                            uint32_t who = first_i;
                            for (uint32_t i = 0; i < s; ++i)
                                if (mshash(cc, bk[i].key) % s2 == p) who = i;
                            store_cell_once(slot_pool + so + off + p, bk[who]);
                        }
                    }
                    if (exhausted) {
                        bool dup = false;
                        for (uint32_t a = 0; a < s; ++a)
                            for (uint32_t b = a + 1; b < s; ++b) dup |= bk[a].key == bk[b].key;
                        atomicOr(&L.exhausted, 1u);
                        if (dup) atomicOr(&L.dup, 1u);
                    }
                }
                if (exhausted) t = 0;
                if (t) atomicMax(&L.max_t, t);
                // a one-key bucket's byte is its key's tag (its trial is 0)
                reinterpret_cast<uint8_t*>(L.tsh)[tid] = (uint8_t)(s == 1 ? key_tag(L.C[0], key0) : t);
                __syncthreads();
                if (tid < BT / 8) {
                    const uint32_t gg = b0 / 8 + tid;
                    if (gg < G) {
                        Group h;
                        h.base = gscan_s[ho + gg].y;
                        h.sizes = L.sizes[gg];
                        h.t_lo = L.tsh[2 * tid];
                        h.t_hi = L.tsh[2 * tid + 1];
                        const u32x4 hw = {h.base, h.sizes, h.t_lo, h.t_hi};
                        __builtin_nontemporal_store(hw, reinterpret_cast<u32x4*>(hdr_pool) + ho + gg);
                    }
                }
                __syncthreads();
            }
            const bool exhausted_any = L.exhausted != 0, dup_any = L.dup != 0;
            const uint32_t max_t = L.max_t;
            __syncthreads();   // flags read by all before the next attempt resets them
            if (exhausted_any) {
                if (dup_any) {
                    status = FKS_EDUPKEY;
                    break;
                }
                continue;
            }
            status = FKS_OK;
            acc_r = r;
            acc_S = S;
            acc_maxt = max_t;
            acc_A = A;
            for (uint32_t tt = tid; tt < T; tt += BT) Cpool[(uint64_t)mi * T + tt] = L.C[tt];
            break;
        }
        if (tid == 0) {
            BDesc out = D;
            out.status = status;
            out.r = acc_r;
            out.S = acc_S;
            out.max_t = acc_maxt;
            bdesc[mi] = out;
            LDesc ld;
            ld.n = status == FKS_OK ? n : 0u;
            ld.T = T;
            ld.magic = magic;
            ld.A = acc_A;
            ld.hdr_off = ho;
            ld.slot_off = so;
            ldesc[mi] = ld;
        }
        __syncthreads();
    }
}

// level-two triples of attempt 0 of every wide map
__global__ void k_wconsts(const WideSeg* __restrict__ segs, const BDesc* __restrict__ bdesc, uint32_t nseg,
                          uint32_t T, Triple* __restrict__ Cpool) {
    const uint64_t total = (uint64_t)nseg * T;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t m = segs[i / T].map, t = (uint32_t)(i % T);
        Cpool[(uint64_t)m * T + t] = level2_triple(bdesc[m].seed, 0, t);
    }
}

// outcome of every wide map: accepted at attempt 0, or left pending (status 1) for
// the per-workgroup kernel, which retries it from attempt 0 on
__global__ void k_wfinish(const WideSeg* __restrict__ segs, uint32_t nseg, const uint32_t* __restrict__ flags,
                          const uint64_t* __restrict__ cbase, uint32_t T, BDesc* __restrict__ bdesc,
                          LDesc* __restrict__ ldesc) {
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < nseg; b += gridDim.x * blockDim.x) {
        const WideSeg& sg = segs[b];
        if (flags[4 * b] != 0 || flags[4 * b + 1] != 0) continue;
        BDesc d = bdesc[sg.map];
        d.status = FKS_OK;
        d.r = 0;
        d.S = (uint32_t)cbase[(uint64_t)b * (kSegParts + 1) + kSegParts];
        d.max_t = flags[4 * b + 3];
        bdesc[sg.map] = d;
        LDesc ld;
        ld.n = sg.n;
        ld.T = T;
        ld.magic = sg.magic;
        ld.A = sg.A;
        ld.hdr_off = sg.hdr_off;
        ld.slot_off = sg.slot_off;
        ldesc[sg.map] = ld;
    }
}

template <bool WANT_VALS, bool WANT_FOUND>
__global__ __launch_bounds__(256) void k_batch_lookup(const LDesc* __restrict__ ldesc,
                                                        const Group* __restrict__ hdr_pool,
                                                        const Cell* __restrict__ slot_pool,
                                                        const Triple* __restrict__ Cpool, uint32_t M,
                                                        const uint32_t* __restrict__ ids,
                                                        const uint64_t* __restrict__ q, uint64_t m,
                                                        uint32_t* __restrict__ vals,
                                                        uint8_t* __restrict__ found, uint32_t missing) {
    constexpr int Q = 4;
    const uint64_t stride = (uint64_t)gridDim.x * 256 * Q;
    for (uint64_t base = (uint64_t)blockIdx.x * 256 * Q; base < m; base += stride) {
        uint64_t x[Q];
        uint32_t id[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const uint64_t i = base + threadIdx.x + (uint64_t)k * 256;
            x[k] = i < m ? q[i] : 0;
            id[k] = i < m ? ids[i] : 0xFFFFFFFFu;
        }
        LDesc d[Q];
        Group h[Q];
        uint32_t kk[Q], s[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            s[k] = 0;
            kk[k] = 0;
            if (id[k] < M) {
                d[k] = ldesc[id[k]];
                if (d[k].n) {
                    const uint32_t j = fastmod(mshash(d[k].A, x[k]), d[k].magic, d[k].n);
                    kk[k] = j & 7u;
                    h[k] = hdr_pool[d[k].hdr_off + (j >> 3)];
                    s[k] = nib(h[k].sizes, kk[k]);
                }
            }
        }
        Cell cl[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            uint32_t p;
            if (s[k]) s[k] = cell_of(h[k], kk[k], Cpool + (uint64_t)id[k] * d[k].T, x[k], p) ? 1u : 0u;
            if (s[k]) cl[k] = load_cell_once(slot_pool + d[k].slot_off + p);
        }
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const uint64_t i = base + threadIdx.x + (uint64_t)k * 256;
            if (i < m) {
                const bool hit = s[k] && cl[k].key == x[k];
                if (WANT_VALS) vals[i] = hit ? cl[k].val : missing;
                if (WANT_FOUND) found[i] = hit ? 1 : 0;
            }
        }
    }
}

__global__ void k_zero_u32(uint32_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

}  // namespace fks

// ---- host side ------------------------------------------------------------------------

struct fks_batch {
    int device;
    uint32_t M, c, T, R;
    uint64_t seed, total_keys, total_groups, pool_cells;
    fks::BDesc* bdesc;        // device
    fks::LDesc* ldesc;        // device
    fks::Triple* Cpool;       // device, M*T
    fks::Group* hdr_pool;     // device
    fks::Cell* slot_pool;     // device
    std::vector<fks::BDesc> host;   // outcome, copied back after the build
    uint64_t device_bytes;
    uint32_t schedule;
    fks_allocator alloc;    // where the pools came from (has_alloc == 0: the default pool)
    int has_alloc;
};

namespace fks {

// schedule id: bits 0..1 workgroup size (0: 256, 1: 512, 2: 1024), bits 4..7 workgroups per CU,
// bit 8: maps of at least kWideMin keys are built by the partition passes, all of them
// together, before the per-workgroup kernel builds the rest
constexpr uint32_t kScheduleWide = 0x100;
constexpr uint32_t kWideMin = 8192;
static bool decode_schedule(uint32_t sched, int& bt, int& per_cu) {
    const uint32_t b = sched & 3u;
    per_cu = (int)((sched >> 4) & 15u);
    if (b > 2 || per_cu < 1 || (sched & ~0x1F3u)) return false;
    bt = 256 << b;
    return true;
}

static std::mutex g_tune_mu;
static std::vector<std::pair<uint64_t, uint32_t>> g_tuned;   // (size-class key, schedule)

uint64_t batch_class_key(uint32_t M, uint64_t total) {
    // size class: log2 of the map count and of the mean map size
    uint32_t lm = 0, ls = 0;
    while ((1ull << (lm + 1)) <= M) ++lm;
    const uint64_t mean = M ? total / M : 0;
    while ((1ull << (ls + 1)) <= mean) ++ls;
    return ((uint64_t)lm << 32) | ls;
}

// wide maps through the partition passes, then 512 threads, 2 per CU
static uint32_t default_schedule() { return kScheduleWide | 1u | (2u << 4); }

// the per-workgroup kernel over the first `count` maps of d_order
static int launch_batch(fks_batch* B, const uint64_t* d_keys, const uint32_t* d_vals, const uint32_t* d_order,
                        uint32_t count, uint32_t* d_queue, uint8_t* rank_s, uint2* gscan_s, Cell* grouped_s,
                        uint32_t sched, hipStream_t st) {
    int bt = 256, per_cu = 3;
    if (!decode_schedule(sched, bt, per_cu)) return FKS_EINVAL;
    if (count == 0) return FKS_OK;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device);
    const unsigned grid = (unsigned)std::max(1, std::min<int>(cus * per_cu, (int)count));
    hipLaunchKernelGGL(k_zero_u32, 1, 64, 0, st, d_queue);
    switch (bt) {
        case 256:
            FKS_TIMED("fks_batch_build", st,
                      hipLaunchKernelGGL(k_batch_build<256>, grid, 256, 0, st, d_keys, d_vals, B->bdesc, B->ldesc,
                                         d_order, count, d_queue, B->c, B->T, B->R, B->Cpool, B->hdr_pool,
                                         B->slot_pool, rank_s, gscan_s, grouped_s));
            break;
        case 512:
            FKS_TIMED("fks_batch_build", st,
                      hipLaunchKernelGGL(k_batch_build<512>, grid, 512, 0, st, d_keys, d_vals, B->bdesc, B->ldesc,
                                         d_order, count, d_queue, B->c, B->T, B->R, B->Cpool, B->hdr_pool,
                                         B->slot_pool, rank_s, gscan_s, grouped_s));
            break;
        default:
            FKS_TIMED("fks_batch_build", st,
                      hipLaunchKernelGGL(k_batch_build<1024>, grid, 1024, 0, st, d_keys, d_vals, B->bdesc,
                                         B->ldesc, d_order, count, d_queue, B->c, B->T, B->R, B->Cpool,
                                         B->hdr_pool, B->slot_pool, rank_s, gscan_s, grouped_s));
            break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

static void batch_release(fks_batch* B, hipStream_t st) {
    dev_free(B->bdesc, st);
    dev_free(B->ldesc, st);
    dev_free(B->Cpool, st);
    dev_free(B->hdr_pool, st);
    dev_free(B->slot_pool, st);
    delete B;
}

}  // namespace fks

using namespace fks;

extern "C" int fks_build_batch_u64(const uint64_t* d_keys, const uint32_t* d_vals, const uint64_t* h_map_offsets,
                                   uint32_t M, uint64_t batch_seed, const fks_params* params, uint32_t schedule,
                                   const fks_allocator* alloc, void* stream, fks_batch** out) {
    if (!out || !h_map_offsets || M == 0 || !allocator_ok(alloc)) return FKS_EINVAL;
    fks_params P;
    fks_params_default(&P);
    if (params) P = *params;
    if (P.c < 1 || P.c > 16 || P.T < 1 || P.T > kTMax || P.R < 1 || P.R > 1024 || P.schedule != 0) return FKS_EINVAL;
    if (h_map_offsets[0] != 0) return FKS_EINVAL;
    uint64_t total = h_map_offsets[M];
    if (total && (!d_keys || !d_vals)) return FKS_EINVAL;
    if (total * P.c >= (1ull << 40)) return FKS_EINVAL;
    AllocScope scope(alloc);
    hipStream_t st = (hipStream_t)stream;
    fks_batch* B = new fks_batch;
    keep_allocator(alloc, B->alloc, B->has_alloc);
    B->M = M;
    B->c = P.c;
    B->T = P.T;
    B->R = P.R;
    B->seed = batch_seed;
    B->total_keys = total;
    (void)hipGetDevice(&B->device);
    B->host.resize(M);
    std::vector<uint32_t> sizes(M);
    uint64_t groups = 0;
    for (uint32_t m = 0; m < M; ++m) {
        if (h_map_offsets[m + 1] < h_map_offsets[m]) {
            delete B;
            return FKS_EINVAL;
        }
        const uint64_t n = h_map_offsets[m + 1] - h_map_offsets[m];
        if (n > kBatchMaxN) {
            delete B;
            return FKS_EINVAL;
        }
        BDesc& d = B->host[m];
        std::memset(&d, 0, sizeof(d));
        d.key_off = h_map_offsets[m];
        d.hdr_off = groups;
        d.slot_off = (uint64_t)P.c * h_map_offsets[m];
        d.seed = sm_out(batch_seed, m);
        d.n = (uint32_t)n;
        d.status = 1;
        sizes[m] = (uint32_t)n;
        groups += (n + 7) / 8;
    }
    B->total_groups = groups;
    B->pool_cells = (uint64_t)P.c * total;
    // largest maps first
    std::vector<uint32_t> order(M);
    for (uint32_t m = 0; m < M; ++m) order[m] = m;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return sizes[a] > sizes[b]; });

    B->bdesc = (BDesc*)dev_alloc(sizeof(BDesc) * M, st);
    B->ldesc = (LDesc*)dev_alloc(sizeof(LDesc) * M, st);
    B->Cpool = (Triple*)dev_alloc(sizeof(Triple) * (uint64_t)M * P.T, st);
    B->hdr_pool = (Group*)dev_alloc(16 * (groups ? groups : 1), st);
    B->slot_pool = (Cell*)dev_alloc(16 * (B->pool_cells ? B->pool_cells : 1), st);
    uint32_t* d_order = (uint32_t*)dev_alloc(4 * M + 256, st);
    uint32_t* d_queue = d_order ? d_order + M + (64 - (M % 64)) % 64 : nullptr;   // own cache line
    uint8_t* rank_s = (uint8_t*)dev_alloc(total ? total : 1, st);
    uint2* gscan_s = (uint2*)dev_alloc(8 * (groups ? groups : 1), st);
    Cell* grouped_s = (Cell*)dev_alloc(16 * (total ? total : 1), st);
    auto cleanup_scratch = [&]() {
        dev_free(d_order, st);
        dev_free(rank_s, st);
        dev_free(gscan_s, st);
        dev_free(grouped_s, st);
    };
    if (!B->bdesc || !B->ldesc || !B->Cpool || !B->hdr_pool || !B->slot_pool || !d_order || !rank_s ||
        !gscan_s || !grouped_s) {
        cleanup_scratch();
        batch_release(B, st);
        return FKS_ENOMEM;
    }
    B->device_bytes = sizeof(BDesc) * M + sizeof(LDesc) * M + sizeof(Triple) * (uint64_t)M * P.T + 16 * groups +
                      16 * B->pool_cells;
    hipError_t e = hipMemcpyAsync(B->bdesc, B->host.data(), sizeof(BDesc) * M, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_order, order.data(), 4 * M, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        cleanup_scratch();
        batch_release(B, st);
        return hip_fail(e);
    }
    uint32_t sched = schedule;
    if (sched == 0) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        sched = default_schedule();
        const uint64_t key = batch_class_key(M, total);
        for (auto& kv : g_tuned)
            if (kv.first == key) sched = kv.second;
    }
    B->schedule = sched;
    int rc = FKS_OK;
    int dummy_bt, dummy_cu;
    if (!decode_schedule(sched, dummy_bt, dummy_cu)) rc = FKS_EINVAL;
    uint32_t count = M;
    if (rc == FKS_OK && (sched & kScheduleWide)) {
        // large maps: attempt 0 of all of them by the partition passes; the order list then
        // holds only the small maps, and a large map that the passes reject follows below
        std::vector<WideSeg> segs;
        uint64_t wide_keys = 0;
        for (uint32_t m = 0; m < M; ++m) {
            const BDesc& d = B->host[m];
            if (d.n < kWideMin) continue;
            WideSeg sg;
            sg.A = level1_triple(d.seed, 0);
            sg.magic = fastmod_magic(d.n);
            sg.in_lo = d.key_off;
            sg.in_hi = d.key_off + d.n;
            sg.hdr_off = d.hdr_off;
            sg.slot_off = d.slot_off;
            sg.n = d.n;
            sg.G = (d.n + 7) / 8;
            sg.map = m;
            sg.c = P.c;
            segs.push_back(sg);
            wide_keys += d.n;
        }
        if (!segs.empty()) {
            const uint32_t nseg = (uint32_t)segs.size(), W = 2;
            WideSeg* d_segs = (WideSeg*)dev_alloc(sizeof(WideSeg) * nseg, st);
            uint32_t* d_flags = (uint32_t*)dev_alloc(16 * (size_t)nseg, st);
            uint64_t* d_cbase = (uint64_t*)dev_alloc(8 * (size_t)nseg * (kSegParts + 1), st);
            void* d_scratch = dev_alloc(wide_scratch_bytes(wide_keys, nseg, W), st);
            if (!d_segs || !d_flags || !d_cbase || !d_scratch) rc = FKS_ENOMEM;
            if (rc == FKS_OK) {
                e = hipMemcpyAsync(d_segs, segs.data(), sizeof(WideSeg) * nseg, hipMemcpyHostToDevice, st);
                if (e != hipSuccess) rc = hip_fail(e);
            }
            if (rc == FKS_OK) {
                hipLaunchKernelGGL(k_wconsts, (unsigned)std::min<uint64_t>(4096, ((uint64_t)nseg * P.T + 255) / 256),
                                   256, 0, st, d_segs, B->bdesc, nseg, P.T, B->Cpool);
                rc = wide_build(d_keys, d_vals, d_segs, nseg, wide_keys, W, B->Cpool, P.T, B->hdr_pool,
                                B->slot_pool, d_flags, d_cbase, d_scratch, st);
            }
            if (rc == FKS_OK) {
                hipLaunchKernelGGL(k_wfinish, (nseg + 255) / 256, 256, 0, st, d_segs, nseg, d_flags, d_cbase, P.T,
                                   B->bdesc, B->ldesc);
                e = hipGetLastError();
                if (e != hipSuccess) rc = hip_fail(e);
            }
            dev_free(d_segs, st);
            dev_free(d_flags, st);
            dev_free(d_cbase, st);
            dev_free(d_scratch, st);
        }
        if (rc == FKS_OK) {
            std::vector<uint32_t> small;
            for (uint32_t m : order)
                if (B->host[m].n < kWideMin) small.push_back(m);
            count = (uint32_t)small.size();
            e = hipMemcpyAsync(d_order, small.data(), 4 * (size_t)count, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);   // the small list is read before it goes out of scope
            if (e != hipSuccess) rc = hip_fail(e);
        }
    }
    if (rc == FKS_OK) rc = launch_batch(B, d_keys, d_vals, d_order, count, d_queue, rank_s, gscan_s, grouped_s, sched, st);
    if (rc == FKS_OK) {
        e = hipMemcpyAsync(B->host.data(), B->bdesc, sizeof(BDesc) * M, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e);
    }
    if (rc == FKS_OK && (sched & kScheduleWide)) {
        // large maps the partition passes left pending go through the per-workgroup kernel
        std::vector<uint32_t> pending;
        for (uint32_t m = 0; m < M; ++m)
            if (B->host[m].status == 1) pending.push_back(m);
        if (!pending.empty()) {
            e = hipMemcpyAsync(d_order, pending.data(), 4 * pending.size(), hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) rc = hip_fail(e);
            if (rc == FKS_OK)
                rc = launch_batch(B, d_keys, d_vals, d_order, (uint32_t)pending.size(), d_queue, rank_s, gscan_s,
                                  grouped_s, sched, st);
            if (rc == FKS_OK) {
                e = hipMemcpyAsync(B->host.data(), B->bdesc, sizeof(BDesc) * M, hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e != hipSuccess) rc = hip_fail(e);
            }
        }
    }
    // a map whose every attempt was rejected: equal keys make it a broken precondition
    for (uint32_t m = 0; rc == FKS_OK && m < M; ++m) {
        BDesc& d = B->host[m];
        if (d.status != FKS_EBUILD) continue;
        bool equal = false;
        rc = has_equal_keys(d_keys + d.key_off, d.n, nullptr, nullptr, st, &equal);
        if (rc == FKS_OK && equal) d.status = FKS_EDUPKEY;
    }
    cleanup_scratch();
    if (rc) {
        batch_release(B, st);
        return rc;
    }
    *out = B;
    return FKS_OK;
}

extern "C" int fks_batch_set_schedule(uint32_t M, uint64_t total_keys, uint32_t schedule) {
    int bt, per_cu;
    if (!decode_schedule(schedule, bt, per_cu)) return FKS_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const uint64_t key = batch_class_key(M, total_keys);
    for (auto& kv : g_tuned)
        if (kv.first == key) {
            kv.second = schedule;
            return FKS_OK;
        }
    g_tuned.emplace_back(key, schedule);
    return FKS_OK;
}

extern "C" int fks_batch_schedules(uint32_t* out, int max_entries) {
    // every valid schedule: 256/512/1024 threads, 1..4 workgroups per CU within the LDS budget,
    // with and without the partition passes for the large maps
    static const uint32_t all[] = {0x10,  0x20,  0x30,  0x11,  0x21,  0x12,
                                   0x110, 0x120, 0x130, 0x111, 0x121, 0x112};
    const int n = (int)(sizeof(all) / sizeof(all[0]));
    if (!out) return n;
    int k = 0;
    for (; k < n && k < max_entries; ++k) out[k] = all[k];
    return k;
}

extern "C" int fks_batch_status(const fks_batch* B, int32_t* h_status, uint32_t* h_r, uint32_t* h_S) {
    if (!B) return FKS_EINVAL;
    for (uint32_t m = 0; m < B->M; ++m) {
        if (h_status) h_status[m] = B->host[m].status;
        if (h_r) h_r[m] = B->host[m].r;
        if (h_S) h_S[m] = B->host[m].S;
    }
    return FKS_OK;
}

extern "C" int fks_batch_info(const fks_batch* B, uint32_t map_index, fks_map_info* info) {
    if (!B || !info || map_index >= B->M) return FKS_EINVAL;
    const BDesc& d = B->host[map_index];
    std::memset(info, 0, sizeof(*info));
    info->n = d.n;
    info->S = d.status == FKS_OK ? d.S : 0;
    info->header_bytes = 16 * ((uint64_t)(d.n + 7) / 8);
    info->slot_bytes = 16 * (uint64_t)info->S;
    info->seed = d.seed;
    info->r = d.r;
    info->kind = 0;
    info->c = B->c;
    info->T = B->T;
    info->R = B->R;
    info->max_t = d.max_t;
    info->device_bytes = B->device_bytes;
    if (d.status != FKS_OK) return d.status;
    int prev = 0;
    FKS_HIP(hipGetDevice(&prev));
    FKS_HIP(hipSetDevice(B->device));
    const int rc = size_histogram(B->hdr_pool + d.hdr_off, d.n, info->size_hist);
    (void)hipSetDevice(prev);
    return rc;
}

extern "C" int fks_batch_export(const fks_batch* B, uint32_t map_index, void* h_header, void* h_slots,
                                uint64_t* h_consts) {
    if (!B || map_index >= B->M) return FKS_EINVAL;
    const BDesc& d = B->host[map_index];
    if (d.status != FKS_OK) return d.status;
    FKS_HIP(hipDeviceSynchronize());
    const uint64_t hb = 16 * ((uint64_t)(d.n + 7) / 8);
    if (h_header && hb) FKS_HIP(hipMemcpy(h_header, B->hdr_pool + d.hdr_off, hb, hipMemcpyDeviceToHost));
    if (h_slots && d.S)
        FKS_HIP(hipMemcpy(h_slots, B->slot_pool + d.slot_off, 16 * (uint64_t)d.S, hipMemcpyDeviceToHost));
    if (h_consts)
        FKS_HIP(hipMemcpy(h_consts, B->Cpool + (uint64_t)map_index * B->T, sizeof(Triple) * B->T,
                          hipMemcpyDeviceToHost));
    return FKS_OK;
}

extern "C" int fks_lookup_batch_u64(const fks_batch* B, const uint32_t* d_map_ids, const uint64_t* d_queries,
                                    uint64_t m, uint32_t* d_vals_out, uint8_t* d_found_out, uint32_t missing,
                                    void* stream) {
    if (!B || (m && (!d_map_ids || !d_queries))) return FKS_EINVAL;
    if (m == 0 || (!d_vals_out && !d_found_out)) return FKS_OK;
    hipStream_t st = (hipStream_t)stream;
    uint64_t g = (m + 1023) / 1024;
    if (g > 65536) g = 65536;
    const unsigned grid = (unsigned)g;
    if (d_vals_out && d_found_out)
        FKS_TIMED("fks_lookup_batch_u64", st,
                  hipLaunchKernelGGL((k_batch_lookup<true, true>), grid, 256, 0, st, B->ldesc, B->hdr_pool,
                                     B->slot_pool, B->Cpool, B->M, d_map_ids, d_queries, m, d_vals_out,
                                     d_found_out, missing));
    else if (d_vals_out)
        FKS_TIMED("fks_lookup_batch_u64", st,
                  hipLaunchKernelGGL((k_batch_lookup<true, false>), grid, 256, 0, st, B->ldesc, B->hdr_pool,
                                     B->slot_pool, B->Cpool, B->M, d_map_ids, d_queries, m, d_vals_out,
                                     d_found_out, missing));
    else
        FKS_TIMED("fks_lookup_batch_u64", st,
                  hipLaunchKernelGGL((k_batch_lookup<false, true>), grid, 256, 0, st, B->ldesc, B->hdr_pool,
                                     B->slot_pool, B->Cpool, B->M, d_map_ids, d_queries, m, d_vals_out,
                                     d_found_out, missing));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

extern "C" void fks_batch_destroy(fks_batch* B) {
    if (!B) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(B->device);
    {
        AllocScope scope(B->has_alloc ? &B->alloc : nullptr);
        batch_release(B, nullptr);
    }
    (void)hipSetDevice(prev);
}
