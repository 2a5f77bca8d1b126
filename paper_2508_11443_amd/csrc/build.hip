// Data-parallel construction of the two-level hash map (Sections 2.2-2.5):
// the host driver of the level-one attempts.
//
// One attempt r runs the partition passes of partition.hip on the stream:
// every key's bucket g k = hash(A_r) k mod n (make_1, Section 2.3) decides its
// partition of 1024 consecutive buckets; one to three radix passes group the
// records by partition; a per-partition histogram gives the bucket sizes and
// the partition's sum of squared sizes, and their exclusive scan the table size
// S = sum s^2 (the offsets of Section 2.2); then one workgroup per partition
// searches level two (make_2) and writes the cells and group headers into cells
// allocated from a bound on S.  The host reads the attempt's outcome once:
// S <= c*n, no bucket above 15 keys, every bucket separated (and S within the
// bound, else the final pass runs again into an exact allocation).
// String maps first fingerprint every key with the attempt's base and run the
// same steps on the fingerprints.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>
#include <vector>

#include "fks_internal.hpp"
#include "partition.hpp"
#include "prof.hpp"
#include "rounds.hpp"

namespace fks {

constexpr int kBlock = 256;

// control words of one attempt (device), read back through Readback
struct Ctrl {
    uint64_t S;
    uint32_t oversize, bad_input, exhausted, dup, max_t, stalled, overflow, pad;   // same layout as Readback
};
static_assert(sizeof(Ctrl) == sizeof(Readback), "read back as one block");
// the final pass reads its two reject words from &oversize
static_assert(offsetof(Ctrl, bad_input) == offsetof(Ctrl, oversize) + sizeof(uint32_t), "adjacent reject words");
// the final pass updates three outcome words from &exhausted
static_assert(offsetof(Ctrl, max_t) == offsetof(Ctrl, exhausted) + 2 * sizeof(uint32_t), "adjacent outcome words");

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t count, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_split_u64(const uint64_t* __restrict__ v, uint64_t n, uint32_t* __restrict__ lo,
                            uint32_t* __restrict__ hi) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = v[i];
        lo[i] = (uint32_t)x;
        hi[i] = (uint32_t)(x >> 32);
    }
}

__global__ void k_zero_ctrl(Ctrl* c) {
    if (threadIdx.x == 0) {
        c->S = 0;
        c->oversize = c->bad_input = c->exhausted = c->dup = c->max_t = c->stalled = c->overflow = c->pad = 0;
    }
}

// an attempt's start: the outcome words cleared and the attempt's T level-two triples
// written from the seed (the same stream the host draws them from)
__global__ void k_attempt_setup(Ctrl* c, Triple* C, uint64_t seed, uint32_t r, uint32_t T) {
    if (threadIdx.x == 0) {
        c->S = 0;
        c->oversize = c->bad_input = c->exhausted = c->dup = c->max_t = c->stalled = c->overflow = c->pad = 0;
    }
    for (uint32_t t = threadIdx.x; t < T; t += blockDim.x) C[t] = level2_triple(seed, r, t);
}

// ---- string fingerprints -----------------------------------------------------

// One lane per string.  Offsets are checked here, before any byte is read through them:
// a pair outside [0, nbytes] or decreasing sets bad_input and reads nothing.
__global__ __launch_bounds__(kBlock) void k_fingerprint(const int64_t* __restrict__ off,
                                                          const uint8_t* __restrict__ bytes, uint64_t nbytes,
                                                          uint64_t n, uint64_t beta, uint64_t* __restrict__ y,
                                                          Ctrl* ctrl) {
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t a = off[i], b = off[i + 1];
        if (a < 0 || b < a || (uint64_t)b > nbytes) {
            bad = true;
            y[i] = 0;
            continue;
        }
        uint32_t w[kChunkWords];
        y[i] = fingerprint_words(bytes + a, (uint64_t)(b - a), beta, w);
    }
    if (bad) atomicOr(&ctrl->bad_input, 1u);
}

// ---- host driver ------------------------------------------------------------------------

static unsigned grid_for(uint64_t items, uint64_t per_block, unsigned cap = 1u << 30) {
    uint64_t g = (items + per_block - 1) / per_block;
    if (g == 0) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

struct Scratch {
    uint64_t* y = nullptr;       // fingerprints (string maps)
    Ctrl* ctrl = nullptr;
    Readback* host = nullptr;    // pinned
};

static void free_scratch(Scratch& w, hipStream_t st) {
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

// Cells allocated before an attempt's final pass, which is launched without waiting for
// the attempt's S (no host round trip between the size pass and the final pass).  S is
// the sum of the squared bucket sizes; with n keys hashed into n buckets the sizes are
// close to Poisson(1), so S has mean 2n - 1 and variance about 11n (the
// fourth moment of Poisson(1) is 15).  Eight standard deviations above the mean hold it
// but for a negligible fraction of builds; a larger S costs one more final pass into an
// exact allocation.  More than c*n cells are never needed: such an attempt is rejected.
static uint64_t cells_guess(uint64_t n, uint32_t c) {
    const uint64_t g = 2 * n + (uint64_t)(8.0 * std::sqrt(11.0 * (double)n)) + 64;
    const uint64_t lim = (uint64_t)c * n;
    return g < lim ? g : lim;
}

// Level-one attempts with the partitioned passes (partition.hip).
// d_aux_in: the high halves of 64-bit values (kind 2), else nullptr.
static int attempts_partitioned(fks_map* M, const uint64_t* d_keys_in, const uint32_t* d_vals,
                                const uint32_t* d_aux_in, const fks_params& P, Ctrl* ctrl, Readback* host,
                                uint64_t* y, hipStream_t st) {
    const uint64_t n = M->n;
    const uint64_t G = (n + 7) / 8;
    const bool bytes = M->kind == 1;
    const bool carry = bytes || M->kind == 2;
    // the per-bucket schedule runs the final pass straight after the size pass, into cells
    // allocated from a bound on S; the paper's rounds need S on the host before their search
    const bool direct = P.schedule == 0;
    const PartPlan plan = part_plan(n);
    const uint32_t Q = plan.Q;
    PartArgs a{};
    a.n = n;
    a.G = G;
    a.aux = carry;
    a.str = bytes;
    a.aux_in = d_aux_in;
    a.vals = d_vals;
    // scratch, carved from one allocation (one allocation and one release per build), freed
    // when the attempts are over; buffers allocated later (the rounds schedule's trials) join
    // the owned list
    std::vector<void*> owned;
    Cell* slots = nullptr;   // direct form: the cells, kept across attempts
    uint64_t cap = 0;
    auto release = [&]() {
        for (void* p : owned) dev_free(p, st);
        owned.clear();
    };
    size_t total = 0;
    auto carve = [&](size_t bytes_) {   // first pass sizes, second pass hands out addresses
        const size_t at = total;
        total += (bytes_ + 255) & ~(size_t)255;
        return at;
    };
    // one or two passes in the direct form reserve their runs on cursors: the records then sit
    // in fixed-capacity regions (binsA of them after a first of two passes, Q after the last)
    const bool cursor = direct && (plan.passes == 1 || plan.passes == 2);
    const uint64_t r1 = cursor ? std::max<uint64_t>(n, plan.cap1 * plan.binsA) : n;
    const uint64_t r2 = cursor ? std::max<uint64_t>(n, plan.capQ * Q) : n;
    const size_t o_k1 = plan.passes >= 2 ? carve(8 * r1) : 0, o_v1 = plan.passes >= 2 ? carve(4 * r1) : 0;
    const size_t o_a1 = plan.passes >= 2 && carry ? carve(4 * r1) : 0;
    const size_t o_k2 = plan.passes >= 1 ? carve(8 * r2) : 0, o_v2 = plan.passes >= 1 ? carve(4 * r2) : 0;
    const size_t o_a2 = plan.passes >= 1 && carry ? carve(4 * r2) : 0;
    const size_t o_cur1 = cursor ? carve(8 * (size_t)plan.binsA) : 0, o_cur2 = cursor ? carve(8 * (size_t)Q) : 0;
    const size_t o_begA = cursor ? carve(8 * (size_t)plan.binsA) : 0, o_begQ = cursor ? carve(8 * (size_t)Q) : 0;
    const size_t o_cnt = carve(4 * plan.matrix), o_off = carve(4 * plan.matrix);
    const size_t o_tsum = carve(4 * part_scan_tiles(plan)), o_tpre = carve(8 * (part_scan_tiles(plan) + 1));
    const size_t o_offA = carve(8 * 257), o_offQ = carve(8 * ((size_t)Q + 1)), o_sqQ = carve(4 * (size_t)Q);
    const size_t o_offAB = plan.passes == 3 ? carve(8 * ((size_t)plan.binsAB + 1)) : 0;
    const size_t o_cbase = carve(8 * ((size_t)Q + 1)), o_sizes = carve(4 * (size_t)Q * (kPartBuckets / 8));
    char* base = nullptr;
    // points the passes' buffers into the scratch at base
    auto attach_scratch = [&]() {
        if (plan.passes >= 2) {
            a.k1 = (uint64_t*)(base + o_k1);
            a.v1 = (uint32_t*)(base + o_v1);
            if (carry) a.a1 = (uint32_t*)(base + o_a1);
        }
        if (plan.passes >= 1) {
            a.k2 = (uint64_t*)(base + o_k2);
            a.v2 = (uint32_t*)(base + o_v2);
            if (carry) a.a2 = (uint32_t*)(base + o_a2);
        }
        a.cnt = (uint32_t*)(base + o_cnt);
        a.off = (uint32_t*)(base + o_off);
        a.tsum = (uint32_t*)(base + o_tsum);
        a.tpre = (uint64_t*)(base + o_tpre);
        a.offA = (uint64_t*)(base + o_offA);
        if (plan.passes == 3) a.offAB = (uint64_t*)(base + o_offAB);
        a.offQ = (uint64_t*)(base + o_offQ);
        a.sqQ = (uint32_t*)(base + o_sqQ);
        a.cbase = (uint64_t*)(base + o_cbase);
        a.sizes = (uint32_t*)(base + o_sizes);
        if (cursor) {
            a.cur1 = (unsigned long long*)(base + o_cur1);
            a.cur2 = (unsigned long long*)(base + o_cur2);
            a.begA = (uint64_t*)(base + o_begA);
            a.begQ = (uint64_t*)(base + o_begQ);
        }
    };
    // (re)takes the scratch and points the passes' buffers into it
    auto ensure_scratch = [&]() {
        if (base) return true;
        base = (char*)dev_alloc(total, st);
        if (!base) return false;
        owned.push_back(base);
        attach_scratch();
        return true;
    };
    auto release_scratch = [&]() {
        release();
        base = nullptr;
    };
    if (!ensure_scratch()) return FKS_ENOMEM;
    // with the device's default pool the scratch goes back, in stream order, as soon as its
    // last reader (the final pass) is queued: the host's wait for the outcome then ends the
    // call with nothing left to release.  The rare second pass or attempt takes it again.
    const bool early_release = direct && dev_pool_default();
    a.overflow = &ctrl->overflow;
    a.S_dev = &ctrl->S;
    a.oversize = &ctrl->oversize;
    a.stalled = &ctrl->stalled;
    // the direct form runs the fused final pass: it sizes the partitions itself
    a.fused = direct;
    a.cursor = cursor;
    const uint32_t* const reject = &ctrl->oversize;   // followed by bad_input
    if (direct) {
        cap = cells_guess(n, P.c);
        slots = (Cell*)dev_alloc(16 * cap, st);
        if (!slots) {
            release();
            return FKS_ENOMEM;
        }
    }
    auto drop_slots = [&]() {
        dev_free(slots, st);
        slots = nullptr;
    };
    auto readback = [&]() {
        hipError_t e = hipMemcpyAsync(host, ctrl, sizeof(Readback), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        return e == hipSuccess ? FKS_OK : hip_fail(e);
    };
    int rc = FKS_OK;
    for (uint32_t r = 0; r < P.R; ++r) {
        const Triple A = level1_triple(M->seed, r);
        const uint64_t beta = level1_beta(M->seed, r);
        a.A = A;
        a.magic = M->magic_n;
        a.keys = d_keys_in;
        hipLaunchKernelGGL(k_attempt_setup, 1, 256, 0, st, ctrl, M->C, M->seed, r, P.T);
        if (bytes) {
            FKS_TIMED("fks_fingerprint", st,
                      hipLaunchKernelGGL(k_fingerprint, grid_for(n, kBlock, 65536), kBlock, 0, st, M->ctx_off,
                                         M->ctx_bytes, M->ctx_nbytes, n, beta, y, ctrl));
            a.keys = y;
        }
        if (!ensure_scratch()) {
            rc = FKS_ENOMEM;
            break;
        }
        PartOut o;
        if ((rc = part_prepare(a, st, o))) break;
        if (direct) {
            // the final pass follows the size pass without a host round trip; the host waits
            // once per attempt, for the outcome
            if ((rc = part_finish(a, o, M->C, P.T, M->header, slots, &ctrl->exhausted, M->ctx_off, M->ctx_bytes,
                                  nullptr, reject, cap, st)))
                break;
            if (early_release) release_scratch();
            if ((rc = readback())) break;
            if (host->bad_input) {
                rc = FKS_EINVAL;
                break;
            }
            if (host->stalled) {
                rc = hip_fail(hipErrorLaunchFailure);
                break;
            }
            if (host->overflow) {
                // a region of the cursor passes overflowed (keys far from uniform over the
                // partitions): the same attempt again with counted passes
                a.cursor = false;
                --r;
                continue;
            }
            if (host->oversize) continue;
            const uint64_t S = host->S;
            if (S > (uint64_t)P.c * n) continue;
            if (S > cap) {
                // more cells than the guess: the same pass again into an exact allocation
                drop_slots();
                cap = S;
                slots = (Cell*)dev_alloc(16 * cap, st);
                if (!slots) {
                    rc = FKS_ENOMEM;
                    break;
                }
                hipLaunchKernelGGL(k_zero_ctrl, 1, 64, 0, st, ctrl);
                if (!base) {
                    // the scratch went back early: the partition passes run again into it
                    if (!ensure_scratch()) {
                        rc = FKS_ENOMEM;
                        break;
                    }
                    if ((rc = part_prepare(a, st, o))) break;
                }
                if ((rc = part_finish(a, o, M->C, P.T, M->header, slots, &ctrl->exhausted, M->ctx_off,
                                      M->ctx_bytes, nullptr, reject, cap, st)))
                    break;
                if (early_release) release_scratch();
                if ((rc = readback())) break;
            }
            if (host->exhausted) {
                if (host->dup) {
                    rc = FKS_EDUPKEY;
                    break;
                }
                continue;
            }
            M->slots = slots;
            slots = nullptr;
            M->S = S;
            M->r = r;
            M->A = A;
            M->beta = beta;
            M->max_t = host->max_t;
            M->device_bytes += 16 * cap;
            release();
            return FKS_OK;
        }
        if ((rc = readback())) break;
        if (host->bad_input) {
            rc = FKS_EINVAL;
            break;
        }
        if (host->oversize) continue;
        const uint64_t S = host->S;
        if (S > (uint64_t)P.c * n) continue;
        Cell* cells = (Cell*)dev_alloc(16 * (S ? S : 1), st);
        if (!cells) {
            rc = FKS_ENOMEM;
            break;
        }
        const uint8_t* given_t = nullptr;
        if (P.schedule == 1) {
            // the paper's flattened rounds decide every bucket's trial; the table
            // write below then only places the keys
            uint8_t* tb = (uint8_t*)dev_alloc(4 * ((n + 3) / 4), st);
            if (!tb) {
                dev_free(cells, st);
                rc = FKS_ENOMEM;
                break;
            }
            owned.push_back(tb);
            hipLaunchKernelGGL(k_fill_u32, grid_for((n + 3) / 4, kBlock, 8192), kBlock, 0, st, (uint32_t*)tb,
                               (n + 3) / 4, 0u);
            bool exhausted = false;
            Triple Ch[kTMax];   // the rounds pass each round's triple by value
            for (uint32_t t = 0; t < P.T; ++t) Ch[t] = level2_triple(M->seed, r, t);
            rc = rounds_search(o.keys, n, S, A, M->magic_n, a.sizes, Ch, P.T, tb, &exhausted, st);
            if (rc) {
                dev_free(cells, st);
                break;
            }
            // a bucket left after T rounds goes through the per-bucket search, which
            // reports the exhaustion (and any duplicate keys) exactly as it would alone
            if (!exhausted) given_t = tb;
        }
        rc = part_finish(a, o, M->C, P.T, M->header, cells, &ctrl->exhausted, M->ctx_off, M->ctx_bytes, given_t,
                         nullptr, ~0ull, st);
        if (rc == FKS_OK) rc = readback();
        if (rc) {
            dev_free(cells, st);
            break;
        }
        if (host->exhausted) {
            dev_free(cells, st);
            if (host->dup) {
                rc = FKS_EDUPKEY;
                break;
            }
            continue;
        }
        M->slots = cells;
        M->S = S;
        M->r = r;
        M->A = A;
        M->beta = beta;
        M->max_t = host->max_t;
        M->device_bytes += 16 * S;
        release();
        return FKS_OK;
    }
    drop_slots();
    release();
    if (rc) return rc;
    // every attempt was rejected: equal keys, which no attempt can separate, make it a
    // broken precondition rather than bad luck
    bool equal = false;
    if ((rc = has_equal_keys(bytes ? y : d_keys_in, n, bytes ? M->ctx_off : nullptr, bytes ? M->ctx_bytes : nullptr,
                             st, &equal)))
        return rc;
    return equal ? FKS_EDUPKEY : FKS_EBUILD;
}

// keys: device u64 keys (or fingerprints); vals; aux_is_index for string maps
static int build_common(fks_map* M, const uint64_t* d_keys_in, const uint32_t* d_vals, const uint32_t* d_aux_in,
                        const int64_t* d_off, const uint8_t* d_bytes, uint64_t nbytes,
                        const fks_params& P, hipStream_t st) {
    const uint64_t n = M->n;
    const uint64_t G = (n + 7) / 8;
    const bool bytes = M->kind == 1;
    Scratch w;
    int rc = FKS_OK;
    auto fail = [&](int code) {
        free_scratch(w, st);
        return code;
    };
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
        // the offsets are checked by the fingerprint pass, before any byte is read through them
        hipError_t e = hipMemcpyAsync(M->ctx_off, d_off, 8 * (n + 1), hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && nbytes) e = hipMemcpyAsync(M->ctx_bytes, d_bytes, nbytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return fail(hip_fail(e));
    }

    M->magic_n = fastmod_magic((uint32_t)n);
    rc = attempts_partitioned(M, d_keys_in, d_vals, d_aux_in, P, w.ctrl, w.host, w.y, st);
    free_scratch(w, st);
    return rc;
}

static void release_partial(fks_map* M, hipStream_t st) {
    dev_free(M->header, st);
    dev_free(M->slots, st);
    dev_free(M->C, st);
    dev_free(M->ctx_off, st);
    dev_free(M->ctx_bytes, st);
    delete M;
}

static fks_map* new_map(uint32_t kind, uint64_t n, uint64_t seed, const fks_params& P, const fks_allocator* alloc) {
    fks_map* M = new fks_map;
    std::memset(M, 0, sizeof(*M));
    keep_allocator(alloc, M->alloc, M->has_alloc);
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
                             const fks_params* params, const fks_allocator* alloc, void* stream, fks_map** out) {
    using namespace fks;
    if (!out || (n && (!d_keys || !d_vals)) || !allocator_ok(alloc)) return FKS_EINVAL;
    fks_params P;
    int rc = check_params(n, params, P);
    if (rc) return rc;
    AllocScope scope(alloc);
    hipStream_t st = (hipStream_t)stream;
    fks_map* M = new_map(0, n, seed, P, alloc);
    rc = n ? build_common(M, d_keys, d_vals, nullptr, nullptr, nullptr, 0, P, st) : build_empty(M, P, st);
    if (rc) {
        release_partial(M, st);
        return rc;
    }
    *out = M;
    return FKS_OK;
}

extern "C" int fks_build_u64_v64(const uint64_t* d_keys, const uint64_t* d_vals, uint64_t n, uint64_t seed,
                                 const fks_params* params, const fks_allocator* alloc, void* stream,
                                 fks_map** out) {
    using namespace fks;
    if (!out || (n && (!d_keys || !d_vals)) || !allocator_ok(alloc)) return FKS_EINVAL;
    fks_params P;
    int rc = check_params(n, params, P);
    if (rc) return rc;
    AllocScope scope(alloc);
    hipStream_t st = (hipStream_t)stream;
    fks_map* M = new_map(2, n, seed, P, alloc);
    if (n == 0) {
        rc = build_empty(M, P, st);
    } else {
        // the construction carries the low halves as values and the high halves as aux words
        uint32_t* lo = (uint32_t*)dev_alloc(4 * n, st);
        uint32_t* hi = (uint32_t*)dev_alloc(4 * n, st);
        if (!lo || !hi) {
            rc = FKS_ENOMEM;
        } else {
            hipLaunchKernelGGL(k_split_u64, grid_for(n, kBlock, 65536), kBlock, 0, st, d_vals, n, lo, hi);
            rc = build_common(M, d_keys, lo, hi, nullptr, nullptr, 0, P, st);
        }
        dev_free(lo, st);
        dev_free(hi, st);
    }
    if (rc) {
        release_partial(M, st);
        return rc;
    }
    *out = M;
    return FKS_OK;
}

extern "C" int fks_build_bytes(const int64_t* d_offsets, const uint8_t* d_bytes, uint64_t nbytes,
                               const uint32_t* d_vals, uint64_t n, uint64_t seed, const fks_params* params,
                               const fks_allocator* alloc, void* stream, fks_map** out) {
    using namespace fks;
    if (!out || !d_offsets || (n && !d_vals) || (nbytes && !d_bytes) || !allocator_ok(alloc)) return FKS_EINVAL;
    fks_params P;
    int rc = check_params(n, params, P);
    if (rc) return rc;
    AllocScope scope(alloc);
    hipStream_t st = (hipStream_t)stream;
    fks_map* M = new_map(1, n, seed, P, alloc);
    if (n) {
        rc = build_common(M, nullptr, d_vals, nullptr, d_offsets, d_bytes, nbytes, P, st);
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
