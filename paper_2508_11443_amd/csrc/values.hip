// Map and reduce over the values of a built map (Section 1: like an array, a
// hash map lets one map a function over its values or reduce them to a single
// value).
//
// A map's table is fixed by its keys, seed and parameters; the values only ride
// in the cells.  Mapping f over the values keeps the group headers, the
// level-two triples and every key word, and rewrites the value of every cell,
// the copies written by the fill rule of Section 2.2 included, so that the new
// table is byte for byte the one a build over the pairs (k, f(v)) writes.
// A reduction visits every key once: a cell holds its own key when the key's
// level-two hash lands on it, while a fill copy of a bucket's lowest key sits
// in a cell that key does not hash to and is skipped.  Both passes stream the
// table in address order.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fks_internal.hpp"
#include "prof.hpp"

namespace fks {

constexpr int kVBlock = 256;
constexpr uint32_t kVGrid = 4096;   // most workgroups of the reduction's first pass (16 per CU; they stride beyond)


__device__ __forceinline__ uint64_t cell_value(const Cell& c, bool v64) {
    return v64 ? ((uint64_t)c.aux << 32) | c.val : (uint64_t)c.val;
}

// v -> f(v) for one of the FKS_VOP_* operations, in the map's value width;
// a gather index outside the table sets `bad` and yields 0
template <bool V64>
__device__ __forceinline__ uint64_t apply_vop(uint32_t op, uint64_t v, uint64_t a, uint64_t b, const void* table,
                                              uint64_t len, bool& bad) {
    uint64_t r;
    switch (op) {
        case FKS_VOP_ADD: r = v + a; break;
        case FKS_VOP_MUL: r = v * a; break;
        case FKS_VOP_XOR: r = v ^ a; break;
        case FKS_VOP_AFFINE: r = v * a + b; break;
        default:
            if (v < len) {
                r = V64 ? ((const uint64_t*)table)[v] : (uint64_t)((const uint32_t*)table)[v];
            } else {
                bad = true;
                r = 0;
            }
    }
    return V64 ? r : (uint64_t)(uint32_t)r;
}

__device__ __forceinline__ uint64_t combine(uint32_t op, uint64_t x, uint64_t y) {
    switch (op) {
        case FKS_VRED_SUM: return x + y;
        case FKS_VRED_MIN: return x < y ? x : y;
        case FKS_VRED_MAX: return x > y ? x : y;
        default: return x ^ y;
    }
}

// one cell per lane; every cell's value word(s) rewritten, key and aux kept
template <bool V64>
__global__ __launch_bounds__(kVBlock) void k_map_values(const Cell* __restrict__ in, Cell* __restrict__ out,
                                                          uint64_t S, uint32_t op, uint64_t a, uint64_t b,
                                                          const void* __restrict__ table, uint64_t len,
                                                          uint32_t* __restrict__ bad_flag) {
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S;
         i += (uint64_t)gridDim.x * blockDim.x) {
        Cell c = load_cell_once(in + i);   // each cell is read once and written once
        const uint64_t v = apply_vop<V64>(op, cell_value(c, V64), a, b, table, len, bad);
        c.val = (uint32_t)v;
        if (V64) c.aux = (uint32_t)(v >> 32);
        store_cell_once(out + i, c);
    }
    if (bad) atomicOr(bad_flag, 1u);
}

// block-wide fold of one value per thread (LDS tree); the result in thread 0
__device__ __forceinline__ uint64_t block_fold(uint64_t v, uint32_t op, uint64_t* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t w = kVBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = combine(op, red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    return red[0];
}

// first pass: each workgroup takes ranges of kVBlock consecutive groups (one group record
// per lane, staged in LDS with an LDS map from each of the range's cells to its bucket),
// then streams the range's cells, consecutive cells on consecutive lanes.  A cell holds its
// own key exactly when the key's level-two hash in the cell's bucket lands on the cell; a
// fill copy of a bucket's lowest key sits elsewhere and is skipped, so each key is folded
// once.  A range with more cells than the LDS map holds (far beyond the ~15 cells of eight
// buckets of random keys) is walked bucket by bucket instead.
constexpr uint32_t kRMapCells = 8192;   // cells of one range mapped in LDS
constexpr uint32_t kRUnroll = 4;        // cells per lane in flight

template <bool V64>
__global__ __launch_bounds__(kVBlock) void k_reduce_ranges(const Group* __restrict__ header,
                                                             const Cell* __restrict__ slots, uint64_t G, uint64_t S,
                                                             const Triple* __restrict__ Cg, uint32_t T, uint32_t op,
                                                             uint64_t ident, uint64_t* __restrict__ partial) {
    extern __shared__ Triple C[];            // the map's T level-two triples
    __shared__ Group rec[kVBlock];
    // (group in the range << 3) | bucket of each of the range's cells; at the end, the
    // workgroup's fold (the map is no longer read then)
    __shared__ __align__(16) uint16_t owner[kRMapCells];
    __shared__ uint64_t mag[16];
    __shared__ uint32_t span[2];
    static_assert(sizeof(owner) >= kVBlock * sizeof(uint64_t), "the fold fits the map");
    const uint32_t tid = threadIdx.x;
    for (uint32_t k = tid; k < T; k += kVBlock) C[k] = Cg[k];
    if (tid < 16) mag[tid] = tid ? fastmod_magic(tid * tid) : 0;
    uint64_t acc = ident;
    for (uint64_t g0 = (uint64_t)blockIdx.x * kVBlock; g0 < G; g0 += (uint64_t)gridDim.x * kVBlock) {
        const uint32_t ng = (uint32_t)min((uint64_t)kVBlock, G - g0);
        __syncthreads();   // the previous range's LDS is no longer read
        Group h{0, 0, 0, 0};
        if (tid < ng) h = header[g0 + tid];
        rec[tid] = h;
        if (tid == 0) span[0] = h.base;
        if (tid == ng - 1) span[1] = h.base + prefix_sq(h.sizes, 8);   // end of the range's cells
        __syncthreads();
        const uint32_t c0 = span[0], nc = span[1] - span[0];
        if (nc <= kRMapCells) {
            // every cell of the lane's group gets its bucket
            if (tid < ng) {
                for (uint32_t k = 0; k < 8; ++k) {
                    const uint32_t sb = nib(h.sizes, k);
                    const uint32_t at = h.base - c0 + prefix_sq(h.sizes, k);
                    for (uint32_t p = 0; p < sb * sb; ++p) owner[at + p] = (uint16_t)((tid << 3) | k);
                }
            }
            __syncthreads();
            for (uint32_t e0 = 0; e0 < nc; e0 += kVBlock * kRUnroll) {
                Cell x[kRUnroll];
#pragma unroll
                for (uint32_t u = 0; u < kRUnroll; ++u) {
                    const uint32_t e = e0 + u * kVBlock + tid;
                    x[u] = e < nc && (uint64_t)c0 + e < S ? load_cell_once(slots + c0 + e) : Cell{0, 0, 0};
                }
#pragma unroll
                for (uint32_t u = 0; u < kRUnroll; ++u) {
                    const uint32_t e = e0 + u * kVBlock + tid;
                    if (e >= nc || (uint64_t)c0 + e >= S) continue;
                    const uint32_t o = owner[e];
                    const Group& r = rec[o >> 3];
                    const uint32_t k = o & 7u, sb = nib(r.sizes, k);
                    const uint32_t t = sb == 1 ? 0u : group_t(r, k);   // a one-key bucket's byte is a tag
                    if (t >= T) continue;
                    const uint32_t local = c0 + e - (r.base + prefix_sq(r.sizes, k));
                    if (fastmod(mshash(C[t], x[u].key), mag[sb], sb * sb) == local)
                        acc = combine(op, acc, cell_value(x[u], V64));
                }
            }
        } else if (tid < ng) {
            // a range too large for the map: the lane walks its own group's buckets
            for (uint32_t k = 0; k < 8; ++k) {
                const uint32_t sb = nib(h.sizes, k);
                const uint32_t t = sb == 1 ? 0u : group_t(h, k);
                if (sb == 0 || t >= T) continue;
                const uint32_t s2 = sb * sb;
                const uint64_t start = (uint64_t)h.base + prefix_sq(h.sizes, k);
                if (start + s2 > S) continue;
                for (uint32_t l = 0; l < s2; ++l) {
                    const Cell x = slots[start + l];
                    if (mshash(C[t], x.key) % s2 == l) acc = combine(op, acc, cell_value(x, V64));
                }
            }
        }
    }
    __syncthreads();   // the last range's map is no longer read
    const uint64_t r = block_fold(acc, op, reinterpret_cast<uint64_t*>(owner));
    if (tid == 0) partial[blockIdx.x] = r;
}

// second pass: one workgroup folds the partials (none for an empty map)
__global__ __launch_bounds__(kVBlock) void k_reduce_final(const uint64_t* __restrict__ partial, uint32_t np,
                                                            uint32_t op, uint64_t ident, uint64_t* __restrict__ out) {
    __shared__ uint64_t red[kVBlock];
    uint64_t acc = ident;
    for (uint32_t i = threadIdx.x; i < np; i += kVBlock) acc = combine(op, acc, partial[i]);
    const uint64_t r = block_fold(acc, op, red);
    if (threadIdx.x == 0) out[0] = r;
}

static void free_map(fks_map* M, hipStream_t st) {
    dev_free(M->header, st);
    dev_free(M->slots, st);
    dev_free(M->C, st);
    dev_free(M->ctx_off, st);
    dev_free(M->ctx_bytes, st);
    delete M;
}

}  // namespace fks

using namespace fks;

extern "C" int fks_map_values(const fks_map* map, uint32_t op, uint64_t a, uint64_t b, const void* d_table,
                              uint64_t table_len, const fks_allocator* alloc, void* stream, fks_map** out) {
    if (!map || !out || op > FKS_VOP_GATHER || !allocator_ok(alloc)) return FKS_EINVAL;
    if (op == FKS_VOP_GATHER && table_len && !d_table) return FKS_EINVAL;
    AllocScope scope(alloc);
    hipStream_t st = (hipStream_t)stream;
    const bool v64 = map->kind == 2;
    const uint64_t G = (map->n + 7) / 8;
    const bool ctx = map->kind == 1 && map->ctx_off && map->ctx_bytes;
    // the new map: the same keys, attempt and parameters; its own copies of the header, the
    // triples and a string map's context, and cells with the mapped values
    fks_map* M = new fks_map(*map);
    keep_allocator(alloc, M->alloc, M->has_alloc);   // the new map's memory comes from this call's allocator
    M->header = nullptr;
    M->slots = nullptr;
    M->C = nullptr;
    M->ctx_off = nullptr;
    M->ctx_bytes = nullptr;
    bool ok = true;
    if (G) ok = ok && (M->header = (Group*)dev_alloc(16 * G, st));
    if (map->S) ok = ok && (M->slots = (Cell*)dev_alloc(16 * map->S, st));
    ok = ok && (M->C = (Triple*)dev_alloc(sizeof(Triple) * map->T, st));
    if (ctx) {
        ok = ok && (M->ctx_off = (int64_t*)dev_alloc(8 * (map->n + 1), st));
        ok = ok && (M->ctx_bytes = (uint8_t*)dev_alloc(map->ctx_nbytes ? map->ctx_nbytes : 1, st));
    }
    uint32_t* flag = ok ? (uint32_t*)dev_alloc(64, st) : nullptr;
    if (!ok || !flag) {
        dev_free(flag, st);
        free_map(M, st);
        return FKS_ENOMEM;
    }
    hipError_t e = hipMemsetAsync(flag, 0, 4, st);
    if (e == hipSuccess && G) e = hipMemcpyAsync(M->header, map->header, 16 * G, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(M->C, map->C, sizeof(Triple) * map->T, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && ctx)
        e = hipMemcpyAsync(M->ctx_off, map->ctx_off, 8 * (map->n + 1), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && ctx && map->ctx_nbytes)
        e = hipMemcpyAsync(M->ctx_bytes, map->ctx_bytes, map->ctx_nbytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && map->S) {
        uint64_t grid = (map->S + kVBlock - 1) / kVBlock;
        if (grid > 65536) grid = 65536;
        if (v64)
            FKS_TIMED("fks_map_values", st,
                      hipLaunchKernelGGL(k_map_values<true>, (unsigned)grid, kVBlock, 0, st, map->slots, M->slots,
                                         map->S, op, a, b, d_table, table_len, flag));
        else
            FKS_TIMED("fks_map_values", st,
                      hipLaunchKernelGGL(k_map_values<false>, (unsigned)grid, kVBlock, 0, st, map->slots, M->slots,
                                         map->S, op, a, b, d_table, table_len, flag));
        e = hipGetLastError();
    }
    uint32_t bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dev_free(flag, st);
    if (e != hipSuccess || bad) {
        free_map(M, st);
        return e != hipSuccess ? hip_fail(e) : FKS_EINVAL;
    }
    *out = M;
    return FKS_OK;
}

namespace fks {

// workgroups of the reduction's first pass (each strides over the table beyond that)
static uint32_t reduce_partials(const fks_map* map) {
    const uint64_t G = (map->n + 7) / 8;
    uint64_t np = (G + kVBlock - 1) / kVBlock;
    return (uint32_t)(np > kVGrid ? kVGrid : np);
}

// the two passes of the reduction into `partial` (room for reduce_partials(map) entries)
static int reduce_launch(const fks_map* map, uint32_t op, uint64_t* d_out, uint64_t* partial, hipStream_t st) {
    const bool v64 = map->kind == 2;
    // the identity of the operation in the map's value width
    const uint64_t ident = op == FKS_VRED_MIN ? (v64 ? ~0ull : 0xFFFFFFFFull) : 0ull;
    const uint64_t G = (map->n + 7) / 8;
    const uint32_t np = reduce_partials(map);
    if (G == 0) {
        hipLaunchKernelGGL(k_reduce_final, 1, kVBlock, 0, st, nullptr, 0u, op, ident, d_out);
    } else {
        const size_t dyn = sizeof(Triple) * map->T;
        if (v64)
            FKS_TIMED("fks_reduce_values", st,
                      hipLaunchKernelGGL(k_reduce_ranges<true>, np, kVBlock, dyn, st, map->header, map->slots, G,
                                         map->S, map->C, map->T, op, ident, partial));
        else
            FKS_TIMED("fks_reduce_values", st,
                      hipLaunchKernelGGL(k_reduce_ranges<false>, np, kVBlock, dyn, st, map->header, map->slots, G,
                                         map->S, map->C, map->T, op, ident, partial));
        hipLaunchKernelGGL(k_reduce_final, 1, kVBlock, 0, st, partial, np, op, ident, d_out);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

}  // namespace fks

extern "C" int fks_reduce_values(const fks_map* map, uint32_t op, uint64_t* d_out, void* stream) {
    if (!map || !d_out || op > FKS_VRED_XOR) return FKS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    uint64_t* partial = nullptr;
    if (map->n) {
        partial = (uint64_t*)dev_alloc(8ull * reduce_partials(map), st);
        if (!partial) return FKS_ENOMEM;
    }
    const int rc = reduce_launch(map, op, d_out, partial, st);
    dev_free(partial, st);
    return rc;
}

// ---- reduction without allocation --------------------------------------------
namespace fks {

// The first pass's partial folds for fks_reduce_values_noalloc: at most kVGrid of them,
// whatever the map's size.  Every device the library runs on holds its own copy for the
// life of the process; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device.
static __device__ __align__(256) uint64_t scratch[kVGrid];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint64_t* g_scratch[kMaxDevices];

// device address of `scratch` on the current device, looked up once per device
static int scratch_on_current_device(uint64_t** out) {
    int dev = 0;
    FKS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return FKS_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        FKS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch[dev] = (uint64_t*)p;
    }
    *out = g_scratch[dev];
    return FKS_OK;
}

}  // namespace fks

extern "C" int fks_reduce_values_noalloc(const fks_map* map, uint32_t op, uint64_t* d_out, void* stream) {
    if (!map || !d_out || op > FKS_VRED_XOR) return FKS_EINVAL;
    // the first pass never has more than kVGrid workgroups; a larger need would be a bug
    if (reduce_partials(map) > kVGrid) return FKS_EINVAL;
    uint64_t* partial = nullptr;
    const int rc = scratch_on_current_device(&partial);
    if (rc != FKS_OK) return rc;
    return reduce_launch(map, op, d_out, partial, (hipStream_t)stream);
}
