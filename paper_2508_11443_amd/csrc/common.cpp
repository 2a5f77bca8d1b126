// Host-side plumbing of the FKS library: error codes, device memory, map
// introspection, export and release.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "fks_internal.hpp"

namespace fks {

static thread_local int g_last_hip_error = 0;

void set_hip_error(hipError_t e) { g_last_hip_error = (int)e; }

int hip_fail(hipError_t e) {
    g_last_hip_error = (int)e;
    if (e == hipErrorOutOfMemory) return FKS_ENOMEM;
    return FKS_EHIP;
}

static std::once_flag g_pool_once[64];

static void configure_pool(int dev) {
    // keep freed stream-ordered blocks cached in the pool instead of returning
    // them to the driver at every synchronisation
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t threshold = ~0ull;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
    }
}

static thread_local const fks_allocator* tl_alloc = nullptr;

AllocScope::AllocScope(const fks_allocator* a) : prev_(tl_alloc) { tl_alloc = a; }
AllocScope::~AllocScope() { tl_alloc = prev_; }

bool dev_pool_default() { return tl_alloc == nullptr; }

void* dev_alloc(size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 16;
    if (tl_alloc) {
        void* p = tl_alloc->alloc((uint64_t)bytes, (void*)s, tl_alloc->user);
        if (!p) set_hip_error(hipErrorOutOfMemory);
        return p;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev >= 0 && dev < 64) std::call_once(g_pool_once[dev], configure_pool, dev);
    void* p = nullptr;
    hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess) {
        set_hip_error(e);
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

// per-workgroup LDS histogram of the 4-bit bucket sizes, folded into 16 global counters
__global__ __launch_bounds__(256) void k_size_hist(const Group* __restrict__ header, uint64_t n,
                                                     unsigned long long* __restrict__ hist) {
    __shared__ uint32_t h[16];
    if (threadIdx.x < 16) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t G = (n + 7) / 8;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t w = header[g].sizes;
        const uint32_t k_end = g + 1 < G || n % 8 == 0 ? 8u : (uint32_t)(n % 8);
        for (uint32_t k = 0; k < k_end; ++k) atomicAdd(&h[nib(w, k)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 16 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

int size_histogram(const Group* header, uint64_t n, uint64_t hist[16]) {
    for (int s = 0; s < 16; ++s) hist[s] = 0;
    if (n == 0) return FKS_OK;
    unsigned long long* d = nullptr;
    hipError_t e = hipMalloc((void**)&d, 16 * sizeof(unsigned long long));
    if (e != hipSuccess) return hip_fail(e);
    uint64_t grid = ((n + 7) / 8 + 255) / 256;
    if (grid > 1024) grid = 1024;
    e = hipMemset(d, 0, 16 * sizeof(unsigned long long));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_size_hist, (unsigned)grid, 256, 0, nullptr, header, n, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(hist, d, 16 * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    return e == hipSuccess ? FKS_OK : hip_fail(e);
}

void dev_free(void* p, hipStream_t s) {
    if (!p) return;
    if (tl_alloc) tl_alloc->free(p, (void*)s, tl_alloc->user);
    else (void)hipFreeAsync(p, s);
}

}  // namespace fks

extern "C" {

void fks_params_default(fks_params* p) {
    if (!p) return;
    p->c = 4;
    p->T = 64;
    p->R = 16;
    p->schedule = 0;
}

const char* fks_strerror(int code) {
    switch (code) {
        case FKS_OK: return "ok";
        case FKS_EINVAL: return "invalid argument";
        case FKS_ENOMEM: return "out of device memory";
        case FKS_EDUPKEY: return "duplicate keys in from_array_nodup input";
        case FKS_EBUILD: return "every level-one attempt was rejected";
        case FKS_EHIP: return "HIP runtime error";
        default: return "unknown error";
    }
}

int fks_last_hip_error(void) { return fks::g_last_hip_error; }

int fks_version(void) { return 10000; }

int fks_info(const fks_map* map, fks_map_info* info) {
    if (!map || !info) return FKS_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->n = map->n;
    info->S = map->S;
    info->header_bytes = 16 * ((map->n + 7) / 8);
    info->slot_bytes = 16 * map->S;
    info->ctx_bytes = map->ctx_nbytes;
    info->seed = map->seed;
    info->r = map->r;
    info->kind = map->kind;
    info->c = map->c;
    info->T = map->T;
    info->R = map->R;
    info->max_t = map->max_t;
    info->device_bytes = map->device_bytes;
    int prev = 0;
    FKS_HIP(hipGetDevice(&prev));
    FKS_HIP(hipSetDevice(map->device));
    const int rc = fks::size_histogram(map->header, map->n, info->size_hist);
    (void)hipSetDevice(prev);
    return rc;
}

int fks_export(const fks_map* map, void* h_header, void* h_slots, uint64_t* h_consts) {
    if (!map) return FKS_EINVAL;
    int prev = 0;
    FKS_HIP(hipGetDevice(&prev));
    FKS_HIP(hipSetDevice(map->device));
    const uint64_t hb = 16 * ((map->n + 7) / 8);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && h_header && hb) e = hipMemcpy(h_header, map->header, hb, hipMemcpyDeviceToHost);
    if (e == hipSuccess && h_slots && map->S) e = hipMemcpy(h_slots, map->slots, 16 * map->S, hipMemcpyDeviceToHost);
    if (e == hipSuccess && h_consts)
        e = hipMemcpy(h_consts, map->C, sizeof(fks::Triple) * map->T, hipMemcpyDeviceToHost);
    (void)hipSetDevice(prev);   // the caller's device, also on failure
    return e == hipSuccess ? FKS_OK : fks::hip_fail(e);
}

void fks_destroy(fks_map* map) {
    if (!map) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(map->device);
    {
        // the memory goes back where the build took it from; frees are ordered on the
        // null stream, after all work already queued on it
        fks::AllocScope scope(map->has_alloc ? &map->alloc : nullptr);
        fks::dev_free(map->header, nullptr);
        fks::dev_free(map->slots, nullptr);
        fks::dev_free(map->C, nullptr);
        fks::dev_free(map->ctx_off, nullptr);
        fks::dev_free(map->ctx_bytes, nullptr);
    }
    (void)hipSetDevice(prev);
    delete map;
}

}  // extern "C"
