// A serving loop over resident maps: builds are admitted against a device
// memory budget and run on their own stream; lookup requests of any size that
// arrive while other work is on the GPU are coalesced into one launch of a
// multi-request lookup kernel, replayed from a captured HIP graph per size
// class, on a second stream, so lookups overlap the builds.  Every request
// gets a completion time; latency percentiles come from those.
//
// Threads: the caller submits; one host thread runs builds (a build waits for
// its own small readbacks), one host thread forms and launches lookup batches
// and retires them through events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "fks_internal.hpp"
#include "prof.hpp"

namespace fks {

constexpr uint32_t kTile = 1024;          // needles per tile: 256 threads x 4
constexpr uint32_t kMaxReqPerLaunch = 256;
constexpr int kRing = 4;                  // lookup launches in flight
constexpr int kBuildWorkers = 3;          // builds in flight (each worker thread has its own stream)

struct alignas(16) LReq {
    const Group* header;
    const Cell* slots;
    const Triple* C;
    const uint64_t* q;
    uint32_t* vals;
    uint8_t* found;
    Triple A;
    uint64_t magic;
    uint64_t m;
    uint32_t n, T;
    uint32_t missing;
    uint32_t tile0;     // first tile of this request in the launch
};

// one launch's request table; the kernel reads the counts from it so that a
// captured graph needs no argument other than the table's address
struct alignas(16) LTab {
    uint32_t nreq, total_tiles, pad0, pad1;
    LReq reqs[kMaxReqPerLaunch];
};

__global__ __launch_bounds__(256) void k_lookup_multi(const LTab* __restrict__ tab) {
    const uint32_t nreq = tab->nreq, total_tiles = tab->total_tiles;
    const LReq* __restrict__ reqs = tab->reqs;
    __shared__ LReq R;
    __shared__ Triple C[kTMax];
    for (uint32_t tile = blockIdx.x; tile < total_tiles; tile += gridDim.x) {
        __syncthreads();
        if (threadIdx.x == 0) {
            // the request owning this tile: last one with tile0 <= tile
            uint32_t lo = 0, hi = nreq;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) / 2;
                if (reqs[mid].tile0 <= tile) lo = mid;
                else hi = mid;
            }
            R = reqs[lo];
        }
        __syncthreads();
        const uint32_t T = R.n ? R.T : 0;
        for (uint32_t t = threadIdx.x; t < T; t += 256) C[t] = R.C[t];
        __syncthreads();
        const uint64_t base = (uint64_t)(tile - R.tile0) * kTile;
        uint64_t x[4];
        Group h[4];
        uint32_t kk[4], s[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t i = base + threadIdx.x + (uint64_t)k * 256;
            x[k] = i < R.m ? R.q[i] : 0;
            s[k] = 0;
            kk[k] = 0;
            if (i < R.m && R.n) {
                const uint32_t j = fastmod(mshash(R.A, x[k]), R.magic, R.n);
                kk[k] = j & 7u;
                h[k] = R.header[j >> 3];
                s[k] = nib(h[k].sizes, kk[k]);
            }
        }
        Cell c[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint32_t p;
            if (s[k]) s[k] = cell_of(h[k], kk[k], C, x[k], p) ? 1u : 0u;
            if (s[k]) c[k] = load_cell_once(R.slots + p);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t i = base + threadIdx.x + (uint64_t)k * 256;
            if (i < R.m) {
                const bool hit = s[k] && c[k].key == x[k];
                if (R.vals) R.vals[i] = hit ? c[k].val : R.missing;
                if (R.found) R.found[i] = hit ? 1 : 0;
            }
        }
    }
}

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// The server's device memory: one slab reserved when the server is created, handed out
// first fit (256-byte aligned) and coalesced on release, so that no build and no eviction
// calls the driver's allocator while requests are served (a stream-ordered allocation
// that has to grow its pool can hold the runtime for a long time).  A block is released
// only after its last use on the device is complete: a build's scratch after the build's
// final wait, a map's memory when the map is evicted idle or the server is destroyed;
// every build runs on the one build stream.  So a block can be handed out again at once.
struct Arena {
    std::mutex mu;
    char* base = nullptr;
    uint64_t size = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> length of every free range
    std::map<uint64_t, uint64_t> used_;   // offset -> length of every block handed out

    void* take(uint64_t bytes) {
        bytes = (bytes + 255) & ~255ull;
        std::lock_guard<std::mutex> lk(mu);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const uint64_t at = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[at + bytes] = len - bytes;
            used_[at] = bytes;
            return base + at;
        }
        return nullptr;
    }
    void give_back(void* p) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu);
        auto u = used_.find((uint64_t)((char*)p - base));
        if (u == used_.end()) return;
        uint64_t at = u->first, len = u->second;
        used_.erase(u);
        auto next = free_.lower_bound(at);
        if (next != free_.end() && next->first == at + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == at) {
                prev->second += len;
                return;
            }
        }
        free_[at] = len;
    }
};

static void* arena_alloc(uint64_t bytes, void*, void* user) { return static_cast<Arena*>(user)->take(bytes); }
static void arena_free(void* p, void*, void* user) { static_cast<Arena*>(user)->give_back(p); }

}  // namespace fks

using namespace fks;

struct fks_server {
    // configuration
    uint64_t budget;
    fks_params params;
    int device;
    hipStream_t build_st[kBuildWorkers] = {}, lookup_st = nullptr;
    // state guarded by mu
    std::mutex mu;
    std::condition_variable cv_build, cv_lookup, cv_done;
    bool stop = false;
    uint64_t used = 0;        // bytes of resident maps plus the reservation of the running build
    uint64_t clock = 0;       // LRU clock
    struct MapSlot {
        fks_map* map = nullptr;
        uint64_t bytes = 0;
        uint64_t last_use = 0;
        int pins = 0;          // queued or running lookups
        int state = 0;         // 0 queued, 1 building, 2 ready, 3 failed, 4 evicted
        int status = 0;
    };
    std::deque<MapSlot> maps;      // deque: references stay valid as it grows
    struct Req {
        int kind;              // 0 build, 1 lookup
        uint32_t map_id;
        const uint64_t* keys;
        const uint32_t* vals;
        uint64_t n;
        uint64_t seed;
        uint64_t m;
        uint32_t* out_vals;
        uint8_t* out_found;
        uint32_t missing;
        hipEvent_t ready = nullptr;   // recorded on the submitter's stream: the inputs are written
        double t_submit = 0, t_start = 0, t_done = 0;
        int status = 0;
        bool done = false;
    };
    std::deque<Req> reqs;
    std::deque<uint64_t> build_q, lookup_q;
    uint64_t n_done = 0;
    // statistics
    uint64_t launches = 0, graph_replays = 0, graph_captures = 0, evictions = 0, coalesced = 0;
    uint64_t queries_done = 0, keys_built = 0;
    double first_submit = -1, last_done = 0;
    // lookup launch resources
    fks::LTab* h_tab[kRing] = {};
    fks::LTab* d_tab[kRing] = {};
    hipStream_t capture_st = nullptr;
    bool use_graphs = true;
    hipEvent_t ev[kRing] = {};
    std::map<std::pair<int, uint32_t>, hipGraphExec_t> graphs;   // (ring slot, grid class)
    std::thread build_thr[kBuildWorkers], lookup_thr;
    // device memory of the maps and of the builds' scratch
    fks::Arena arena;
    fks_allocator alloc{};
};

namespace fks {

static uint64_t estimate_bytes(uint64_t n, const fks_params& p) {
    // header + the largest table an accepted attempt may have + level-two triples
    return 16 * ((n + 7) / 8) + 16 * (uint64_t)p.c * n + sizeof(Triple) * p.T + 4096;
}

// Evict least recently used idle maps until `need` more bytes fit; mu held.  Nothing is
// evicted unless the idle maps free enough: false then, and the caller waits for pinned
// maps to drain (or gives up when even that cannot make room).
static bool make_room(fks_server* S, uint64_t need) {
    if (S->used + need <= S->budget) return true;
    if (need > S->budget) return false;
    uint64_t idle = 0;
    for (const auto& ms : S->maps)
        if (ms.state == 2 && ms.pins == 0) idle += ms.bytes;
    if (S->used - idle + need > S->budget) return false;
    while (S->used + need > S->budget) {
        int best = -1;
        for (size_t i = 0; i < S->maps.size(); ++i) {
            auto& ms = S->maps[i];
            if (ms.state == 2 && ms.pins == 0 && (best < 0 || ms.last_use < S->maps[best].last_use)) best = (int)i;
        }
        if (best < 0) return false;
        auto& ms = S->maps[best];
        fks_destroy(ms.map);
        ms.map = nullptr;
        S->used -= ms.bytes;
        ms.bytes = 0;
        ms.state = 4;
        S->evictions++;
    }
    return true;
}

static void finish_req(fks_server* S, uint64_t id, int status, double t) {
    auto& r = S->reqs[id];
    if (r.ready) {
        // every wait on it has been satisfied: the request's work is finished or never ran
        (void)hipEventDestroy(r.ready);
        r.ready = nullptr;
    }
    r.status = status;
    r.t_done = t;
    r.done = true;
    S->n_done++;
    if (t > S->last_done) S->last_done = t;
}

// build worker w (of kBuildWorkers, each on its own stream): takes the oldest queued build,
// waits until its reservation is admitted, builds it
static void build_loop(fks_server* S, int w) {
    (void)hipSetDevice(S->device);
    const hipStream_t st = S->build_st[w];
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_build.wait(lk, [&] { return S->stop || !S->build_q.empty(); });
        if (S->stop) return;
        const uint64_t id = S->build_q.front();
        S->build_q.pop_front();
        auto& rq = S->reqs[id];
        const uint64_t est = estimate_bytes(rq.n, S->params);
        // admission: wait until the reservation fits, evicting idle maps; a build larger
        // than the whole budget fails at once and leaves the resident maps alone
        while (est <= S->budget && !make_room(S, est)) {
            // room can still appear once the lookups pinning resident maps drain, or once the
            // other worker's build ends (its reservation becomes a map that can be evicted)
            uint64_t ready_bytes = 0;
            bool building = false;
            for (auto& ms : S->maps) {
                if (ms.state == 2) ready_bytes += ms.bytes;
                building = building || ms.state == 1;
            }
            if ((!building && S->used - ready_bytes + est > S->budget) || S->stop) break;
            S->cv_build.wait_for(lk, std::chrono::milliseconds(1));
        }
        if (S->stop) return;
        auto& slot = S->maps[rq.map_id];
        if (S->used + est > S->budget) {
            slot.state = 3;
            slot.status = FKS_ENOMEM;
            finish_req(S, id, FKS_ENOMEM, now_ms());
            S->cv_lookup.notify_all();
            S->cv_done.notify_all();
            continue;
        }
        S->used += est;
        slot.state = 1;
        rq.t_start = now_ms();
        const uint64_t* keys = rq.keys;
        const uint32_t* vals = rq.vals;
        const uint64_t n = rq.n, seed = rq.seed;
        const hipEvent_t ready = rq.ready;
        fks_params p = S->params;
        lk.unlock();
        fks_map* m = nullptr;
        // the build reads the keys only after the submitter's stream has written them
        int rc = ready ? (hipStreamWaitEvent(st, ready, 0) == hipSuccess ? FKS_OK : FKS_EHIP) : FKS_OK;
        if (rc == FKS_OK) rc = fks_build_u64(keys, vals, n, seed, &p, &S->alloc, st, &m);
        const double t = now_ms();
        lk.lock();
        S->used -= est;
        if (rc == FKS_OK) {
            slot.map = m;
            slot.bytes = m->device_bytes;
            slot.state = 2;
            slot.last_use = ++S->clock;
            S->used += slot.bytes;
            S->keys_built += n;
        } else {
            slot.state = 3;
            slot.status = rc;
        }
        finish_req(S, id, rc, t);
        S->cv_lookup.notify_all();
        S->cv_done.notify_all();
    }
}

// graph per (ring slot, grid size): one kernel node reading the slot's table
static hipGraphExec_t graph_for(fks_server* S, int slot, uint32_t grid) {
    auto key = std::make_pair(slot, grid);
    auto it = S->graphs.find(key);
    if (it != S->graphs.end()) return it->second;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(S->capture_st, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    hipLaunchKernelGGL(k_lookup_multi, grid, 256, 0, S->capture_st, S->d_tab[slot]);
    if (hipStreamEndCapture(S->capture_st, &g) != hipSuccess || !g) return nullptr;
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) ex = nullptr;
    (void)hipGraphDestroy(g);
    if (ex) {
        S->graphs[key] = ex;
        S->graph_captures++;
    }
    return ex;
}

static void lookup_loop(fks_server* S) {
    (void)hipSetDevice(S->device);
    struct Flight {
        bool busy = false;
        int status = FKS_OK;   // FKS_EHIP when the launch could not be queued
        std::vector<uint64_t> ids;
    } flight[kRing];
    int next = 0;
    std::unique_lock<std::mutex> lk(S->mu);
    // a launch whose event has completed: its requests are done; mu held
    auto retire = [&](Flight& f) {
        const double t = now_ms();
        for (uint64_t id : f.ids) {
            auto& r = S->reqs[id];
            S->maps[r.map_id].pins--;
            if (f.status == FKS_OK) S->queries_done += r.m;
            finish_req(S, id, f.status, t);
        }
        f.busy = false;
        f.status = FKS_OK;
        f.ids.clear();
        S->cv_done.notify_all();
        S->cv_build.notify_all();
    };
    for (;;) {
        // retire finished launches
        bool any_busy = false;
        for (int k = 0; k < kRing; ++k) {
            if (!flight[k].busy) continue;
            if (hipEventQuery(S->ev[k]) == hipSuccess) retire(flight[k]);
            else any_busy = true;
        }
        // requests whose map is ready (or can never be)
        std::vector<uint64_t> ready;
        uint64_t tiles = 0;
        for (auto it = S->lookup_q.begin(); it != S->lookup_q.end();) {
            auto& r = S->reqs[*it];
            auto& ms = S->maps[r.map_id];
            if (ms.state == 3 || ms.state == 4) {
                ms.pins--;
                finish_req(S, *it, ms.state == 3 ? ms.status : FKS_EINVAL, now_ms());
                it = S->lookup_q.erase(it);
                S->cv_done.notify_all();
                continue;
            }
            if (ms.state == 2 && ready.size() < kMaxReqPerLaunch && tiles < (1u << 30)) {
                ready.push_back(*it);
                tiles += (r.m + kTile - 1) / kTile;
                it = S->lookup_q.erase(it);
                continue;
            }
            ++it;
        }
        if (S->stop && S->lookup_q.empty() && !any_busy) return;
        if (ready.empty()) {
            if (any_busy) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                S->cv_lookup.wait_for(lk, std::chrono::milliseconds(2));
            }
            continue;
        }
        // wait for a free ring slot
        while (flight[next].busy) {
            lk.unlock();
            (void)hipEventSynchronize(S->ev[next]);
            lk.lock();
            retire(flight[next]);
        }
        LTab* tab = S->h_tab[next];
        uint32_t tile0 = 0;
        uint32_t nr = 0;
        std::vector<hipEvent_t> waits;
        for (uint64_t id : ready) {
            auto& r = S->reqs[id];
            if (r.ready) waits.push_back(r.ready);
            auto& ms = S->maps[r.map_id];
            ms.last_use = ++S->clock;
            const fks_map* mp = ms.map;
            LReq& e = tab->reqs[nr++];
            e.header = mp->header;
            e.slots = mp->slots;
            e.C = mp->C;
            e.q = r.keys;
            e.vals = r.out_vals;
            e.found = r.out_found;
            e.A = mp->A;
            e.magic = mp->magic_n;
            e.m = r.m;
            e.n = (uint32_t)mp->n;
            e.T = mp->T;
            e.missing = r.missing;
            e.tile0 = tile0;
            tile0 += (uint32_t)((r.m + kTile - 1) / kTile);
            r.t_start = now_ms();
        }
        tab->nreq = nr;
        tab->total_tiles = tile0;
        // grid class: the next power of two of the tile count, at most 8192 workgroups
        uint32_t grid = 1;
        while (grid < tile0 && grid < 8192) grid <<= 1;
        const int slot = next;
        next = (next + 1) % kRing;
        flight[slot].busy = true;
        flight[slot].ids = ready;
        S->launches++;
        S->coalesced += nr;
        const size_t bytes = offsetof(LTab, reqs) + sizeof(LReq) * nr;
        lk.unlock();
        // the launch reads each request's needles only after its submitter's stream wrote them
        hipError_t e = hipSuccess;
        for (hipEvent_t w : waits)
            if (e == hipSuccess) e = hipStreamWaitEvent(S->lookup_st, w, 0);
        if (e == hipSuccess) e = hipMemcpyAsync(S->d_tab[slot], tab, bytes, hipMemcpyHostToDevice, S->lookup_st);
        bool replayed = false;
        if (e == hipSuccess) {
            hipGraphExec_t ex = S->use_graphs ? graph_for(S, slot, grid) : nullptr;
            if (ex) replayed = hipGraphLaunch(ex, S->lookup_st) == hipSuccess;
            if (!replayed) {
                FKS_TIMED("fks_lookup_multi", S->lookup_st,
                          hipLaunchKernelGGL(k_lookup_multi, grid, 256, 0, S->lookup_st, S->d_tab[slot]));
                e = hipGetLastError();
            }
        }
        // the slot retires when this event completes (at once when nothing was queued)
        (void)hipEventRecord(S->ev[slot], S->lookup_st);
        lk.lock();
        if (e != hipSuccess) {
            set_hip_error(e);
            flight[slot].status = FKS_EHIP;
        }
        if (replayed) S->graph_replays++;
    }
}

}  // namespace fks

// ---- C ABI ---------------------------------------------------------------------------

extern "C" int fks_server_create(uint64_t budget_bytes, const fks_params* params, uint32_t flags,
                                 fks_server** out) {
    if (!out || budget_bytes == 0) return FKS_EINVAL;
    fks_server* S = new fks_server;
    fks_params_default(&S->params);
    if (params) S->params = *params;
    S->budget = budget_bytes;
    S->use_graphs = (flags & 1u) == 0;
    int rc = FKS_OK;
    hipError_t e = hipGetDevice(&S->device);
    for (int w = 0; w < kBuildWorkers && e == hipSuccess; ++w)
        e = hipStreamCreateWithFlags(&S->build_st[w], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->lookup_st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->capture_st, hipStreamNonBlocking);
    // the arena: the budget for resident maps, plus room for the running build's scratch
    // (under 32 bytes per key; a build admitted under the budget has fewer than
    // budget / (16 c + 2) keys) and for rounding
    if (e == hipSuccess) {
        const uint64_t max_keys = budget_bytes / (16ull * S->params.c + 2);
        S->arena.size = budget_bytes + 32 * max_keys + (256ull << 20);
        e = hipMalloc((void**)&S->arena.base, S->arena.size);
        if (e == hipSuccess) S->arena.free_[0] = S->arena.size;
        else S->arena.base = nullptr;
        S->alloc = fks_allocator{arena_alloc, arena_free, &S->arena};
    }
    for (int k = 0; k < kRing && e == hipSuccess; ++k) {
        e = hipHostMalloc((void**)&S->h_tab[k], sizeof(LTab), hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void**)&S->d_tab[k], sizeof(LTab));
        if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) rc = hip_fail(e);
    if (rc) {
        for (int k = 0; k < kRing; ++k) {
            if (S->h_tab[k]) (void)hipHostFree(S->h_tab[k]);
            if (S->d_tab[k]) (void)hipFree(S->d_tab[k]);
            if (S->ev[k]) (void)hipEventDestroy(S->ev[k]);
        }
        for (int w = 0; w < kBuildWorkers; ++w)
            if (S->build_st[w]) (void)hipStreamDestroy(S->build_st[w]);
        if (S->lookup_st) (void)hipStreamDestroy(S->lookup_st);
        if (S->capture_st) (void)hipStreamDestroy(S->capture_st);
        if (S->arena.base) (void)hipFree(S->arena.base);
        delete S;
        return rc;
    }
    for (int w = 0; w < kBuildWorkers; ++w) S->build_thr[w] = std::thread(build_loop, S, w);
    S->lookup_thr = std::thread(lookup_loop, S);
    *out = S;
    return FKS_OK;
}

// an event recorded on the submitter's stream now: the server's work on the request waits for it
static int mark_ready(void* stream, hipEvent_t* ev) {
    hipError_t e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    if (e == hipSuccess) {
        e = hipEventRecord(*ev, (hipStream_t)stream);
        if (e != hipSuccess) (void)hipEventDestroy(*ev);
    }
    if (e != hipSuccess) {
        *ev = nullptr;
        return hip_fail(e);
    }
    return FKS_OK;
}

extern "C" int fks_server_submit_build(fks_server* S, const uint64_t* d_keys, const uint32_t* d_vals, uint64_t n,
                                       uint64_t seed, void* stream, uint64_t* req_id, uint32_t* map_id) {
    if (!S || (n && (!d_keys || !d_vals)) || n >= (1ull << 30)) return FKS_EINVAL;
    hipEvent_t ready = nullptr;
    if (int rc = mark_ready(stream, &ready)) return rc;
    std::lock_guard<std::mutex> lk(S->mu);
    const uint64_t id = S->reqs.size();
    fks_server::Req r;
    r.kind = 0;
    r.map_id = (uint32_t)S->maps.size();
    r.keys = d_keys;
    r.vals = d_vals;
    r.n = n;
    r.seed = seed;
    r.m = 0;
    r.out_vals = nullptr;
    r.out_found = nullptr;
    r.missing = 0;
    r.ready = ready;
    r.t_submit = now_ms();
    if (S->first_submit < 0) S->first_submit = r.t_submit;
    S->reqs.push_back(r);
    S->maps.emplace_back();
    S->build_q.push_back(id);
    if (req_id) *req_id = id;
    if (map_id) *map_id = r.map_id;
    S->cv_build.notify_all();   // a worker waiting for admission must not take the only wake-up
    return FKS_OK;
}

extern "C" int fks_server_submit_lookup(fks_server* S, uint32_t map_id, const uint64_t* d_queries, uint64_t m,
                                        uint32_t* d_vals_out, uint8_t* d_found_out, uint32_t missing,
                                        void* stream, uint64_t* req_id) {
    if (!S || (m && !d_queries)) return FKS_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (map_id >= S->maps.size()) return FKS_EINVAL;
    }
    hipEvent_t ready = nullptr;
    if (m) {
        if (int rc = mark_ready(stream, &ready)) return rc;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    const uint64_t id = S->reqs.size();
    fks_server::Req r;
    r.kind = 1;
    r.map_id = map_id;
    r.keys = d_queries;
    r.vals = nullptr;
    r.n = 0;
    r.seed = 0;
    r.m = m;
    r.out_vals = d_vals_out;
    r.out_found = d_found_out;
    r.missing = missing;
    r.ready = ready;
    r.t_submit = now_ms();
    if (S->first_submit < 0) S->first_submit = r.t_submit;
    S->reqs.push_back(r);
    if (req_id) *req_id = id;
    if (m == 0) {
        finish_req(S, id, FKS_OK, r.t_submit);
        S->cv_done.notify_all();
        return FKS_OK;
    }
    S->maps[map_id].pins++;
    S->lookup_q.push_back(id);
    S->cv_lookup.notify_one();
    return FKS_OK;
}

extern "C" int fks_server_poll(fks_server* S, uint64_t req_id, int* done, int* status, double* latency_ms) {
    if (!S) return FKS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (req_id >= S->reqs.size()) return FKS_EINVAL;
    const auto& r = S->reqs[req_id];
    if (done) *done = r.done ? 1 : 0;
    if (status) *status = r.status;
    if (latency_ms) *latency_ms = r.done ? r.t_done - r.t_submit : -1.0;
    return FKS_OK;
}

extern "C" int fks_server_wait_all(fks_server* S) {
    if (!S) return FKS_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->n_done == S->reqs.size(); });
    return FKS_OK;
}

extern "C" int fks_server_latencies(fks_server* S, double* h_submit_ms, double* h_done_ms, int32_t* h_kind,
                                    int32_t* h_status, uint64_t max_entries) {
    if (!S) return FKS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    const uint64_t n = std::min<uint64_t>(max_entries, S->reqs.size());
    for (uint64_t i = 0; i < n; ++i) {
        const auto& r = S->reqs[i];
        if (h_submit_ms) h_submit_ms[i] = r.t_submit;
        if (h_done_ms) h_done_ms[i] = r.done ? r.t_done : -1.0;
        if (h_kind) h_kind[i] = r.kind;
        if (h_status) h_status[i] = r.status;
    }
    return (int)n;
}

extern "C" int fks_server_stats(fks_server* S, fks_server_stats_t* st) {
    if (!S || !st) return FKS_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(st, 0, sizeof(*st));
    st->requests = S->reqs.size();
    st->completed = S->n_done;
    st->lookup_launches = S->launches;
    st->graph_replays = S->graph_replays;
    st->graphs_captured = S->graph_captures;
    st->coalesced_requests = S->coalesced;
    st->evictions = S->evictions;
    st->resident_bytes = S->used;
    st->queries_done = S->queries_done;
    st->keys_built = S->keys_built;
    st->span_ms = S->first_submit < 0 ? 0.0 : S->last_done - S->first_submit;
    uint32_t resident = 0;
    for (const auto& m : S->maps) resident += m.state == 2;
    st->resident_maps = resident;
    return FKS_OK;
}

extern "C" const fks_map* fks_server_map(fks_server* S, uint32_t map_id) {
    if (!S) return nullptr;
    std::lock_guard<std::mutex> lk(S->mu);
    if (map_id >= S->maps.size() || S->maps[map_id].state != 2) return nullptr;
    return S->maps[map_id].map;
}

extern "C" void fks_server_destroy(fks_server* S) {
    if (!S) return;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return S->n_done == S->reqs.size(); });
        S->stop = true;
    }
    S->cv_build.notify_all();
    S->cv_lookup.notify_all();
    for (int w = 0; w < kBuildWorkers; ++w) S->build_thr[w].join();
    S->lookup_thr.join();
    (void)hipStreamSynchronize(S->lookup_st);
    for (int w = 0; w < kBuildWorkers; ++w) (void)hipStreamSynchronize(S->build_st[w]);
    for (auto& kv : S->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& m : S->maps)
        if (m.map) fks_destroy(m.map);
    for (int k = 0; k < kRing; ++k) {
        (void)hipHostFree(S->h_tab[k]);
        (void)hipFree(S->d_tab[k]);
        (void)hipEventDestroy(S->ev[k]);
    }
    for (int w = 0; w < kBuildWorkers; ++w) (void)hipStreamDestroy(S->build_st[w]);
    (void)hipStreamDestroy(S->lookup_st);
    (void)hipStreamDestroy(S->capture_st);
    (void)hipFree(S->arena.base);
    delete S;
}
