// Per-kernel timing with HIP events, recorded on the stream each kernel is
// launched on.  Off by default; when on, every library launch is bracketed by
// two events and the elapsed times are folded into per-kernel totals when the
// caller reads them.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "prof.hpp"

namespace fks {

namespace {

struct Pending {
    const char* name;
    hipEvent_t start, stop;
};

struct Total {
    std::string name;
    uint64_t launches = 0;
    double ms = 0.0;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_free;
std::vector<Total> g_totals;

hipEvent_t take_event() {
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void fold_locked() {
    for (auto& p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            Total* t = nullptr;
            for (auto& x : g_totals)
                if (x.name == p.name) t = &x;
            if (!t) {
                g_totals.push_back(Total{p.name, 0, 0.0});
                t = &g_totals.back();
            }
            t->launches += 1;
            t->ms += ms;
        }
        g_free.push_back(p.start);
        g_free.push_back(p.stop);
    }
    g_pending.clear();
}

}  // namespace

bool prof_on() { return g_on; }

ProfScope::ProfScope(const char* name, hipStream_t st) : name_(name), st_(st) {
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    start_ = take_event();
    stop_ = take_event();
    if (start_ && stop_) (void)hipEventRecord(start_, st_);
}

ProfScope::~ProfScope() {
    if (!start_ || !stop_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipEventRecord(stop_, st_);
    g_pending.push_back(Pending{name_, start_, stop_});
    // keep the pending list short: fold once it grows
    if (g_pending.size() > 4096) fold_locked();
}

}  // namespace fks

extern "C" {

int fks_prof_enable(int on) {
    std::lock_guard<std::mutex> lk(fks::g_mu);
    fks::g_on = on != 0;
    return FKS_OK;
}

void fks_prof_reset(void) {
    std::lock_guard<std::mutex> lk(fks::g_mu);
    fks::fold_locked();
    fks::g_totals.clear();
}

int fks_prof_read(fks_prof_entry* out, int max_entries) {
    std::lock_guard<std::mutex> lk(fks::g_mu);
    fks::fold_locked();
    int n = (int)fks::g_totals.size();
    if (!out) return n;
    int k = 0;
    for (; k < n && k < max_entries; ++k) {
        std::memset(&out[k], 0, sizeof(out[k]));
        std::strncpy(out[k].name, fks::g_totals[k].name.c_str(), sizeof(out[k].name) - 1);
        out[k].launches = fks::g_totals[k].launches;
        out[k].total_ms = fks::g_totals[k].ms;
    }
    return k;
}

}  // extern "C"
