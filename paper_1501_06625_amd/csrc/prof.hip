// prof.hip -- storage and query of the per-kernel event timings.
#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "prof.hpp"

namespace hcn {
namespace {
struct Rec {
    const char *name;
    hipEvent_t a, b;
};
std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
thread_local int g_paused = 0;
}  // namespace

bool prof_on() { return g_paused == 0 && g_on.load(std::memory_order_relaxed); }

void prof_pause(bool on) { g_paused += on ? 1 : -1; }

hipEvent_t prof_event() {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void prof_record(const char *name, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.push_back(Rec{name, a, b});
}

}  // namespace hcn

using namespace hcn;

extern "C" {

int hcn_profile_enable(int on) {
    g_on.store(on != 0);
    return HCN_OK;
}

int hcn_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &r : g_recs) {
        (void)hipEventSynchronize(r.b);
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    return HCN_OK;
}

int hcn_profile_query(const char *kernel, double *total_ms, int64_t *launches) {
    if (!kernel || !total_ms || !launches) return HCN_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto &r : g_recs) {
        if (std::strcmp(r.name, kernel) != 0) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return HCN_EDEVICE;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return HCN_EDEVICE;
        tot += ms;
        ++cnt;
    }
    *total_ms = tot;
    *launches = cnt;
    return HCN_OK;
}

}  // extern "C"
