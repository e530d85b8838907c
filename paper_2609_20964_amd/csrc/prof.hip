// Kernel timing instrumentation (see prof.h and wg_profile_* in wgeo.h).
#include <atomic>
#include <mutex>
#include <vector>

#include "prof.h"

namespace wg {
namespace prof {

namespace {

struct Rec {
    int kind;
    hipEvent_t a, b;
    double units;
};

std::atomic<unsigned> g_mask{0};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
thread_local Rec t_open[WG_PROF_KINDS];

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence (no cache writeback at the marker)
    hipEvent_t e;
    WG_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    return e;
}

struct Totals {
    double ms = 0, units = 0;
    int64_t launches = 0;
} g_tot[WG_PROF_KINDS];

// Resolve every finished record into the totals (waits for the events).
void drain_locked() {
    for (auto &r : g_recs) {
        WG_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        WG_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        g_tot[r.kind].ms += ms;
        g_tot[r.kind].units += r.units;
        g_tot[r.kind].launches += 1;
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
}

}  // namespace

bool on(int kind) { return kind >= 0 && kind < WG_PROF_KINDS && ((g_mask.load() >> kind) & 1u); }

void record(int kind, hipStream_t s, double units, bool start) {
    std::lock_guard<std::mutex> lk(g_mu);
    Rec &o = t_open[kind];
    if (start) {
        o.kind = kind;
        o.units = units;
        o.a = take_event();
        WG_HIP(hipEventRecord(o.a, s));
    } else {
        o.b = take_event();
        WG_HIP(hipEventRecord(o.b, s));
        g_recs.push_back(o);
        if (g_recs.size() > 4096) drain_locked();
    }
}

}  // namespace prof
}  // namespace wg

extern "C" {

void wg_profile_enable(unsigned kinds_mask) { wg::prof::g_mask.store(kinds_mask); }

int wg_profile_read(int kind, double *total_ms, int64_t *launches, double *units) {
    if (kind < 0 || kind >= WG_PROF_KINDS) return WG_EINVAL;
    try {
        std::lock_guard<std::mutex> lk(wg::prof::g_mu);
        wg::prof::drain_locked();
        const auto &t = wg::prof::g_tot[kind];
        if (total_ms) *total_ms = t.ms;
        if (launches) *launches = t.launches;
        if (units) *units = t.units;
        return WG_OK;
    } catch (const wg::Error &e) {
        return e.code;
    }
}

void wg_profile_reset(void) {
    try {
        std::lock_guard<std::mutex> lk(wg::prof::g_mu);
        wg::prof::drain_locked();
        for (auto &t : wg::prof::g_tot) t = {};
    } catch (...) {
    }
}

}  // extern "C"
