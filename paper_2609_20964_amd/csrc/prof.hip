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
    unsigned long long group;
};

std::atomic<unsigned> g_mask{0};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
thread_local Rec t_open[WG_PROF_KINDS];
thread_local unsigned long long t_group = 0;

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

// Walk test counters on the device they were first asked for on (allocated
// once, while profiling, and kept until the process ends).
unsigned long long *g_walk = nullptr;
constexpr int kWalkCounts = 4;

}  // namespace

bool on(int kind) { return kind >= 0 && kind < WG_PROF_KINDS && ((g_mask.load() >> kind) & 1u); }

void set_group(unsigned long long g) { t_group = g; }

void drop_group(unsigned long long g) {
    if (g == 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_recs.begin(); it != g_recs.end();) {
        if (it->group == g) {
            g_pool.push_back(it->a);
            g_pool.push_back(it->b);
            it = g_recs.erase(it);
        } else {
            ++it;
        }
    }
}

unsigned long long *walk_counters() {
    if (!on(WG_PROF_SDF)) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_walk) {
        WG_HIP(hipMalloc(&g_walk, kWalkCounts * sizeof(unsigned long long)));
        WG_HIP(hipMemset(g_walk, 0, kWalkCounts * sizeof(unsigned long long)));
    }
    return g_walk;
}

void record(int kind, hipStream_t s, double units, bool start) {
    std::lock_guard<std::mutex> lk(g_mu);
    Rec &o = t_open[kind];
    if (start) {
        o.kind = kind;
        o.units = units;
        o.group = t_group;
        o.a = take_event();
        WG_HIP(hipEventRecord(o.a, s));
    } else {
        o.b = take_event();
        WG_HIP(hipEventRecord(o.b, s));
        g_recs.push_back(o);
        if (g_recs.size() > 4096) drain_locked();
    }
}

// Streaming copy: a workgroup moves 4 x 256 consecutive 16-byte vectors, each
// thread four of them 4 KiB apart (all four loads issued before the stores);
// one pass, no grid stride.
__global__ __launch_bounds__(256) void k_stream_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                      size_t n4) {
    const size_t i = (size_t)blockIdx.x * 1024 + threadIdx.x;
    if (i + 768 < n4) {
        const float4 a = src[i], b = src[i + 256], c = src[i + 512], d = src[i + 768];
        dst[i] = a;
        dst[i + 256] = b;
        dst[i + 512] = c;
        dst[i + 768] = d;
    } else {
        for (size_t k = i; k < n4; k += 256) dst[k] = src[k];
    }
}

}  // namespace prof
}  // namespace wg

extern "C" {

int wg_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream) {
    if (!dst || !src || bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0) return WG_EINVAL;
    if (bytes == 0) return WG_OK;
    const size_t n4 = bytes / 16;
    const size_t blocks = (n4 + 1023) / 1024;
    if (blocks > 0x7fffffffu) return WG_EINVAL;
    wg::prof::k_stream_copy<<<(unsigned)blocks, 256, 0, (hipStream_t)hip_stream>>>(
        static_cast<const float4 *>(src), static_cast<float4 *>(dst), n4);
    return hipGetLastError() == hipSuccess ? WG_OK : WG_EDEVICE;
}

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
        if (wg::prof::g_walk) {
            WG_HIP(hipDeviceSynchronize());
            WG_HIP(hipMemset(wg::prof::g_walk, 0, wg::prof::kWalkCounts * sizeof(unsigned long long)));
        }
    } catch (...) {
    }
}

int wg_profile_walk_counts(uint64_t out[4]) {
    if (!out) return WG_EINVAL;
    try {
        std::lock_guard<std::mutex> lk(wg::prof::g_mu);
        for (int k = 0; k < wg::prof::kWalkCounts; ++k) out[k] = 0;
        if (wg::prof::g_walk) {
            WG_HIP(hipDeviceSynchronize());
            WG_HIP(hipMemcpy(out, wg::prof::g_walk, wg::prof::kWalkCounts * sizeof(uint64_t), hipMemcpyDeviceToHost));
        }
        return WG_OK;
    } catch (const wg::Error &e) {
        return e.code;
    }
}

}  // extern "C"
