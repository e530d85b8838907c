// Kernel timing instrumentation (internal): when a kind is enabled, each of
// its launches is bracketed by HIP events on the launching stream and the
// durations are accumulated for wg_profile_read.
#pragma once

#include "common.h"

namespace wg {
namespace prof {

bool on(int kind);
void record(int kind, hipStream_t s, double units, bool start);

// RAII bracket around one launch.
struct Scope {
    int kind;
    hipStream_t s;
    double units;
    bool active;
    Scope(int k, hipStream_t st, double u) : kind(k), s(st), units(u), active(on(k)) {
        if (active) record(kind, s, units, true);
    }
    ~Scope() {
        if (active) record(kind, s, units, false);
    }
};

}  // namespace prof
}  // namespace wg
