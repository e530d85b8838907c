// Kernel timing instrumentation (internal): when a kind is enabled, each of
// its launches is bracketed by HIP events on the launching stream and the
// durations are accumulated for wg_profile_read.
#pragma once

#include "common.h"

namespace wg {
namespace prof {

bool on(int kind);
void record(int kind, hipStream_t s, double units, bool start);

// Records of this thread's launches carry the group last set here (0 by
// default); drop_group() removes the records of a group not yet drained, for
// launches that turned out to do nothing (an inner solve's iteration that was
// enqueued after the one that stopped it).
void set_group(unsigned long long g);
void drop_group(unsigned long long g);

// Device counters of the distance walk's tests (see wg_profile_walk_counts),
// or null while the walk's kind is not being timed.
unsigned long long *walk_counters();

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
