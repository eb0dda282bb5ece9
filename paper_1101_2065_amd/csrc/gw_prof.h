// Live kernel timing.  While a sink is installed on the calling host thread
// (gw_profile_begin), ProfScope brackets one kernel launch with HIP events on
// the launch's stream and records its algorithmic work; gw_profile_read sums
// per kernel class.  Launches recorded into a hipGraph are not timed.
#pragma once

#include <hip/hip_runtime.h>

namespace gwk {

struct ProfSink;
extern thread_local ProfSink *g_prof;

int prof_begin(ProfSink *s, hipStream_t st, const char *cls, double flops, double bytes);
void prof_end(ProfSink *s, hipStream_t st, int slot);

struct ProfScope {
    ProfSink *s;
    hipStream_t st;
    int slot = -1;
    ProfScope(hipStream_t st_, const char *cls, double flops, double bytes) : s(g_prof), st(st_) {
        if (s) slot = prof_begin(s, st, cls, flops, bytes);
    }
    ~ProfScope() {
        if (s && slot >= 0) prof_end(s, st, slot);
    }
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;
};

}  // namespace gwk
