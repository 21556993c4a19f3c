// prof.hpp -- optional per-kernel timing with HIP events recorded on the
// launch stream around each launch (off unless hcn_profile_enable(1)).
#pragma once

#include <hip/hip_runtime.h>

namespace hcn {

bool prof_on();
// profiling held off on the calling thread while a ProfPause lives (entry
// points that must not create events)
void prof_pause(bool on);
struct ProfPause {
    ProfPause() { prof_pause(true); }
    ~ProfPause() { prof_pause(false); }
};
void prof_record(const char *name, hipEvent_t start, hipEvent_t stop);
hipEvent_t prof_event();

struct ProfScope {
    const char *name;
    hipStream_t stream;
    hipEvent_t start = nullptr;
    ProfScope(const char *n, hipStream_t s) : name(n), stream(s) {
        if (prof_on()) {
            start = prof_event();
            (void)hipEventRecord(start, stream);
        }
    }
    ~ProfScope() {
        if (start) {
            hipEvent_t stop = prof_event();
            (void)hipEventRecord(stop, stream);
            prof_record(name, start, stop);
        }
    }
};

}  // namespace hcn
