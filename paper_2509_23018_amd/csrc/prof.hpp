// Optional HIP-event timing of the library's own kernel launches (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gw {

bool prof_on();
void prof_enable(bool on);
void prof_reset();
// Sum of recorded durations for `name` (waits for the recorded events).
void prof_read(const char* name, int64_t* launches, double* total_ms);

// Records a start event on construction and an end event on destruction,
// both on stream s, when profiling is enabled.  Wrap exactly one launch.
class ProfScope {
public:
    ProfScope(const char* name, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

private:
    const char* name_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr;
};

}  // namespace gw
