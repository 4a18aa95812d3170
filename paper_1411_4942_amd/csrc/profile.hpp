// Optional per-kernel timing with HIP events recorded on the launch stream.
// Off by default; pm_profile_enable(1) turns it on for the process.
#pragma once

#include <hip/hip_runtime.h>

namespace pm {

bool profiling();

// Records a start event on construction and a stop event on destruction,
// both on stream s, when profiling is on.
class ProfScope {
public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

private:
    const char *name_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace pm
