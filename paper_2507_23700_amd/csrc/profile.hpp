// Optional per-phase timing: hipEvent pairs recorded on the launch stream
// around each kernel phase while profiling is enabled.
#pragma once

#include <hip/hip_runtime.h>

namespace ax {

bool profiling();
void prof_record(const char *name, hipEvent_t a, hipEvent_t b);
hipEvent_t prof_event();

// Records a start event on construction and a stop event on destruction.
struct ProfScope {
    const char *name;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(const char *n, hipStream_t st) : name(n), s(st)
    {
        if (profiling()) {
            a = prof_event();
            b = prof_event();
            if (a && b)
                (void)hipEventRecord(a, s);
        }
    }
    ~ProfScope()
    {
        if (a && b) {
            (void)hipEventRecord(b, s);
            prof_record(name, a, b);
        }
    }
};

}  // namespace ax
