// m1_trace.hpp -- named ranges on the host timeline (roctx): time steps, 3-D time
// steps and engine rounds show up as ranges in a marker trace of the profiler.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace m1 {

// Push a range for the lifetime of the object.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace m1
