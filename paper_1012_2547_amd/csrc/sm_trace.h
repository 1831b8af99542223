// Named host-side ranges for profilers (roctx): under rocprofv3 --marker-trace
// they show the phases of a search (count, writes, copies) on the timeline. A
// range is a few nanoseconds when no profiler is attached.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace sm {

struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace sm
