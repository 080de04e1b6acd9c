// roctx ranges around the library's entry points and passes, for tracing tools
// (rocprofv3 --marker-trace).  The ranges mark host-side enqueue spans; without
// a tool attached a push/pop costs a function call.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

namespace ss {

struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace ss
