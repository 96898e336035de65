// Named host-side ranges (ROCTx) around the solves and the phases of the
// time step.  A profiler run with marker tracing (rocprofv3 --marker-trace)
// records them on the host timeline beside the kernels; a range covers the
// host's enqueueing and waiting, not the kernels' own execution.  Without a
// profiler attached a range costs two calls that return at once.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

namespace dg {

class TraceRange {
public:
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace dg
