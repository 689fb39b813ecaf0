// Named host-side ranges for profilers (roctx): a range covers one call of
// the C ABI or one phase of it (session set-up, a replayed window of steps,
// container assembly, the forward / adjoint / update launches of a step).
// rocprofv3 --marker-trace records them beside the kernel trace; with no
// profiler attached a range costs two calls into the roctx library.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

namespace edpc {

struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace edpc
