// Host-side trace ranges (roctx): plan creation, the power iteration, the
// FISTA solve and the server's steps and plan builds appear as named ranges
// on the host timeline of `rocprofv3 --marker-trace`, beside the kernels of
// `--kernel-trace`.  Without a profiler attached a range costs two calls
// into the roctx library.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace sl1m {

// One roctx range over the enclosing host scope.
class TraceRange {
 public:
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace sl1m
