// Named ranges around the C-ABI entry points, for profilers that collect
// ROCTx markers (rocprofv3 --marker-trace shows each call with its name).
// Without a profiler attached a push/pop pair is two calls into an inert
// library; nothing is recorded and nothing touches the GPU.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace lps {

struct ApiRange {
  explicit ApiRange(const char* name) { roctxRangePushA(name); }
  ~ApiRange() { roctxRangePop(); }
  ApiRange(const ApiRange&) = delete;
  ApiRange& operator=(const ApiRange&) = delete;
};

}  // namespace lps

// Opens a range named after the enclosing entry point; it closes on every
// return path.
#define LPS_API_RANGE() ::lps::ApiRange lps_api_range_(__func__)
