// trace.hpp -- named host-side ranges (ROCTx) around the solvers' phases.
//
// A profiler that records markers (rocprofv3 --marker-trace) shows each range
// with its host start and end, nested under the entry point that opened it,
// beside the kernels launched inside it. With no tool attached a range costs
// two calls into a library that returns at once. Ranges are per host thread.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace pcgmi {

class Range {
public:
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

}  // namespace pcgmi
