// Named host ranges for tracing tools (rocprofv3 --marker-trace shows them
// beside the kernels they enclose): one per C-ABI call, per level of the
// host-driven level loops, per batch of a stacked call and per step of the
// served path's scheduler and lanes. Without a tool attached a range costs
// a call that returns at once.
#pragma once

#include <stdio.h>

#include <rocprofiler-sdk-roctx/roctx.h>

namespace rpq {

class TraceRange {
public:
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    TraceRange(const char *fmt, long long a) {
        char buf[96];
        snprintf(buf, sizeof buf, fmt, a);
        roctxRangePushA(buf);
    }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace rpq
