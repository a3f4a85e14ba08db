// Named host range around one API call (roctx, bf_trace.cpp): shown by
// rocprofv3 --marker-trace on the host timeline next to the call's kernels.
#pragma once

namespace bf {

void trace_push(const char* name);
void trace_pop();

struct TraceRange {
    explicit TraceRange(const char* name) { trace_push(name); }
    ~TraceRange() { trace_pop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace bf
