// roctx ranges around the library's API calls: with a tracing tool attached
// (rocprofv3 --marker-trace) each call shows as a named range on the host
// timeline next to the kernels it launched; without one a push or pop is a
// call into the roctx library that returns at once.
#include <rocprofiler-sdk-roctx/roctx.h>

#include "bf_trace.h"

namespace bf {

void trace_push(const char* name) { (void)roctxRangePushA(name); }
void trace_pop() { (void)roctxRangePop(); }

}  // namespace bf
