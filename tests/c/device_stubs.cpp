// Stand-ins for the library's device-side launchers (and its roctx ranges), so
// that its host-only code (bf_host.cpp, bf_stream.cpp) links into a program
// without device code: the sanitizer build of the C ABI harness, which calls
// only host-only entry points.  Each launcher returns an error; none is
// reached by that harness.
#include <hip/hip_runtime.h>

#include "../../paper_1702_04728_amd/csrc/bf_gate.h"
#include "../../paper_1702_04728_amd/csrc/bf_internal.h"
#include "../../paper_1702_04728_amd/csrc/bf_trace.h"

namespace bf {
hipError_t launch_fp32(const LaunchArgs&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_mfma(const LaunchArgs&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_fp32_up128(const LaunchArgs&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_mfma_up128(const LaunchArgs&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_stream_flags(const StreamState*, float*, uint8_t*, int, int, hipStream_t)
{
    return hipErrorNoBinaryForGpu;
}
hipError_t launch_ingest_gate(uint64_t, uint64_t, int32_t*, const uint32_t*, uint32_t*, uint32_t, hipStream_t)
{
    return hipErrorNoBinaryForGpu;
}
hipError_t launch_wall_clock_probe(uint64_t*, hipStream_t) { return hipErrorNoBinaryForGpu; }
void trace_push(const char*) {}
void trace_pop() {}
hipError_t noalloc_scratch(int, float2** out)
{
    *out = nullptr;
    return hipErrorNoBinaryForGpu;
}
}  // namespace bf
