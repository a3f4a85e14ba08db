// Device side of the serving loop (beamform_stream).  Lossy ingest: after a
// frame's last launch, the output entry of every active slot whose frame did
// not arrive is zeroed, and every active entry's valid flag is written (kept
// out of the beamforming kernels, which only skip a missing slot).  Device-
// gated pacing: a one-wave wait for a chunk's arrival time on the device's
// wall clock.
#include <hip/hip_runtime.h>

#include "bf_gate.h"
#include "bf_internal.h"

namespace bf {
namespace {

static_assert(sizeof(StreamState) <= 4 * 64 * kGateStateWordsPerLane, "gate copies the whole state");

constexpr int kFlagThreads = 256;

__global__ __launch_bounds__(kFlagThreads) void bf_stream_flags_kernel(const StreamState* st, float* out,
                                                                       uint8_t* out_valid, int max_slots)
{
    const int u = blockIdx.x;
    if (u >= st->n_active) return;
    const int32_t sv = st->slot[u];
    const bool missing = (sv & kSlotMissing) != 0;
    const size_t entry = (size_t)st->ring_index * max_slots + (sv & kSlotMask);
    if (out_valid && threadIdx.x == 0) out_valid[entry] = missing ? 0 : 1;
    if (missing) {
        float4* o = reinterpret_cast<float4*>(out + entry * kOutPerUnit);
        for (int i = threadIdx.x; i < kOutPerUnit / 4; i += kFlagThreads)
            o[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// The wave copies the launch's state into place, then one lane reads the
// device wall clock, sleeping between reads, until the chunk's arrival tick;
// the wait is bounded by max_ticks from its start.
__global__ __launch_bounds__(64) void bf_ingest_gate_kernel(uint64_t arrival_tick, uint64_t max_ticks,
                                                            int32_t* timed_out, const uint32_t* state_src,
                                                            uint32_t* state_dst, uint32_t state_words)
{
    // Branch-free so that all of a lane's loads are issued before one wait (one
    // host round trip) and the stores follow without waits: indices past the
    // end are clamped to the last word, which such lanes load and store again
    // with its own value.
    if (state_words > 0) {
        const uint32_t last = state_words - 1;
        uint32_t v[kGateStateWordsPerLane];
#pragma unroll
        for (int j = 0; j < kGateStateWordsPerLane; ++j)
            v[j] = __hip_atomic_load(state_src + min(threadIdx.x + 64u * j, last), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_SYSTEM);
#pragma unroll
        for (int j = 0; j < kGateStateWordsPerLane; ++j) state_dst[min(threadIdx.x + 64u * j, last)] = v[j];
    }
    if (threadIdx.x != 0) return;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        const uint64_t now = wall_clock64();
        if (now >= arrival_tick) return;
        if (now - t0 > max_ticks) {
            *timed_out = 1;
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// System-scope release store: visible to the host (out may be pinned host
// memory) once the kernel's completion has been observed.
__global__ __launch_bounds__(64) void bf_wall_clock_probe_kernel(uint64_t* out)
{
    if (threadIdx.x == 0) __hip_atomic_store(out, wall_clock64(), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace

hipError_t launch_ingest_gate(uint64_t arrival_tick, uint64_t max_ticks, int32_t* timed_out,
                              const uint32_t* state_src, uint32_t* state_dst, uint32_t state_words,
                              hipStream_t stream)
{
    if (state_words > 64 * kGateStateWordsPerLane) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bf_ingest_gate_kernel, dim3(1), dim3(64), 0, stream, arrival_tick, max_ticks,
                       timed_out, state_src, state_dst, state_words);
    return hipGetLastError();
}

hipError_t launch_wall_clock_probe(uint64_t* out, hipStream_t stream)
{
    hipLaunchKernelGGL(bf_wall_clock_probe_kernel, dim3(1), dim3(64), 0, stream, out);
    return hipGetLastError();
}

hipError_t launch_stream_flags(const StreamState* st, float* out, uint8_t* out_valid, int max_slots,
                               int n_active, hipStream_t stream)
{
    if (n_active <= 0) return hipSuccess;
    hipLaunchKernelGGL(bf_stream_flags_kernel, dim3(n_active), dim3(kFlagThreads), 0, stream, st, out,
                       out_valid, max_slots);
    return hipGetLastError();
}

}  // namespace bf
