// Device side of the serving loop (beamform_stream).  Lossy ingest: after a
// frame's last launch, the output entry of every active slot whose frame did
// not arrive is zeroed, and every active entry's valid flag is written (kept
// out of the beamforming kernels, which only skip a missing slot).  Device-
// gated pacing: a one-wave wait on the receiver's arrival count.
#include <hip/hip_runtime.h>

#include "bf_gate.h"
#include "bf_internal.h"

namespace bf {
namespace {

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

// One lane polls the receiver's words with system-scope loads (they bypass
// the GPU caches, so the host's stores are seen), sleeping between polls; the
// device wall clock bounds the wait.
__global__ __launch_bounds__(64) void bf_ingest_gate_kernel(const uint32_t* gate, uint32_t target,
                                                            uint64_t max_ticks, int32_t* timed_out)
{
    if (threadIdx.x != 0) return;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        const uint32_t open = __hip_atomic_load(gate + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint32_t have = __hip_atomic_load(gate, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
        if (open != 0 || (int32_t)(have - target) >= 0) return;
        if (wall_clock64() - t0 > max_ticks) {
            *timed_out = 1;
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

}  // namespace

hipError_t launch_ingest_gate(const uint32_t* gate, uint32_t target, uint64_t max_ticks,
                              int32_t* timed_out, hipStream_t stream)
{
    hipLaunchKernelGGL(bf_ingest_gate_kernel, dim3(1), dim3(64), 0, stream, gate, target, max_ticks,
                       timed_out);
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
