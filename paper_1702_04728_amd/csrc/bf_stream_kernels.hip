// Device side of the serving loop's lossy ingest (beamform_stream): after a
// frame's last launch, the output entry of every active slot whose frame did
// not arrive is zeroed, and every active entry's valid flag is written.  Kept
// out of the beamforming kernels, which only skip a missing slot.
#include <hip/hip_runtime.h>

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

}  // namespace

hipError_t launch_stream_flags(const StreamState* st, float* out, uint8_t* out_valid, int max_slots,
                               int n_active, hipStream_t stream)
{
    if (n_active <= 0) return hipSuccess;
    hipLaunchKernelGGL(bf_stream_flags_kernel, dim3(n_active), dim3(kFlagThreads), 0, stream, st, out,
                       out_valid, max_slots);
    return hipGetLastError();
}

}  // namespace bf
