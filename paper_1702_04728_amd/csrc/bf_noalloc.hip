// Fixed device workspace of the allocation-free tracking entry point
// (beamform_frame_tracking_noalloc): the per-channel-frame E-W weight table
// lives in a file-scope device array instead of plan-owned allocations.
//
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and only that address is ever handed to a kernel or a
// copy.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bf_internal.h"

namespace {

// [kNoAllocRows][4][4] complex E-W weights (2 MiB); every GPU the library runs
// on holds its own copy until the process ends.
static __device__ __align__(256) float2 scratch[bf::kNoAllocRows * bf::kBeamEW * bf::kCyl];

std::mutex g_scratch_mutex;
float2* g_scratch_ptr[bf::kMaxDevices] = {};

}  // namespace

namespace bf {

hipError_t noalloc_scratch(int device, float2** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<float2*>(ptr);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace bf
