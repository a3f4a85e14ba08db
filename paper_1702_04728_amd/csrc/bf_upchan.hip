// Second pass of the paper's own up-channelisation (Sec. 3: a fine
// channelisation by 128 times to 3 kHz, then Stokes I integrated to 16 sub-
// channels of 24.4 kHz per 0.983 ms; Sec. 3.2: every 128 samples transformed
// by an FFT).
//
// The first pass (the beamforming kernels in their `fine` mode) runs the time
// transform first, as for the 16-point path, but over the samples u + 8 tau of
// each 128-sample block b: after E-W and N-S beamforming (linear, so they
// commute with the time transform) it leaves, per beam and pol,
//   Y_u[k] = sum_tau x[128 b + u + 8 tau] w16^(k tau),   u < 8, k < 16.
// The 128-point DFT of the block then splits, with s' = k + 16 r, as
//   X[s'] = sum_u w8^(r u) (w128^(u k) Y_u[k]),
// a twiddle and an 8-point DFT over u.  Fine bin s' is centre-shifted to
// q' = (s' + 64) mod 128 and summed, squared, over both pols and the frame's
// blocks into sub-channel q = ((q' + 4) / 8) mod 16 (the 8 fine channels
// nearest its centre).
//
// One thread per (channel-frame, E-W beam j, N-S beam m); consecutive threads
// take consecutive m, so every load is 64 lanes x 8 B contiguous, and all of a
// thread's fine bins and sub-channel sums stay in its registers.
#include <hip/hip_runtime.h>

#include "bf_device.h"

namespace bf {
namespace {

using namespace dev;

constexpr int kUpThreads = 256;

// In-place 8-point DFT, natural order: y[r] <- sum_u y[u] w8^(r u).
__device__ __forceinline__ void dft8(float2 (&y)[8])
{
    dft4(y[0], y[2], y[4], y[6]);  // even samples: E[r] in y[0], y[2], y[4], y[6]
    dft4(y[1], y[3], y[5], y[7]);  // odd samples: O[r] in y[1], y[3], y[5], y[7]
    const float2 e[4] = {y[0], y[2], y[4], y[6]};
    const float2 o[4] = {y[1], tw32<4>(y[3]), tw32<8>(y[5]), tw32<12>(y[7])};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        y[r] = cadd(e[r], o[r]);
        y[r + 4] = csub(e[r], o[r]);
    }
}

__global__ __launch_bounds__(kUpThreads) void bf_upchan128_kernel(UpchanArgs a)
{
    const long long gid = (long long)blockIdx.x * kUpThreads + threadIdx.x;
    const int unit = (int)(gid >> 10);
    if (unit >= a.n_units) return;
    const int beam = (int)(gid & 1023), j = beam >> 8, m = beam & 255;

    float acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.f;
    const float2* base = a.fine + (size_t)unit * a.n_blk128 * 8 * kFinePerIter;
    for (int p = 0; p < 2; ++p) {
        const float2* line = base + (size_t)(p * 4 + j) * kBeamNS + m;
        for (int b = 0; b < a.n_blk128; ++b) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                float2 y[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    y[u] = line[((size_t)(b * 8 + u) * 16 + k) * 8 * kBeamNS];
#pragma unroll
                for (int u = 1; u < 8; ++u) y[u] = cmul(y[u], a.tw128[u * 16 + k]);
                dft8(y);
                // fine bin k + 16 r -> sub-channel ((k + 4) / 8 + 8 + 2 r) mod 16
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int q = ((k + 4) / 8 + 8 + 2 * r) & 15;
                    acc[q] = fmaf(y[r].x, y[r].x, fmaf(y[r].y, y[r].y, acc[q]));
                }
            }
        }
    }

    float4* dst = reinterpret_cast<float4*>(a.out + ((size_t)unit * kBeams + beam) * kUp);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        dst[i] = make_float4(acc[4 * i], acc[4 * i + 1], acc[4 * i + 2], acc[4 * i + 3]);
}

}  // namespace

hipError_t launch_upchan128(const UpchanArgs& a, hipStream_t stream)
{
    if (a.n_units <= 0) return hipSuccess;
    UpchanArgs args = a;
    void* params[] = {&args};
    const long long threads = (long long)a.n_units * kBeams;
    const dim3 grid((unsigned)((threads + kUpThreads - 1) / kUpThreads));
    return hipLaunchKernel(reinterpret_cast<const void*>(&bf_upchan128_kernel), grid,
                           dim3(kUpThreads), params, 0, stream);
}

}  // namespace bf
