// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "beamform.h"

namespace bf {

// Fixed geometry of the CHIME array as the kernels are specialised for it
// (Sec. 1, Sec. 2, Sec. 3.1 of the paper).
constexpr int kCyl = 4;
constexpr int kFeed = 256;
constexpr int kPol = 2;
constexpr int kInputs = kCyl * kFeed * kPol;  // 2048
constexpr int kPad = 2;
constexpr int kBins = kFeed * kPad;            // 512
constexpr int kBeamNS = 256;
constexpr int kBeamEW = 4;
constexpr int kBeams = kBeamNS * kBeamEW;      // 1024
constexpr int kUp = 16;                        // time-DFT length
constexpr int kOutPerUnit = kBeams * kUp;      // floats per channel-frame

// Everything a kernel launch needs; device pointers only.
struct LaunchArgs {
    const uint8_t* in;     // [n_frames][n_chan][n_time][2048]
    float* out;            // [n_frames][n_chan][1024][16]
    const int32_t* lut;    // [n_chan][256] kept bin per N-S beam
    const float2* ew;      // [n_chan][4][4] E-W weights W[j][c]
    const float2* tw;      // [32][16] N-S inter-stage twiddles w512^(b c)
    const void* mf;        // matrix-core tables (FP16 path), layout below
    int32_t n_chan;
    int32_t n_units;       // n_frames * n_chan channel-frames
    int32_t n_blk;         // n_time / 16
};

hipError_t launch_fp32(const LaunchArgs& a, hipStream_t stream);
hipError_t launch_mfma(const LaunchArgs& a, hipStream_t stream);

// Matrix-core tables of the FP16 path, in per-lane fragment order:
//   [8][64] x 8 halves  stage-1 DFT-32 block, tile tau in 0..3, hi then lo
//   [4][64] x 8 halves  stage-2 DFT-16 block, tile mu in 0..1, hi then lo
//   [64][8] float2      per-lane inter-stage twiddles w512^(b c)
constexpr size_t kMfmaTableBytes = (8 * 64 + 4 * 64) * 16 + 64 * 8 * 8;
void build_mfma_tables(void* host_buf);

}  // namespace bf

struct bf_plan {
    bf_config cfg{};                 // host-array pointers cleared; copies below
    std::vector<double> cyl_x, sin_theta, sin_phi, freqs;
    std::vector<int32_t> lut;        // [n_chan][256]
    int32_t n_chan = 0;
    int device = 0;
    int32_t* d_lut = nullptr;
    float2* d_ew = nullptr;
    float2* d_tw = nullptr;
    void* d_mf = nullptr;
    std::string err;
};
