// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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

constexpr int kAccPerThreadMax = 64;          // per-bin power accumulators per thread (max over kernels)
constexpr int kPartialPerWg = 256 * kAccPerThreadMax;  // floats of one workgroup's partial sums

// Device state of one streaming launch (see beamform_stream).
struct StreamState {
    int32_t ring_index;    // ring entry of the frame this launch belongs to
    int32_t chunk_index;   // chunk of the frame
    int32_t n_chunks;      // chunks per frame
    int32_t n_active;      // active slots; slot[0 .. n_active) are processed
    int32_t slot[BF_STREAM_MAX_SLOTS];  // slot index, | kSlotMissing when its frame is missing
};
// A slot whose current frame did not arrive complete: its output entry is
// zeroed (and flagged invalid) instead of beamformed.
constexpr int32_t kSlotMissing = 1 << 30;
constexpr int32_t kSlotMask = kSlotMissing - 1;
constexpr size_t kStreamStateHeader = 4 * sizeof(int32_t);

// Everything a kernel launch needs; device pointers only.
//   batch mode (st == nullptr): unit u = frame * n_chan + chan reads
//     in[u][n_blk * 16][2048], writes out[u][1024][16], tables row u % n_chan;
//   stream mode: unit u < st->n_active is slot st->slot[u], ring entry
//     e = st->ring_index * max_slots + slot; it reads samples
//     [chunk_index * n_blk * 16, +n_blk * 16) of in[e][n_time][2048], tables
//     row slot, keeps per-bin partial sums in partial[slot][4][kPartialPerWg]
//     between chunks and writes out[e] at the frame's last chunk.
// With ew_by_unit (batch mode only) the E-W weights are per channel-frame:
// row u of ew instead of row u % n_chan (tracking beams).
struct LaunchArgs {
    const uint8_t* in;
    float* out;
    const int32_t* lut;    // [rows][256] kept bin per N-S beam
    const float2* ew;      // [rows][4][4] E-W weights W[j][c]
    const float2* tw;      // [32][16] N-S inter-stage twiddles w512^(b c)
    const void* mf;        // matrix-core tables (FP16 path), layout below
    const StreamState* st; // stream mode state, or nullptr
    float* partial;        // stream mode partial sums
    int32_t n_chan;
    int32_t n_units;       // batch mode: n_frames * n_chan; stream mode: max_slots
    int32_t n_blk;         // 16-sample blocks per launch
    int32_t n_time;        // stream mode: samples per frame (ring entry stride)
    int32_t max_slots;     // stream mode: slots per ring entry
    int32_t sym_ew;        // 1: x[3-c] = -x[c] and sin(phi[3-j]) = -sin(phi[j]) exactly
    int32_t cyl_sym;       // 1: x[3-c] = -x[c] exactly (W[j][3-c] = conj W[j][c] for any phi)
    int32_t split_v;       // matrix-core path: 1 = E-W output also as hi + lo (FP32-class)
    int32_t ew_by_unit;    // 1: ew has one row per unit (batch mode)
    // 8-bit output (batch mode): out_u8[u][1024][16] = clamp(rint(P scale + offset))
    // with scale/offset rows u % n_chan; out is unused when out_u8 is set
    uint8_t* out_u8;
    const float* scale;
    const float* offset;
    // Complex beams out (batch mode, the pre-detection beams): instead of
    // integrating power, the kept beams of every (16-sample block it,
    // sub-channel k, line (p, j)) go to fine[unit][it][k][p * 4 + j][m]
    // (complex FP32).
    float2* fine;
    // 128-point up-channelisation: tw128[m] = w128^m, m < 128 (FP64 rounded
    // once)
    const float2* tw128;
};

// Rows (channel-frames) of the fixed E-W weight table of the allocation-free
// tracking entry point, and the devices whose copy of it can be addressed.
constexpr int kNoAllocRows = BF_NOALLOC_MAX_ROWS;
constexpr int kMaxDevices = 64;
// Device address of the calling device's fixed table (looked up on the first
// call for that device, which must be current; cached afterwards).
hipError_t noalloc_scratch(int device, float2** out);

hipError_t launch_fp32(const LaunchArgs& a, hipStream_t stream);
hipError_t launch_mfma(const LaunchArgs& a, hipStream_t stream);
// Serving loop, after a frame's last launch: zero the output entries of the
// active slots marked missing in st and write out_valid (optional,
// [depth][max_slots]) for every active slot; grid of n_active workgroups.
hipError_t launch_stream_flags(const StreamState* st, float* out, uint8_t* out_valid, int max_slots,
                               int n_active, hipStream_t stream);
// The 128-point up-channelisation in one pass (batch mode, n_time % 128 == 0).
hipError_t launch_fp32_up128(const LaunchArgs& a, hipStream_t stream);
hipError_t launch_mfma_up128(const LaunchArgs& a, hipStream_t stream);

// Matrix-core tables of the FP16 path, in per-lane fragment order:
//   [8][64] x 8 halves  stage-1 DFT-32 block, tile tau in 0..3, hi then lo
//   [4][64] x 8 halves  stage-2 DFT-16 block, tile mu in 0..1, hi then lo
//   [64][8] float2      per-lane inter-stage twiddles w512^(b c)
constexpr size_t kMfmaTableBytes = (8 * 64 + 4 * 64) * 16 + 64 * 8 * 8;
void build_mfma_tables(void* host_buf);

}  // namespace bf
