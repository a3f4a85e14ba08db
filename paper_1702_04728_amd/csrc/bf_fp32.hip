// FP32 FFT path of the hybrid beamformer, one fused kernel.
//
// What is computed (paper Sec. 3, Sec. 3.1, Sec. 3.2): for every channel-frame
// (384 samples x 2048 inputs of 4+4-bit complex voltages), Stokes-I power of
// 1024 beams (256 N-S FFT beams clamped to the desired pointings x 4 E-W beams
// by exact phasing) in 16 up-channelised sub-channels, integrated over the
// frame's 24 blocks of 16 samples.
//
// All stages are linear up to the detector, and each acts on its own axis:
// the time DFT on samples, E-W phasing on cylinders, the N-S transform on
// feeds.  They therefore commute, and this kernel applies them in the order
// that keeps data on chip: time DFT first (on the raw integer samples), then
// E-W phasing, then the zero-padded 512-point N-S transform, then |.|^2.
// Because the clamping only picks which N-S bins become output beams, power
// is integrated per FFT bin and the Eq. (1) bin table is applied once per
// frame when the result is written.  The paper's separate transpose kernel
// disappears: the time axis is consumed while the block is in registers.
//
// Decomposition: one workgroup (256 threads) per (channel-frame, s0), where
// s0 in [0, 4) selects the sub-channels s = s0 + 4*s2 (s2 in [0, 4)).  Per
// 16-sample block:
//   A  wave w takes (feed, pol) pairs 128 w .. 128 w + 127 of all four
//      cylinders: each lane reads 16 samples of 8 consecutive inputs of one
//      cylinder and forms their stride-4 sums (a DFT-4 over the sample stride,
//      exact integers); the rest of the time DFT (a twiddle and a DFT-4 over
//      the sample phase) and E-W phasing are then one fixed complex 16 x 16
//      matrix per (channel, class) per (feed, pol), applied on the matrix cores
//      (FP16 hi + lo matrix, exact integer operands, FP32 results: ~22
//      significant bits), and the E-W beams of all four sub-channels go to LDS
//      as FP32;
//   B1 each 16-lane group (s2, jp, p) reads the lines of E-W beams jp and
//      3 - jp of polarisation p (lane b holds feeds 16a + b);
//   B2 each group transforms its two lines: 512 = 32 x 16 with the upper half
//      of the input zero, so step 1 is a pruned 32-point DFT per lane (two
//      16-point FFTs), then twiddles w512^(b c), a 16-lane transpose through LDS
//      and a 16-point FFT per lane; |X|^2 accumulates in registers per line.
// After the last block the two polarisations' per-bin powers are summed in
// LDS and gathered by the bin table into out[beam][q].
#include <hip/hip_runtime.h>

#include "bf_device.h"

namespace bf {
namespace {

using namespace dev;

constexpr int kXpStride = 17;                    // padded row of a transpose buffer
constexpr int kXpBuf = 16 * kXpStride;           // float2 per buffer
// a group's {E, O} buffers plus 16 float2, so that consecutive groups start
// 32 banks apart (1120 words, not a multiple of 64)
constexpr int kGroupF2 = 2 * kXpBuf + 16;
constexpr int kUnionF2 = 16 * kGroupF2;          // 16 groups (8960 float2)
constexpr int kTF4 = 4 * 1024;                   // time-DFT output: 4 s2 x 1024 float4
static_assert(kUnionF2 * 8 >= kTF4 * 16, "union region must hold the time-DFT output");
static_assert(kUnionF2 * 8 >= 16 * 512 * 4, "union region must hold the per-bin powers");

// x (1 - i t): the tangent part of a twiddle w = cos(phi) (1 - i tan(phi)), two FMAs;
// the cosine is folded into the butterfly that follows.
__device__ __forceinline__ float2 tan_part(float2 x, float t)
{
    return make_float2(fmaf(t, x.y, x.x), fmaf(-t, x.x, x.y));
}
__device__ __forceinline__ float2 tan_part1(float2 x) { return make_float2(x.x + x.y, x.y - x.x); }

// Outputs of a radix-4 butterfly whose odd-input sums carry a common factor c:
// (t0 + c u2, t1 - i c u3, t0 - c u2, t1 + i c u3), as FMAs.
__device__ __forceinline__ void dft4_out(float2& o0, float2& o1, float2& o2, float2& o3, float2 t0,
                                         float2 t1, float2 u2, float2 u3, float c)
{
    o0 = make_float2(fmaf(c, u2.x, t0.x), fmaf(c, u2.y, t0.y));
    o2 = make_float2(fmaf(-c, u2.x, t0.x), fmaf(-c, u2.y, t0.y));
    o1 = make_float2(fmaf(c, u3.y, t1.x), fmaf(-c, u3.x, t1.y));
    o3 = make_float2(fmaf(-c, u3.y, t1.x), fmaf(c, u3.x, t1.y));
}

constexpr float kTan8 = 0.41421356237309504880f;   // tan(pi/8) = cos(3pi/8) / cos(pi/8)
constexpr float kTan38 = 2.41421356237309504880f;  // tan(3pi/8)

// In-place 16-point FFT, natural order in and out: v[k] <- sum_a v[a] w16^(a k).
// Radix 4 x 4: a = 4 a1 + a2, k = k1 + 4 k2.  The second step's twiddles
// w16^(a2 k1) = cos (1 - i tan) are applied as their tangent parts, the cosines
// folded into that step's butterflies (144 instructions instead of 160).
__device__ __forceinline__ void fft16(float2 (&v)[16])
{
#pragma unroll
    for (int a2 = 0; a2 < 4; ++a2) dft4(v[a2], v[4 + a2], v[8 + a2], v[12 + a2]);
    // element [4 k1 + a2] now holds u[a2][k1]; row k1 is the DFT-4 over a2 of
    // u[a2][k1] w16^(a2 k1)
    dft4(v[0], v[1], v[2], v[3]);
    {   // k1 = 1: w16^1 = C1 (1 - i tan(pi/8)), w16^2 = C2 (1 - i), w16^3 = C3 (1 - i tan(3pi/8))
        const float2 x0 = v[4], x1 = tan_part(v[5], kTan8), x2 = tan_part1(v[6]),
                     x3 = tan_part(v[7], kTan38);
        const float2 t0 = make_float2(fmaf(kR2, x2.x, x0.x), fmaf(kR2, x2.y, x0.y));
        const float2 t1 = make_float2(fmaf(-kR2, x2.x, x0.x), fmaf(-kR2, x2.y, x0.y));
        // C1 x1 +- C3 x3 = C1 (x1 +- tan(pi/8) x3)
        const float2 u2 = make_float2(fmaf(kTan8, x3.x, x1.x), fmaf(kTan8, x3.y, x1.y));
        const float2 u3 = make_float2(fmaf(-kTan8, x3.x, x1.x), fmaf(-kTan8, x3.y, x1.y));
        dft4_out(v[4], v[5], v[6], v[7], t0, t1, u2, u3, kC16_1);
    }
    {   // k1 = 2: w16^2 = C2 (1 - i), w16^4 = -i, w16^6 = -i C2 (1 - i)
        const float2 x0 = v[8], x1 = tan_part1(v[9]), x2 = v[10], x3 = tan_part1(v[11]);
        const float2 t0 = make_float2(x0.x + x2.y, x0.y - x2.x);   // x0 - i x2
        const float2 t1 = make_float2(x0.x - x2.y, x0.y + x2.x);   // x0 + i x2
        const float2 u2 = make_float2(x1.x + x3.y, x1.y - x3.x);   // x1 - i x3
        const float2 u3 = make_float2(x1.x - x3.y, x1.y + x3.x);   // x1 + i x3
        dft4_out(v[8], v[9], v[10], v[11], t0, t1, u2, u3, kR2);
    }
    {   // k1 = 3: w16^3 = C3 (1 - i tan(3pi/8)), w16^6 = -i C2 (1 - i), w16^9 = -C1 (1 - i tan(pi/8))
        const float2 x0 = v[12], x1 = tan_part(v[13], kTan38), x2 = tan_part1(v[14]),
                     x3 = tan_part(v[15], kTan8);
        const float2 t0 = make_float2(fmaf(kR2, x2.y, x0.x), fmaf(-kR2, x2.x, x0.y));  // x0 - i C2 x2
        const float2 t1 = make_float2(fmaf(-kR2, x2.y, x0.x), fmaf(kR2, x2.x, x0.y));  // x0 + i C2 x2
        // C3 x1 -+ C1 x3 = C1 (tan(pi/8) x1 -+ x3)
        const float2 u2 = make_float2(fmaf(kTan8, x1.x, -x3.x), fmaf(kTan8, x1.y, -x3.y));
        const float2 u3 = make_float2(fmaf(kTan8, x1.x, x3.x), fmaf(kTan8, x1.y, x3.y));
        dft4_out(v[12], v[13], v[14], v[15], t0, t1, u2, u3, kC16_1);
    }
    // element [4 k1 + k2] holds V[k1 + 4 k2]: transpose the 4 x 4 index
    float2 t;
    t = v[1]; v[1] = v[4]; v[4] = t;
    t = v[2]; v[2] = v[8]; v[8] = t;
    t = v[3]; v[3] = v[12]; v[12] = t;
    t = v[6]; v[6] = v[9]; v[9] = t;
    t = v[7]; v[7] = v[13]; v[13] = t;
    t = v[11]; v[11] = v[14]; v[14] = t;
}

// Zero-padded 512-point N-S transform of one line held as x[a] = line[16 a + b]
// by lane b of a 16-lane group; accumulates |X_k|^2 for k = 2 b + r + 32 d into
// acc[r][d].  bufE / bufO: this group's two transpose buffers (adjacent).
// kFine: instead, the kept beams of the line go to fine_dst (the pre-detection
// beams), gathered through the transpose buffers.
template <bool kFine>
__device__ __forceinline__ void ns_line_power(const float2 (&x)[16], float (&acc)[2][16],
                                              float2* __restrict__ bufE,
                                              float2* __restrict__ bufO,
                                              const float4* __restrict__ tw, int b,
                                              const int32_t (&lv)[kFine ? 16 : 1],
                                              float2* __restrict__ fine_dst)
{
    float2 E[16], O[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) E[a] = x[a];
    O[0] = x[0];
    O[1] = tw32<1>(x[1]);
    O[2] = tw32<2>(x[2]);
    O[3] = tw32<3>(x[3]);
    O[4] = tw32<4>(x[4]);
    O[5] = tw32<5>(x[5]);
    O[6] = tw32<6>(x[6]);
    O[7] = tw32<7>(x[7]);
    O[8] = tw32<8>(x[8]);
    O[9] = tw32<9>(x[9]);
    O[10] = tw32<10>(x[10]);
    O[11] = tw32<11>(x[11]);
    O[12] = tw32<12>(x[12]);
    O[13] = tw32<13>(x[13]);
    O[14] = tw32<14>(x[14]);
    O[15] = tw32<15>(x[15]);
    // step 1: Z[2c'] = E[c'], Z[2c'+1] = O[c'] is the pruned 32-point DFT over a
    fft16(E);
    fft16(O);
    // step 2: Z[c] *= w512^(b c) (tw[c' * 16 + b] holds the twiddles of bins
    // 2 c' and 2 c' + 1); step 3a: transpose through LDS
    // (twiddles read in batches of four, each issued a batch ahead of use)
    float4 w[2][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[0][i] = tw[i * 16 + b];
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
        if (c4 < 3) {
#pragma unroll
            for (int i = 0; i < 4; ++i) w[(c4 + 1) & 1][i] = tw[(4 * (c4 + 1) + i) * 16 + b];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = 4 * c4 + i;
            const float4 wc = w[c4 & 1][i];
            bufE[c * kXpStride + b] = cmul(E[c], make_float2(wc.x, wc.y));
            bufO[c * kXpStride + b] = cmul(O[c], make_float2(wc.z, wc.w));
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int bb = 0; bb < 16; ++bb) {
        E[bb] = bufE[b * kXpStride + bb];
        O[bb] = bufO[b * kXpStride + bb];
    }
    wave_lds_sync();
    // step 3b: 16-point FFT over b gives X[c + 32 d] for c = 2 b (E) and 2 b + 1 (O)
    fft16(E);
    fft16(O);
    if constexpr (kFine) {
        float2* bins = bufE;  // 512 bins fit in the group's two buffers
#pragma unroll
        for (int d = 0; d < 16; ++d) {
            bins[2 * b + 32 * d] = E[d];
            bins[2 * b + 1 + 32 * d] = O[d];
        }
        wave_lds_sync();
        write_fine_line<16>(bins, lv, fine_dst, b);
        wave_lds_sync();
    } else {
#pragma unroll
        for (int d = 0; d < 16; ++d) {
            acc[0][d] = fmaf(E[d].x, E[d].x, fmaf(E[d].y, E[d].y, acc[0][d]));
            acc[1][d] = fmaf(O[d].x, O[d].x, fmaf(O[d].y, O[d].y, acc[1][d]));
        }
    }
}
static_assert(2 * kXpBuf >= 512, "a group's transpose buffers must hold one line's bins");

// E-W phasing of a 16-lane group: lane b forms feeds 16 a + b of the group's two
// E-W beams (W[0], W[1]) of one polarisation from one time-DFT slice Tp (stride
// 2 float2 per slot: the other pol interleaved).  With kSym (mirror-symmetric
// geometry, the group's beams jp and 3 - jp) the pair shares its cylinder sums.
template <bool kSym>
__device__ __forceinline__ void ew_group(const float2* __restrict__ Tp, const float2 (&W)[2][4],
                                         float2 (&v0)[16], float2 (&v1)[16], int b)
{
#pragma unroll
    for (int aa = 0; aa < 16; ++aa) {
        float2 y[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) y[c] = Tp[2 * (c * 256 + 16 * aa + b)];
        if constexpr (kSym) {
            const float2 S0 = cadd(y[0], y[3]), S1 = cadd(y[1], y[2]);
            const float2 D0 = csub(y[0], y[3]), D1 = csub(y[1], y[2]);
            const float2 P = make_float2(fmaf(W[0][0].x, S0.x, W[0][1].x * S1.x),
                                         fmaf(W[0][0].x, S0.y, W[0][1].x * S1.y));
            const float2 Q = make_float2(fmaf(W[0][0].y, D0.x, W[0][1].y * D1.x),
                                         fmaf(W[0][0].y, D0.y, W[0][1].y * D1.y));
            v0[aa] = make_float2(P.x - Q.y, P.y + Q.x);
            v1[aa] = make_float2(P.x + Q.y, P.y - Q.x);
        } else {
            float2 p0 = make_float2(0.f, 0.f), p1 = make_float2(0.f, 0.f);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                p0 = cmac(p0, y[c], W[0][c]);
                p1 = cmac(p1, y[c], W[1][c]);
            }
            v0[aa] = p0;
            v1[aa] = p1;
        }
    }
}

// E-W output of the matrix-core step in LDS (float2 units): line (E-W beam j,
// pol p, sub-channel s0 + 4 s2) 16 p + 4 s2 + j at kEwLine apart; feed 16 a + b
// at 16 b + 2 ((a >> 1) ^ ((b >> 1) & 7)) + (a & 1), so that each group's
// 16-byte reads of consecutive a (one b per lane) spread over all banks.
constexpr int kEwLine = 258;
static_assert(kUnionF2 >= 32 * kEwLine, "union region must hold the E-W output");
__device__ __forceinline__ int ew_pos(int b, int a) { return 16 * b + 2 * ((a >> 1) ^ ((b >> 1) & 7)) + (a & 1); }

template <bool kFine>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void bf_fp32_kernel(LaunchArgs a)
{
    __shared__ __align__(16) float2 s_union[kUnionF2];
    __shared__ __align__(16) float4 s_tw[16 * 16];  // [c'][b]: w512^(b 2c'), w512^(b (2c'+1))
    // the (channel, class) matrix in fragment order [hi0, hi1, lo0, lo1][lane],
    // read back every block (in registers it would push the kernel past 256 VGPRs)
    __shared__ __align__(16) half8 s_G[4][64];

    const Work wk = work_of_block();
    UnitIO io;
    if (!resolve_unit(a, wk, io)) return;
    const int t = threadIdx.x;
    const int g = t >> 4;      // group: s2 = g >> 2 (= wave), jp = (g >> 1) & 1, p = g & 1
    const int b = t & 15;
    const int s2 = g >> 2, jp = (g >> 1) & 1, pol = g & 1;
    const int jl[2] = {jp, 3 - jp};  // the group's two E-W beams
    const int lane = t & 63, w = t >> 6, q = lane >> 4, n = lane & 15;

    {
        const int c2 = t >> 4, bb = t & 15;
        const float2 w0 = a.tw[(2 * c2) * 16 + bb], w1 = a.tw[(2 * c2 + 1) * 16 + bb];
        s_tw[t] = make_float4(w0.x, w0.y, w1.x, w1.y);
    }
    if (t < 64) {
        half8 Gh[2], Gl[2];
        load_ew_mats(a.ew + (size_t)io.ew_row * kBeamEW * kCyl, wk.s0, lane, Gh, Gl);
        s_G[0][lane] = Gh[0];
        s_G[1][lane] = Gh[1];
        s_G[2][lane] = Gl[0];
        s_G[3][lane] = Gl[1];
    }
    __syncthreads();

    const uint8_t* src = io.in;
    const int in_off = 512 * q + 128 * w + 8 * n;  // cylinder q, (feed, pol) 128 w + 8 n + e
    float2* bufE = s_union + g * kGroupF2;
    float2* bufO = bufE + kXpBuf;

    int32_t lv[kFine ? 16 : 1] = {};  // bin-table entries of the beams this lane writes
    if constexpr (kFine) load_lut_lane<16>(a.lut + (size_t)io.row * kBeamNS, lv, b);

    uint2 raw[16];
    load_block_at(block_base(src, 0), raw, in_off);

    float acc[2][2][16];  // [line l: beam jl[l]][E/O][d]
    constexpr int kAcc = sizeof(acc) / sizeof(float);
    if (io.first) {
#pragma unroll
        for (int l = 0; l < 2; ++l)
#pragma unroll
            for (int d = 0; d < 16; ++d) acc[l][0][d] = acc[l][1][d] = 0.f;
    } else {
        load_partial<kAcc>(&acc[0][0][0], io.partial, t);
    }

    for (int blk = 0; blk < a.n_blk; ++blk) {
        // A: stride-4 sums of this lane's 8 inputs, then the time-DFT tail and
        // E-W phasing on the matrix cores; tile e = input e of each lane, output
        // row 4 q + i = feed 16 (4 w + q) + 4 i + (e >> 1), pol e & 1, column
        // n = (s2, j)
        {
            uint32_t yr[4][2], yi[4][2];
            time_y_class(wk.s0, raw, yr, yi);
            const half8 Gh[2] = {s_G[0][lane], s_G[1][lane]}, Gl[2] = {s_G[2][lane], s_G[3][lane]};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                floatx4 Xr, Xi;
                ew_tile(yr, yi, e, Gh, Gl, Xr, Xi);
                float2* line = s_union + (16 * (e & 1) + n) * kEwLine;
#pragma unroll
                for (int i = 0; i < 4; ++i) line[ew_pos(4 * i + (e >> 1), 4 * w + q)] = make_float2(Xr[i], Xi[i]);
            }
        }
        __syncthreads();
        // B1: this group's two lines, feeds 16 a + b
        float2 v0[16], v1[16];
        {
            const float2* L0 = s_union + (16 * pol + 4 * s2 + jl[0]) * kEwLine;
            const float2* L1 = s_union + (16 * pol + 4 * s2 + jl[1]) * kEwLine;
#pragma unroll
            for (int aa = 0; aa < 16; aa += 2) {
                const float4 x0 = *reinterpret_cast<const float4*>(L0 + ew_pos(b, aa));
                const float4 x1 = *reinterpret_cast<const float4*>(L1 + ew_pos(b, aa));
                v0[aa] = make_float2(x0.x, x0.y);
                v0[aa + 1] = make_float2(x0.z, x0.w);
                v1[aa] = make_float2(x1.x, x1.y);
                v1[aa + 1] = make_float2(x1.z, x1.w);
            }
        }
        __syncthreads();
        // B2: N-S transform of both lines, power into per-bin accumulators; the
        // next block's samples are fetched during the second line (issued
        // there, the 32 registers they take are free for the first line).  The
        // last block fetches itself again rather than branch: one basic block
        // schedules with fewer live registers.
        const int k = wk.s0 + 4 * s2;
        ns_line_power<kFine>(v0, acc[0], bufE, bufO, s_tw, b, lv,
                             kFine ? fine_line_ptr(a, wk.unit, blk, k, pol * 4 + jl[0]) : nullptr);
        load_block_at(block_base(src, min(blk + 1, a.n_blk - 1)), raw, in_off);
        ns_line_power<kFine>(v1, acc[1], bufE, bufO, s_tw, b, lv,
                             kFine ? fine_line_ptr(a, wk.unit, blk, k, pol * 4 + jl[1]) : nullptr);
        __syncthreads();
    }
    if constexpr (kFine) return;  // complex beams only

    if (!io.last) {  // frame continues in the next chunk's launch
        store_partial<kAcc>(&acc[0][0][0], io.partial, t);
        return;
    }
    // per-bin powers -> LDS (pol 0 writes, pol 1 adds), then gather by the bin
    // table into out[beam][q]
    float* P = reinterpret_cast<float*>(s_union);
#pragma unroll
    for (int ph = 0; ph < 2; ++ph) {
        if (pol == ph) {
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                float* row = P + (s2 * 4 + jl[l]) * 512 + 2 * b;
#pragma unroll
                for (int d = 0; d < 16; ++d) {
                    if (ph == 0) {
                        row[32 * d] = acc[l][0][d];
                        row[32 * d + 1] = acc[l][1][d];
                    } else {
                        row[32 * d] += acc[l][0][d];
                        row[32 * d + 1] += acc[l][1][d];
                    }
                }
            }
        }
        __syncthreads();
    }
    write_output(P, a, io, wk.s0, t);
}

// The paper's 128-point up-channelisation in one pass (layout of the fine
// slices and the wave -> sub-channel map: time_dft128 and Work128).  512
// threads = 32 groups (wave w = g >> 2, jp, pol); per 128-sample block and per
// bin k of the workgroup's parity: all threads form the 8 fine slices of bin k
// (128 KB in LDS), wave w's groups take the slice whose fine channel lands in
// its sub-channel through E-W phasing and the N-S transform into |X|^2 per bin.
constexpr int kUnion128F2 = 32 * kGroupF2;       // 32 groups' transposes (17,920 float2)
static_assert(kUnion128F2 * 8 >= 8 * kSlice128 * 16, "union region must hold the 8 fine slices");
static_assert(kUnion128F2 * 8 >= 8 * 4 * 512 * 4, "union region must hold the per-bin powers");

template <bool kSym>
__global__ __launch_bounds__(kThreads128) __attribute__((amdgpu_waves_per_eu(2, 2)))
void bf_fp32_up128_kernel(LaunchArgs a)
{
    __shared__ __align__(16) float2 s_union[kUnion128F2];
    __shared__ __align__(16) float4 s_tw[16 * 16];  // [c'][b]: w512^(b 2c'), w512^(b (2c'+1))
    __shared__ __align__(16) float2 s_w128[128];    // w128^m

    const Work128 wk = work128_of_block();
    if (wk.unit >= a.n_units) return;  // uniform across the workgroup
    const int t = threadIdx.x;
    const int g = t >> 4;
    const int b = t & 15;
    const int w = g >> 2, jp = (g >> 1) & 1, pol = g & 1;
    const int jl[2] = {jp, 3 - jp};
    const int qw = q128_of_wave(wk.par, w);
    const int row = wk.unit % a.n_chan;

    if (t < 256) {
        const int c2 = t >> 4, bb = t & 15;
        const float2 w0 = a.tw[(2 * c2) * 16 + bb], w1 = a.tw[(2 * c2 + 1) * 16 + bb];
        s_tw[t] = make_float4(w0.x, w0.y, w1.x, w1.y);
    }
    float2 W[2][4];
#pragma unroll
    for (int l = 0; l < 2; ++l)
#pragma unroll
        for (int c = 0; c < 4; ++c) W[l][c] = a.ew[((size_t)row * kBeamEW + jl[l]) * kCyl + c];

    const __amdgpu_buffer_rsrc_t src = unit_rsrc(a.in + (size_t)wk.unit * a.n_time * kInputs,
                                                 a.n_time * kInputs);
    const float2* Tp = reinterpret_cast<const float2*>(s_union) + pol;
    float2* bufE = s_union + g * kGroupF2;
    float2* bufO = bufE + kXpBuf;
    const int32_t lv[1] = {0};

    float acc[2][2][16];
#pragma unroll
    for (int l = 0; l < 2; ++l)
#pragma unroll
        for (int d = 0; d < 16; ++d) acc[l][0][d] = acc[l][1][d] = 0.f;

    const int n_blk128 = a.n_time / 128;
    if (t < 128) s_w128[t] = a.tw128[t];
    __syncthreads();
    for (int blk = 0; blk < n_blk128; ++blk) {
        for (int i = 0; i < 8; ++i) {
            const int k = k128_of(wk.par, i);
            time_dft128_bin(k, src, blk * 128 * kInputs, s_w128,
                            reinterpret_cast<float*>(s_union), t);
            __syncthreads();
            float2 v0[16], v1[16];
            ew_group<kSym>(Tp + 2 * r128_for(k, qw) * kSlice128, W, v0, v1, b);
            __syncthreads();
            ns_line_power<false>(v0, acc[0], bufE, bufO, s_tw, b, lv, nullptr);
            ns_line_power<false>(v1, acc[1], bufE, bufO, s_tw, b, lv, nullptr);
            __syncthreads();
        }
    }
    // per-bin powers -> LDS (pol 0 writes, pol 1 adds), gathered by the bin table
    float* P = reinterpret_cast<float*>(s_union);
#pragma unroll
    for (int ph = 0; ph < 2; ++ph) {
        if (pol == ph) {
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                float* rowp = P + (w * 4 + jl[l]) * 512 + 2 * b;
#pragma unroll
                for (int d = 0; d < 16; ++d) {
                    if (ph == 0) {
                        rowp[32 * d] = acc[l][0][d];
                        rowp[32 * d + 1] = acc[l][1][d];
                    } else {
                        rowp[32 * d] += acc[l][0][d];
                        rowp[32 * d + 1] += acc[l][1][d];
                    }
                }
            }
        }
        __syncthreads();
    }
    write_beams128(P, a.lut + (size_t)row * kBeamNS, a.out + (size_t)wk.unit * kOutPerUnit,
                   wk.par, t);
}

}  // namespace

hipError_t launch_fp32_up128(const LaunchArgs& a, hipStream_t stream)
{
    if (a.n_units <= 0) return hipSuccess;
    LaunchArgs args = a;
    void* params[] = {&args};
    const void* k = a.sym_ew ? reinterpret_cast<const void*>(&bf_fp32_up128_kernel<true>)
                             : reinterpret_cast<const void*>(&bf_fp32_up128_kernel<false>);
    return hipLaunchKernel(k, dev::grid128_for(a.n_units), dim3(dev::kThreads128), params, 0, stream);
}

hipError_t launch_fp32(const LaunchArgs& a, hipStream_t stream)
{
    if (a.n_units <= 0) return hipSuccess;
    LaunchArgs args = a;
    void* params[] = {&args};
    // every E-W geometry takes the same matrix-core form
    const void* k = a.fine ? reinterpret_cast<const void*>(&bf_fp32_kernel<true>)
                           : reinterpret_cast<const void*>(&bf_fp32_kernel<false>);
    return hipLaunchKernel(k, dev::grid_for(a.n_units), dim3(dev::kThreads), params, 0, stream);
}

}  // namespace bf
