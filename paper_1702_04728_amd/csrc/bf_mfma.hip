// FP16-MFMA path of the hybrid beamformer: the N-S transform as a four-step
// 512 = 32 x 16 DFT on gfx950 matrix cores (v_mfma_f32_16x16x32_f16, FP32
// accumulation).
//
// Same outer structure as the FP32 kernel (paper Sec. 3, Sec. 3.1, Sec. 3.2):
// one workgroup per (channel-frame, sub-channel class s0); per 16-sample
// block the time DFT runs first on the raw samples (bins s0 + 4 s2), then
// E-W phasing, then the zero-padded N-S transform, then |.|^2 integrated per
// FFT bin and gathered through the Eq. (1) table at the end of the frame.
//
// The N-S transform of a 256-feed line x[16 a + b] (a, b < 16) into bins
// k = c + 32 d (c < 32, d < 16), upper half of the 512-point input zero:
//   stage 1  Z[c][b]  = sum_a w32^(a c) x[16 a + b]         (MFMA)
//   twiddle  Z'[c][b] = Z[c][b] w512^(b c)                   (FP32 VALU)
//   stage 2  X[c + 32 d] = sum_b w16^(b d) Z'[c][b]          (MFMA)
// Complex products are real 2x2 blocks.  Stage 1 takes the line as the A
// operand (rows b, K = (a, re/im)) against the fixed B = DFT-32 block
// (columns (c, re/im)); its accumulator layout (lane (q, n) holds rows
// b = 4q..4q+3 of column c = n [+16]) is exactly the B-operand layout stage 2
// needs with K = (b, re/im) and columns c, so no data moves between lanes.
// Wave s2 of the workgroup owns the 8 lines (4 E-W beams x 2 pols) of
// sub-channel s0 + 4 s2; lane (q, n) forms, during E-W phasing, the A
// fragment of feeds 16 a + n, a = 4q..4q+3, of all 8 lines.
//
// Precision (FP16 operands, FP32 accumulation; max relative power error
// about 5e-4 against FP64 on noise-plus-source and RFI-like inputs): the E-W
// output is rounded once to FP16; both DFT matrices are carried as a hi + lo
// pair of FP16 values (two MFMAs); the twiddled stage-1 output is split into
// hi + lo as well, and stage 2 sums hi*hi + lo*hi + hi*lo.  Rounding the
// matrices or the stage-1 output only once leaks each strong coherent source
// into the other beams of its sub-channel at the 2e-3 level.
#include <hip/hip_runtime.h>

#include "bf_device.h"

namespace bf {
namespace {

using namespace dev;

// Four complex values -> A/B fragment (re, im interleaved), round to nearest.
__device__ __forceinline__ half8 pack_half8(const float2 (&v)[4])
{
    half8 h;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h[2 * i] = (_Float16)v[i].x;
        h[2 * i + 1] = (_Float16)v[i].y;
    }
    return h;
}

// hi = fp16(v), lo = fp16(v - hi): together they carry ~22 significant bits.
// hi is the compiler's own packed round-to-nearest conversion.  The empty asm
// makes each value opaque first, so that the compiler cannot fold the
// conversion into the FMA that produced the value (a mixed-precision FMA with
// an FP16 result, which would also keep that FMA in FP32 for the lo half: two
// instructions per value instead of one per pair, 6-10 % of the kernel's
// time); it emits no instruction.  lo is one mixed-precision FMA per value,
// x - hi, which is exact in FP32 (the compiler does not form it itself, so it
// is written out).  Both halves feed matrix-core instructions, and the
// hardware needs two wait states between a VALU write of a register and an
// MFMA read of it; the compiler inserts them only after instructions it can
// see, so the block of lo instructions ends with its own s_nop.
__device__ __forceinline__ void split_half8(const float2 (&v)[4], half8& hi, half8& lo)
{
    float x[8];
    uint32_t h[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x[2 * i] = v[i].x;
        x[2 * i + 1] = v[i].y;
        asm volatile("" : "+v"(x[2 * i]), "+v"(x[2 * i + 1]));
        half2v hp;
        hp[0] = (_Float16)x[2 * i];
        hp[1] = (_Float16)x[2 * i + 1];
        h[i] = __builtin_bit_cast(uint32_t, hp);
    }
    uint32_t l[4];
    asm("v_fma_mixlo_f16 %0, %4, -1.0, %8 op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixhi_f16 %0, %4, -1.0, %9 op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixlo_f16 %1, %5, -1.0, %10 op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixhi_f16 %1, %5, -1.0, %11 op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixlo_f16 %2, %6, -1.0, %12 op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixhi_f16 %2, %6, -1.0, %13 op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixlo_f16 %3, %7, -1.0, %14 op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixhi_f16 %3, %7, -1.0, %15 op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"
        "s_nop 1"
        : "=&v"(l[0]), "=&v"(l[1]), "=&v"(l[2]), "=&v"(l[3])
        : "v"(h[0]), "v"(h[1]), "v"(h[2]), "v"(h[3]),
          "v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(x[3]), "v"(x[4]), "v"(x[5]), "v"(x[6]), "v"(x[7]));
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 hv = {h[0], h[1], h[2], h[3]}, lv = {l[0], l[1], l[2], l[3]};
    hi = __builtin_bit_cast(half8, hv);
    lo = __builtin_bit_cast(half8, lv);
}

// E-W phasing of one (sub-channel, feed, pol) across the four cylinders:
// b_j = sum_c W[j][c] y_c, written to v[j][ia] for j = 0..3.  Forms (kEw):
//   kEwMirror: cylinders and E-W directions both symmetric about the centre,
//     W[j][3-c] = W[3-j][c] = conj(W[j][c]); with S_c = y_c + y_(3-c),
//     D_c = y_c - y_(3-c) (c = 0, 1): b_j = P_j + i Q_j, b_(3-j) = P_j - i Q_j,
//     P_j = sum Re W[j][c] S_c, Q_j = sum Im W[j][c] D_c (28 operations per
//     feed instead of 56);
//   kEwCyl: cylinders symmetric, directions arbitrary (tracking beams):
//     W[j][3-c] = conj(W[j][c]) still, so b_j = P_j + i Q_j for every j from
//     the shared S_c, D_c (48 operations);
//   kEwGeneral: the plain four-cylinder sums (56 operations).
constexpr int kEwGeneral = 0, kEwCyl = 1, kEwMirror = 2;
template <int kEw>
__device__ __forceinline__ void ew_phase(const float2 (&y)[4], const float2 (&W)[4][4],
                                         float2 (&v)[4][4], int ia)
{
    if constexpr (kEw != kEwGeneral) {
        const float2 S0 = cadd(y[0], y[3]), S1 = cadd(y[1], y[2]);
        const float2 D0 = csub(y[0], y[3]), D1 = csub(y[1], y[2]);
        constexpr int kJ = kEw == kEwMirror ? 2 : 4;
#pragma unroll
        for (int j = 0; j < kJ; ++j) {
            const float2 P = make_float2(fmaf(W[j][0].x, S0.x, W[j][1].x * S1.x),
                                         fmaf(W[j][0].x, S0.y, W[j][1].x * S1.y));
            const float2 Q = make_float2(fmaf(W[j][0].y, D0.x, W[j][1].y * D1.x),
                                         fmaf(W[j][0].y, D0.y, W[j][1].y * D1.y));
            v[j][ia] = make_float2(P.x - Q.y, P.y + Q.x);
            if constexpr (kEw == kEwMirror) v[3 - j][ia] = make_float2(P.x + Q.y, P.y - Q.x);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int c = 0; c < 4; ++c) acc = cmac(acc, y[c], W[j][c]);
            v[j][ia] = acc;
        }
    }
}

// Fixed operands of the four-step transform in this lane's fragment order
// (stage-1 B tiles, stage-2 A tiles, each as hi + lo; inter-stage twiddles).
struct NsTables {
    half8 F1h[4], F1l[4], FDh[2], FDl[2];
    float2 tw[8];
};
__device__ __forceinline__ void load_ns_tables(const void* mf, NsTables& m, int lane)
{
    const half8* f1 = reinterpret_cast<const half8*>(mf);
    const half8* fd = f1 + 8 * 64;
    const float2* twp = reinterpret_cast<const float2*>(fd + 4 * 64);
#pragma unroll
    for (int tau = 0; tau < 4; ++tau) {
        m.F1h[tau] = f1[(2 * tau) * 64 + lane];
        m.F1l[tau] = f1[(2 * tau + 1) * 64 + lane];
    }
#pragma unroll
    for (int mu = 0; mu < 2; ++mu) {
        m.FDh[mu] = fd[(2 * mu) * 64 + lane];
        m.FDl[mu] = fd[(2 * mu + 1) * 64 + lane];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) m.tw[e] = twp[lane * 8 + e];
}

// E-W phasing of one time-DFT slice Ts (float4 per slot = both pols) straight
// into stage-1 A fragments: lane (q, n) forms feeds 16 a + n, a = 4 q + ia, of
// the 8 lines (E-W beam j, pol p), rounded once to FP16 (A) or, with kSplitV,
// as hi + lo (A, Alo).
template <int kEw, bool kSplitV>
__device__ __forceinline__ void ew_fragments(const float4* __restrict__ Ts, const float2 (&W)[4][4],
                                             half8 (&A)[4][2], half8 (&Alo)[4][2], int q, int n)
{
    if constexpr (kEw == kEwMirror) {  // both pols per LDS read
        float2 v[2][4][4];  // [p][j][ia]
#pragma unroll
        for (int ia = 0; ia < 4; ++ia) {
            float2 y0[4], y1[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float4 x4 = Ts[c * 256 + 16 * (4 * q + ia) + n];
                y0[c] = make_float2(x4.x, x4.y);
                y1[c] = make_float2(x4.z, x4.w);
            }
            ew_phase<kEw>(y0, W, v[0], ia);
            ew_phase<kEw>(y1, W, v[1], ia);
        }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if constexpr (kSplitV) split_half8(v[p][j], A[j][p], Alo[j][p]);
                else A[j][p] = pack_half8(v[p][j]);
            }
    } else {  // one pol at a time keeps the live set within 2 waves/SIMD
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            float2 v[4][4];  // [j][ia]
#pragma unroll
            for (int ia = 0; ia < 4; ++ia) {
                float2 y[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float4 x4 = Ts[c * 256 + 16 * (4 * q + ia) + n];
                    y[c] = p ? make_float2(x4.z, x4.w) : make_float2(x4.x, x4.y);
                }
                ew_phase<kEw>(y, W, v, ia);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if constexpr (kSplitV) split_half8(v[j], A[j][p], Alo[j][p]);
                else A[j][p] = pack_half8(v[j]);
            }
        }
    }
}

// N-S transform of one line on the matrix cores, stage 1 and the twiddle:
// the twiddled stage-1 output as hi + lo B fragments of stage 2.
template <bool kSplitV>
__device__ __forceinline__ void ns_stage1(const half8& A, const half8& Alo, const NsTables& m,
                                          half8 (&Bh)[2], half8 (&Bl)[2])
{
    // stage 1: Z = x (rows b) x DFT-32 block, matrix as hi + lo
    floatx4 D1[4];
#pragma unroll
    for (int tau = 0; tau < 4; ++tau) {
        const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
        D1[tau] = mfma16(A, m.F1h[tau], zero);
        D1[tau] = mfma16(A, m.F1l[tau], D1[tau]);
        if constexpr (kSplitV) D1[tau] = mfma16(Alo, m.F1h[tau], D1[tau]);
    }
    // twiddle in FP32, split into hi + lo B fragments (K = (b, re/im), column c)
#pragma unroll
    for (int nu = 0; nu < 2; ++nu) {
        float2 z[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            z[i] = cmul(make_float2(D1[nu][i], D1[nu + 2][i]), m.tw[4 * nu + i]);
        split_half8(z, Bh[nu], Bl[nu]);
    }
}
// Stage 2 for columns c = n + 16 nu: X = DFT-16 block (rows (d, re/im)) x Z';
// X[mu][i] holds (mu = 0: re, 1: im) of bin n + 16 nu + 32 (4 q + i).
__device__ __forceinline__ void ns_stage2(const half8& Bh, const half8& Bl, const NsTables& m,
                                          floatx4 (&X)[2])
{
#pragma unroll
    for (int mu = 0; mu < 2; ++mu) {
        const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
        X[mu] = mfma16(m.FDh[mu], Bh, zero);
        X[mu] = mfma16(m.FDl[mu], Bh, X[mu]);
        X[mu] = mfma16(m.FDh[mu], Bl, X[mu]);
    }
}

// hi = fp16 pair (x, y), lo = fp16 pair (x - hi.x, y - hi.y) (see split_half8),
// for x, y straight from matrix-core accumulators.  The hi conversion reads
// them in code the compiler sees, so it waits for the matrix instruction's
// result there (no opaque copy first, unlike split_half8: an MFMA result
// cannot be folded into a conversion anyway); the lo asm comes after it.
__device__ __forceinline__ void split_pair(float x, float y, uint32_t& hi, uint32_t& lo)
{
    half2v hp;
    hp[0] = (_Float16)x;
    hp[1] = (_Float16)y;
    hi = __builtin_bit_cast(uint32_t, hp);
    asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixhi_f16 %0, %1, -1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
        : "=&v"(lo)
        : "v"(hi), "v"(x), "v"(y));
}

// E-W output in LDS, one line (E-W beam j, pol p, sub-channel s0 + 4 s2) per
// kLineStride dwords, line 16 p + 4 s2 + j; each dword one complex FP16
// value (re low); feed 16 a + b at dword 16 b + 4 ((a >> 2) ^ ((b >> 2) & 3))
// + (a & 3), so the stage-1 reads (four consecutive a per lane, 16 b per
// quarter-wave) and the E-W writes (4 a x 16 lines per instruction) each
// spread over all banks.
constexpr int kLineStride = 260;
constexpr int kELines = 32;

// kSplitV: also carry the E-W output as hi + lo (stage 1 sums hi*hi + lo*hi +
// hi*lo): every operand then holds ~22 significant bits and the result is
// FP32-class (max relative power error ~1e-6 against FP64).
// kFine: the pre-detection beams (each line's kept beams written out instead
// of its power summed).
//
// Per 16-sample block: each wave takes the 128 (feed, pol) pairs 128 w ..
// 128 w + 127 of all four cylinders (lane (c, r) reads cylinder c's bytes
// 128 w + 8 r .. + 7 of every sample row), forms their stride-4 sums (time_y)
// and, per input e of the lane, one matrix-core tile of 16 (feed, pol) rows x
// (all 4 sub-channels x 4 E-W beams) into LDS; then wave w takes sub-channel
// s0 + 4 w's 8 lines through the four-step N-S transform and |.|^2.
// (The FP32-class debug form needs more than half the LDS of a CU, so it runs
// one workgroup per CU.)
template <bool kSplitV, bool kFine>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kSplitV && kFine ? 1 : 2, 2)))
void bf_mfma_kernel(LaunchArgs a)
{
    __shared__ __align__(16) uint32_t s_E[(kSplitV ? 2 : 1) * kELines * kLineStride];
    __shared__ __align__(16) float2 s_bins[kFine ? 4 * 512 : 1];  // per wave: one line's bins
    static_assert(sizeof(s_E) >= 4 * 4 * 512 * sizeof(float), "E-W area must hold the per-bin powers");

    const Work wk = work_of_block();
    UnitIO io;
    if (!resolve_unit(a, wk, io)) return;
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6, q = lane >> 4, n = lane & 15;

    NsTables mt;
    load_ns_tables(a.mf, mt, lane);
    half8 Gh[2], Gl[2];
    load_ew_mats(a.ew + (size_t)io.ew_row * kBeamEW * kCyl, wk.s0, lane, Gh, Gl);

    int32_t lv[kFine ? 4 : 1] = {};  // bin-table entries of the beams this lane writes
    if constexpr (kFine) load_lut_lane<4>(a.lut + (size_t)io.row * kBeamNS, lv, lane);

    const uint8_t* src = io.in;
    const int in_off = 512 * q + 128 * w + 8 * n;  // cylinder q, (feed, pol) 128 w + 8 n + e
    uint2 raw[16];
    load_block_at(block_base(src, 0), raw, in_off);

    float acc[4][2][4];  // [E-W beam j][c = n + 16 nu][d = 4 q + i]
    constexpr int kAcc = sizeof(acc) / sizeof(float);
    if (io.first) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int nu = 0; nu < 2; ++nu)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[j][nu][i] = 0.f;
    } else {
        load_partial<kAcc>(&acc[0][0][0], io.partial, t);
    }

    uint32_t* const E = s_E;
    [[maybe_unused]] uint32_t* const Elo = s_E + kELines * kLineStride;
    for (int blk = 0; blk < a.n_blk; ++blk) {
        uint32_t yr[4][2], yi[4][2];
        time_y_class(wk.s0, raw, yr, yi);
        if (blk + 1 < a.n_blk) load_block_at(block_base(src, blk + 1), raw, in_off);

        // time-DFT tail + E-W phasing: tile e = input e of each lane; output
        // row 4 q + i is feed 16 (4 w + q) + 4 i + (e >> 1), pol e & 1, of
        // column n = (s2, j)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            floatx4 Xr, Xi;
            ew_tile(yr, yi, e, Gh, Gl, Xr, Xi);
            const int line = (16 * (e & 1) + n) * kLineStride;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int pos = line + 16 * (4 * i + (e >> 1)) + 4 * (w ^ i) + q;
                if constexpr (kSplitV) {
                    uint32_t hi, lo;
                    split_pair(Xr[i], Xi[i], hi, lo);
                    E[pos] = hi;
                    Elo[pos] = lo;
                } else {
                    half2v hp;
                    hp[0] = (_Float16)Xr[i];
                    hp[1] = (_Float16)Xi[i];
                    E[pos] = __builtin_bit_cast(uint32_t, hp);
                }
            }
        }
        __syncthreads();

        // stage-1 A fragments of this wave's 8 lines: lane (q, n) holds feeds
        // 16 a + n, a = 4 q .. 4 q + 3
        half8 A[4][2];
        [[maybe_unused]] half8 Alo[4][2];
        const int rd = 16 * n + 4 * (q ^ (n >> 2));
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int pos = (16 * p + 4 * w + j) * kLineStride + rd;
                A[j][p] = __builtin_bit_cast(half8, *reinterpret_cast<const uint4*>(E + pos));
                if constexpr (kSplitV)
                    Alo[j][p] = __builtin_bit_cast(half8, *reinterpret_cast<const uint4*>(Elo + pos));
            }
        __syncthreads();

#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                half8 Bh[2], Bl[2];
                ns_stage1<kSplitV>(A[j][p], kSplitV ? Alo[j][p] : A[j][p], mt, Bh, Bl);
#pragma unroll
                for (int nu = 0; nu < 2; ++nu) {
                    floatx4 X[2];
                    ns_stage2(Bh[nu], Bl[nu], mt, X);
                    if constexpr (kFine) {  // bin n + 16 nu + 32 (4 q + i): (re, im) = (X[0], X[1])
                        float2* bins = s_bins + w * 512;
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            bins[n + 16 * nu + 32 * (4 * q + i)] = make_float2(X[0][i], X[1][i]);
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            acc[j][nu][i] = fmaf(X[0][i], X[0][i], fmaf(X[1][i], X[1][i], acc[j][nu][i]));
                    }
                }
                if constexpr (kFine) {
                    wave_lds_sync();
                    write_fine_line<4>(s_bins + w * 512, lv,
                                       fine_line_ptr(a, wk.unit, blk, wk.s0 + 4 * w, p * 4 + j), lane);
                    wave_lds_sync();
                }
            }
    }
    if constexpr (kFine) return;  // complex beams only

    if (!io.last) {  // frame continues in the next chunk's launch
        store_partial<kAcc>(&acc[0][0][0], io.partial, t);
        return;
    }
    // per-bin powers -> LDS (bin k = c + 32 d), then gather into out[beam][q]
    float* P = reinterpret_cast<float*>(s_E);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int nu = 0; nu < 2; ++nu)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                P[(w * 4 + j) * 512 + n + 16 * nu + 32 * (4 * q + i)] = acc[j][nu][i];
    __syncthreads();
    write_output(P, a, io, wk.s0, t);
}

// The paper's 128-point up-channelisation in one pass (fine slices and the
// wave -> sub-channel map: time_dft128 and Work128).  512 threads = 8 waves;
// per 128-sample block and per bin k of the workgroup's parity, all threads
// form the 8 fine slices of bin k (128 KB in LDS) and wave w takes the slice
// whose fine channel lands in its sub-channel through E-W phasing and the
// matrix-core N-S transform into |X|^2 per bin.
template <int kEw, bool kSplitV>
__global__ __launch_bounds__(kThreads128) __attribute__((amdgpu_waves_per_eu(2, 2)))
void bf_mfma_up128_kernel(LaunchArgs a)
{
    __shared__ __align__(16) float4 s_T[8 * kSlice128];  // 8 fine slices, then per-bin powers
    __shared__ __align__(16) float2 s_w128[128];         // w128^m
    // the N-S matrix-core tables, read back per bin: held in registers through
    // the time DFT they would push the kernel into spills
    __shared__ __align__(16) uint4 s_ns[kMfmaTableBytes / 16];

    const Work128 wk = work128_of_block();
    if (wk.unit >= a.n_units) return;  // uniform across the workgroup
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6, q = lane >> 4, n = lane & 15;
    const int qw = q128_of_wave(wk.par, w);
    const int row = wk.unit % a.n_chan;

    for (int i = t; i < (int)(kMfmaTableBytes / 16); i += kThreads128)
        s_ns[i] = reinterpret_cast<const uint4*>(a.mf)[i];
    float2 W[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c) W[j][c] = a.ew[((size_t)row * kBeamEW + j) * kCyl + c];

    const __amdgpu_buffer_rsrc_t src = unit_rsrc(a.in + (size_t)wk.unit * a.n_time * kInputs,
                                                 a.n_time * kInputs);
    float acc[4][2][4];  // [E-W beam j][c = n + 16 nu][d = 4 q + i]
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int nu = 0; nu < 2; ++nu)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[j][nu][i] = 0.f;

    const int n_blk128 = a.n_time / 128;
    if (t < 128) s_w128[t] = a.tw128[t];
    __syncthreads();
    for (int blk = 0; blk < n_blk128; ++blk) {
        // bins in pairs of one class (i and i + 4: k and k + 4, or k and
        // k + 12), which share the block's stride sums
        Y128 y;
        for (int i0 = 0; i0 < 8; ++i0) {
            const int i = (i0 >> 1) + 4 * (i0 & 1);
            const int k = k128_of(wk.par, i);
            if ((i0 & 1) == 0) stride_sums128_class(k & 3, src, blk * 128 * kInputs, y, t);
            slices128(k, y, s_w128, reinterpret_cast<float*>(s_T), t);
            __syncthreads();
            half8 A[4][2];
            [[maybe_unused]] half8 Alo[4][2];
            ew_fragments<kEw, kSplitV>(s_T + r128_for(k, qw) * kSlice128, W, A, Alo, q, n);
            __syncthreads();
            NsTables mt;
            load_ns_tables(s_ns, mt, lane);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    half8 Bh[2], Bl[2];
                    ns_stage1<kSplitV>(A[j][p], kSplitV ? Alo[j][p] : A[j][p], mt, Bh, Bl);
#pragma unroll
                    for (int nu = 0; nu < 2; ++nu) {
                        floatx4 X[2];
                        ns_stage2(Bh[nu], Bl[nu], mt, X);
#pragma unroll
                        for (int ii = 0; ii < 4; ++ii)
                            acc[j][nu][ii] = fmaf(X[0][ii], X[0][ii], fmaf(X[1][ii], X[1][ii], acc[j][nu][ii]));
                    }
                }
        }
    }
    // per-bin powers -> LDS (bin c + 32 d of wave w, E-W beam j), then gather
    float* P = reinterpret_cast<float*>(s_T);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int nu = 0; nu < 2; ++nu)
#pragma unroll
            for (int ii = 0; ii < 4; ++ii)
                P[(w * 4 + j) * 512 + n + 16 * nu + 32 * (4 * q + ii)] = acc[j][nu][ii];
    __syncthreads();
    write_beams128(P, a.lut + (size_t)row * kBeamNS, a.out + (size_t)wk.unit * kOutPerUnit,
                   wk.par, t);
}

}  // namespace

hipError_t launch_mfma_up128(const LaunchArgs& a, hipStream_t stream)
{
    if (a.n_units <= 0) return hipSuccess;
    LaunchArgs args = a;
    void* params[] = {&args};
    // [E-W form][split]
    static const void* const kKernels[3][2] = {
        {reinterpret_cast<const void*>(&bf_mfma_up128_kernel<kEwGeneral, false>),
         reinterpret_cast<const void*>(&bf_mfma_up128_kernel<kEwGeneral, true>)},
        {reinterpret_cast<const void*>(&bf_mfma_up128_kernel<kEwCyl, false>),
         reinterpret_cast<const void*>(&bf_mfma_up128_kernel<kEwCyl, true>)},
        {reinterpret_cast<const void*>(&bf_mfma_up128_kernel<kEwMirror, false>),
         reinterpret_cast<const void*>(&bf_mfma_up128_kernel<kEwMirror, true>)}};
    const int ew = a.sym_ew ? kEwMirror : a.cyl_sym ? kEwCyl : kEwGeneral;
    return hipLaunchKernel(kKernels[ew][a.split_v ? 1 : 0], dev::grid128_for(a.n_units),
                           dim3(dev::kThreads128), params, 0, stream);
}

hipError_t launch_mfma(const LaunchArgs& a, hipStream_t stream)
{
    if (a.n_units <= 0) return hipSuccess;
    LaunchArgs args = a;
    void* params[] = {&args};
    // [split][fine]; every E-W geometry takes the same matrix-core form
    static const void* const kKernels[2][2] = {
        {reinterpret_cast<const void*>(&bf_mfma_kernel<false, false>),
         reinterpret_cast<const void*>(&bf_mfma_kernel<false, true>)},
        {reinterpret_cast<const void*>(&bf_mfma_kernel<true, false>),
         reinterpret_cast<const void*>(&bf_mfma_kernel<true, true>)}};
    const void* k = kKernels[a.split_v ? 1 : 0][a.fine ? 1 : 0];
    return hipLaunchKernel(k, dev::grid_for(a.n_units), dim3(dev::kThreads), params, 0, stream);
}

}  // namespace bf
