// Device code shared by the beamformer kernels: complex helpers, the
// sub-channel-class time DFT that opens every kernel, and the end-of-frame
// gather of per-bin powers into clamped beams.
#pragma once

#include <hip/hip_runtime.h>

#include "bf_internal.h"

namespace bf {
namespace dev {

constexpr int kThreads = 256;

// cos / sin of 2 pi k / 32 for the first octant.
constexpr float kC16_1 = 0.92387953251128675613f;  // cos(pi/8)
constexpr float kS16_1 = 0.38268343236508977173f;  // sin(pi/8)
constexpr float kR2 = 0.70710678118654752440f;     // cos(pi/4)
constexpr float kC32_1 = 0.98078528040323044913f;  // cos(pi/16)
constexpr float kS32_1 = 0.19509032201612826785f;  // sin(pi/16)
constexpr float kC32_3 = 0.83146961230254523708f;  // cos(3pi/16)
constexpr float kS32_3 = 0.55557023301960222474f;  // sin(3pi/16)

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 w)
{
    return make_float2(fmaf(a.x, w.x, -a.y * w.y), fmaf(a.x, w.y, a.y * w.x));
}
// acc + a * w, complex
__device__ __forceinline__ float2 cmac(float2 acc, float2 a, float2 w)
{
    return make_float2(fmaf(a.x, w.x, fmaf(-a.y, w.y, acc.x)), fmaf(a.x, w.y, fmaf(a.y, w.x, acc.y)));
}

// Multiply by (-i)^K.
template <int K>
__device__ __forceinline__ float2 rot(float2 a)
{
    constexpr int k = ((K % 4) + 4) % 4;
    if constexpr (k == 0) return a;
    else if constexpr (k == 1) return make_float2(a.y, -a.x);
    else if constexpr (k == 2) return make_float2(-a.x, -a.y);
    else return make_float2(-a.y, a.x);
}

template <int K>
__device__ __forceinline__ float2 cs32()
{
    static_assert(K >= 0 && K <= 8, "first octant only");
    if constexpr (K == 0) return make_float2(1.f, 0.f);
    else if constexpr (K == 1) return make_float2(kC32_1, kS32_1);
    else if constexpr (K == 2) return make_float2(kC16_1, kS16_1);
    else if constexpr (K == 3) return make_float2(kC32_3, kS32_3);
    else if constexpr (K == 4) return make_float2(kR2, kR2);
    else if constexpr (K == 5) return make_float2(kS32_3, kC32_3);
    else if constexpr (K == 6) return make_float2(kS16_1, kC16_1);
    else if constexpr (K == 7) return make_float2(kS32_1, kC32_1);
    else return make_float2(0.f, 1.f);
}

// Multiply by w32^K = e^{-2 pi i K / 32}.
template <int K>
__device__ __forceinline__ float2 tw32(float2 a)
{
    constexpr int k = ((K % 32) + 32) % 32;
    if constexpr (k % 8 == 0) return rot<k / 8>(a);
    else if constexpr (k < 8) {
        const float2 cs = cs32<k>();
        return cmul(a, make_float2(cs.x, -cs.y));
    } else {
        return rot<k / 8>(tw32<k % 8>(a));  // w32^k = (-i)^(k/8) w32^(k%8)
    }
}

template <int K>
__device__ __forceinline__ float2 tw16(float2 a) { return tw32<2 * K>(a); }

// In-place DFT-4: X_k = sum_n x_n (-i)^(n k).
__device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d)
{
    const float2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = csub(b, d);
    a = cadd(t0, t2);
    c = csub(t0, t2);
    b = cadd(t1, rot<1>(t3));
    d = csub(t1, rot<1>(t3));
}

// Orders LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup -> (channel-frame, sub-channel class s0).  Workgroups are
// dispatched round-robin over the 8 XCDs; the four s0 workgroups of one
// channel-frame differ only in bits 3-4 of the id, so they run on the same XCD
// and read each raw block from HBM once, then from that XCD's L2.
struct Work {
    int unit, s0;
};
__device__ __forceinline__ Work work_of_block()
{
    const int x = blockIdx.x;
    Work w;
    w.s0 = (x >> 3) & 3;
    w.unit = ((x >> 5) << 3) | (x & 7);
    return w;
}
inline dim3 grid_for(int n_units) { return dim3(((n_units + 7) / 8) * 32); }

// Where one workgroup's channel-frame (or chunk of it) lives; see LaunchArgs.
struct UnitIO {
    const uint8_t* in;
    float* out;
    float* partial;  // this workgroup's partial sums (stream mode), else nullptr
    int row;         // row of the bin table (and of the static E-W weights)
    int ew_row;      // row of the E-W weights
    uint8_t* out_u8; // 8-bit output of this unit, or nullptr (FP32 output)
    bool first, last;
};
// False when the workgroup has no unit (uniform across the workgroup).
__device__ __forceinline__ bool resolve_unit(const LaunchArgs& a, const Work& wk, UnitIO& io)
{
    if (a.st == nullptr) {
        if (wk.unit >= a.n_units) return false;
        io.in = a.in + (size_t)wk.unit * a.n_blk * (kUp * kInputs);
        io.out = a.out + (size_t)wk.unit * kOutPerUnit;
        io.partial = nullptr;
        io.row = wk.unit % a.n_chan;
        io.ew_row = a.ew_by_unit ? wk.unit : io.row;
        io.out_u8 = a.out_u8 ? a.out_u8 + (size_t)wk.unit * kOutPerUnit : nullptr;
        io.first = io.last = true;
        return true;
    }
    if (wk.unit >= a.st->n_active) return false;
    const int32_t sv = a.st->slot[wk.unit];
    const int slot = sv & kSlotMask;
    const bool missing = (sv & kSlotMissing) != 0;
    const size_t entry = (size_t)a.st->ring_index * a.max_slots + slot;
    const int chunk = a.st->chunk_index;
    io.in = a.in + (entry * a.n_time + (size_t)chunk * a.n_blk * kUp) * kInputs;
    io.out = a.out + entry * kOutPerUnit;
    io.partial = a.partial + ((size_t)slot * 4 + wk.s0) * kPartialPerWg;
    io.row = slot;
    io.ew_row = slot;
    io.out_u8 = nullptr;
    io.first = chunk == 0;
    io.last = chunk == a.st->n_chunks - 1;
    // a missing frame has no input to read; bf_stream_flags_kernel zeroes its
    // output entry and writes every active entry's valid flag
    return !missing;
}

// Partial per-bin sums of a workgroup, element e of thread t at e * 256 + t.
template <int N>
__device__ __forceinline__ void load_partial(float* acc, const float* __restrict__ p, int t)
{
    static_assert(N <= kAccPerThreadMax, "partial-sum slot too small");
#pragma unroll
    for (int e = 0; e < N; ++e) acc[e] = p[e * kThreads + t];
}
template <int N>
__device__ __forceinline__ void store_partial(const float* acc, float* __restrict__ p, int t)
{
    static_assert(N <= kAccPerThreadMax, "partial-sum slot too small");
#pragma unroll
    for (int e = 0; e < N; ++e) p[e * kThreads + t] = acc[e];
}

// a + b + c in one instruction.  Written in C++, a + b + bias with a bias
// whose bits the nibbles cannot reach becomes an OR and two adds.
__device__ __forceinline__ uint32_t add3_u32(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// One word of class-S0 stride-4 sums: v[t2] holds 4 inputs' bytes (4+4-bit,
// offset binary) of sample t1 + 4 t2 for a fixed t1;
//   y = sum_t2 x[t1 + 4 t2] (-i)^(t2 S0)        (4-point DFT over the stride)
// as bytewise integer sums biased so that no byte borrows: byte k of yr (yi)
// is Re (Im) y + 32 of input k, in every class.
template <int S0>
__device__ __forceinline__ void stride_sum(const uint32_t (&v)[4], uint32_t& yr, uint32_t& yi)
{
    // nibble planes: r, m hold the 4 offset-binary nibbles (value + 8) as bytes
    constexpr uint32_t kLo = 0x0f0f0f0fu;
    constexpr uint32_t kBias = 0x20202020u;  // +32 per byte keeps differences >= 0
    uint32_t r[4], m[4];
#pragma unroll
    for (int t2 = 0; t2 < 4; ++t2) {
        r[t2] = (v[t2] >> 4) & kLo;
        m[t2] = v[t2] & kLo;
    }
    // x_k = x[t1 + 4k]; y = sum_k x_k (-i)^(k S0), each byte = value + 32
    if constexpr (S0 == 0) {
        yr = r[0] + r[1] + r[2] + r[3];  // = sum(value) + 32
        yi = m[0] + m[1] + m[2] + m[3];
    } else if constexpr (S0 == 1) {  // x0 - i x1 - x2 + i x3
        yr = add3_u32(r[0], m[1], kBias) - (r[2] + m[3]);
        yi = add3_u32(m[0], r[3], kBias) - (r[1] + m[2]);
    } else if constexpr (S0 == 2) {  // x0 - x1 + x2 - x3
        yr = add3_u32(r[0], r[2], kBias) - (r[1] + r[3]);
        yi = add3_u32(m[0], m[2], kBias) - (m[1] + m[3]);
    } else {  // x0 + i x1 - x2 - i x3
        yr = add3_u32(r[0], m[3], kBias) - (m[1] + r[2]);
        yi = add3_u32(m[0], r[1], kBias) - (m[2] + r[3]);
    }
}

// Integer part of the class-S0 time DFT of this thread's 8 inputs (the 8
// consecutive bytes raw holds of each of the 16 sample rows): byte k of
// yr[t1][w] (yi[t1][w]) is Re (Im) y[t1] + 32 of input 4 w + k (stride_sum).
template <int S0>
__device__ __forceinline__ void time_y(const uint2 (&raw)[16], uint32_t (&yr)[4][2], uint32_t (&yi)[4][2])
{
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
        for (int t1 = 0; t1 < 4; ++t1) {
            uint32_t v[4];
#pragma unroll
            for (int t2 = 0; t2 < 4; ++t2) v[t2] = w ? raw[t1 + 4 * t2].y : raw[t1 + 4 * t2].x;
            stride_sum<S0>(v, yr[t1][w], yi[t1][w]);
        }
}

__device__ __forceinline__ void time_y_class(int s0, const uint2 (&raw)[16], uint32_t (&yr)[4][2],
                                             uint32_t (&yi)[4][2])
{
    switch (s0) {
    case 0: time_y<0>(raw, yr, yi); break;
    case 1: time_y<1>(raw, yr, yi); break;
    case 2: time_y<2>(raw, yr, yi); break;
    default: time_y<3>(raw, yr, yi); break;
    }
}

// Raw samples of one block of 16: the 8 bytes at offset `off` (8-byte aligned)
// of each sample row.
__device__ __forceinline__ void load_block_at(const uint8_t* __restrict__ blk, uint2 (&raw)[16], int off)
{
#pragma unroll
    for (int tau = 0; tau < 16; ++tau)
        raw[tau] = *reinterpret_cast<const uint2*>(blk + tau * kInputs + off);
}

// Samples of 16-sample block `it`.
__device__ __forceinline__ const uint8_t* block_base(const uint8_t* in, int it)
{
    return in + (size_t)it * (kUp * kInputs);
}

// Complex beams out (the pre-detection beams): the 512 bins of one line
// (sub-channel k, line p * 4 + j, block it) sit in LDS at bins[]; the kept
// beam of every N-S pointing m is bins[lut[m]].  Lane `lane` of 256 / N lanes
// writes the beams m = lane + (256 / N) i, i < N, whose table entries it holds
// in registers (read once per kernel by load_lut_lane): a table read inside
// the line loop would wait, through the shared load/store counter, for every
// beam store issued before it.
template <int N>
__device__ __forceinline__ void load_lut_lane(const int32_t* __restrict__ lut, int32_t (&lv)[N], int lane)
{
#pragma unroll
    for (int i = 0; i < N; ++i) lv[i] = lut[lane + (kBeamNS / N) * i];
}
template <int N>
__device__ __forceinline__ void write_fine_line(const float2* __restrict__ bins, const int32_t (&lv)[N],
                                                float2* __restrict__ dst, int lane)
{
#pragma unroll
    for (int i = 0; i < N; ++i) dst[lane + (kBeamNS / N) * i] = bins[lv[i]];
}
// Line (p * 4 + j) of sub-channel k, block it of a unit in the complex-beam
// buffer.
__device__ __forceinline__ float2* fine_line_ptr(const LaunchArgs& a, int unit, int it, int k, int line)
{
    return a.fine + ((((size_t)unit * a.n_blk + it) * 16 + k) * 8 + line) * kBeamNS;
}

// ---------------------------------------------------------------------------
// Matrix-core building blocks (v_mfma_f32_16x16x32_f16, FP32 accumulation).
// Fragment layouts: lane l holds row (A) or column (B) l % 16 and K values
// 8 (l / 16) .. 8 (l / 16) + 7; the accumulator lane l holds column l % 16,
// rows 4 (l / 16) .. 4 (l / 16) + 3.
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma16(half8 a, half8 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// cos and sin of 2 pi k / 16.
static __constant__ float kCos16[16] = {1.f, kC16_1, kR2, kS16_1, 0.f, -kS16_1, -kR2, -kC16_1,
                                 -1.f, -kC16_1, -kR2, -kS16_1, 0.f, kS16_1, kR2, kC16_1};
static __constant__ float kSin16[16] = {0.f, kS16_1, kR2, kC16_1, 1.f, kC16_1, kR2, kS16_1,
                                 0.f, -kS16_1, -kR2, -kC16_1, -1.f, -kC16_1, -kR2, -kS16_1};

// The last step of the class-s0 time DFT and E-W phasing together are one
// complex 16 x 16 matrix per (channel, class), applied to each (feed, pol):
//   b[s2][j] = sum_c W[j][c] sum_t1 w16^(t1 (s0 + 4 s2)) y_c[t1]
// (y_c[t1] the stride-4 sums of cylinder c, time_y; s0 + 4 s2 the
// sub-channel, j the E-W beam).  As a real 32 x 32 block on the matrix cores:
// K = (cylinder c, t1, re/im) with lane (c, .) holding cylinder c's 8 values,
// columns (s2, j) = 4 s2 + j, N-tile 0 giving the real and N-tile 1 the
// imaginary part of b.  The y values are small integers, exact in FP16; the
// matrix is carried as hi + lo (two MFMAs per tile), so the E-W output keeps
// ~22 significant bits before the N-S transform.  Entries formed in FP32
// from the weight row W[j][c] (ew_row, [4][4]) at the start of the frame,
// each rounded to FP32 once and then split: left to itself the compiler
// folds some of the hi conversions into the products' fused multiply-adds
// (one rounding from the exact value) and not the lo subtractions, and where
// the FP32 value is an FP16 rounding tie the two hi values then differ by one
// FP16 ulp, which hi + lo keeps.
__device__ __forceinline__ void load_ew_mats(const float2* __restrict__ ew_row, int s0, int lane,
                                             half8 (&Gh)[2], half8 (&Gl)[2])
{
    const int c = lane >> 4, col = lane & 15;
    const int j = col & 3, s = s0 + 4 * (col >> 2);
    const float2 wjc = ew_row[j * kCyl + c];
#pragma unroll
    for (int t1 = 0; t1 < 4; ++t1) {
        const int k = (t1 * s) & 15;
        const float2 m = cmul(wjc, make_float2(kCos16[k], -kSin16[k]));  // W[j][c] w16^(t1 s)
        // real output: Re y m.x - Im y m.y; imaginary output: Re y m.y + Im y m.x
        const float v[2][2] = {{m.x, -m.y}, {m.y, m.x}};
#pragma unroll
        for (int nu = 0; nu < 2; ++nu)
#pragma unroll
            for (int ri = 0; ri < 2; ++ri) {
                float x = v[nu][ri];
                asm volatile("" : "+v"(x));
                const _Float16 hi = (_Float16)x;
                Gh[nu][2 * t1 + ri] = hi;
                Gl[nu][2 * t1 + ri] = (_Float16)(x - (float)hi);
            }
    }
}

// A fragment of input m of one word column (K = (t1, re/im)): y[t1] exactly,
// from the biased bytes of stride_sum.  One byte permute places Re and Im of
// one t1 in the low bytes of two halves, the exponent bits of 1024 make each
// half 1024 + byte, and one packed FP16 subtraction of 1024 + 32 leaves y.
__device__ __forceinline__ half8 y_fragment1(const uint32_t (&yr)[4], const uint32_t (&yi)[4], int m)
{
    const uint32_t sel = 0x0c000c00u | ((4u + m) << 16) | (uint32_t)m;  // (yr byte m, 0, yi byte m, 0)
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 d;
#pragma unroll
    for (int t1 = 0; t1 < 4; ++t1) d[t1] = __builtin_amdgcn_perm(yi[t1], yr[t1], sel) | 0x64006400u;
    const half8 bias = {1056.f16, 1056.f16, 1056.f16, 1056.f16, 1056.f16, 1056.f16, 1056.f16, 1056.f16};
    return __builtin_bit_cast(half8, d) - bias;
}
// The same for input 4 wd + m of time_y's two word columns.
__device__ __forceinline__ half8 y_fragment(const uint32_t (&yr)[4][2], const uint32_t (&yi)[4][2], int wd,
                                            int m)
{
    const uint32_t r[4] = {yr[0][wd], yr[1][wd], yr[2][wd], yr[3][wd]};
    const uint32_t i[4] = {yi[0][wd], yi[1][wd], yi[2][wd], yi[3][wd]};
    return y_fragment1(r, i, m);
}

// One tile of the fused time-DFT tail + E-W product: input e (0..7) of every
// lane (cylinder lane / 16, tile row lane % 16) against the (channel, class)
// matrix; Xr and Xi get the real and imaginary parts in accumulator layout
// (row 4 (lane / 16) + i, column (s2, j) = lane % 16).
__device__ __forceinline__ void ew_tile(const uint32_t (&yr)[4][2], const uint32_t (&yi)[4][2], int e,
                                        const half8 (&Gh)[2], const half8 (&Gl)[2], floatx4& Xr,
                                        floatx4& Xi)
{
    const half8 Ay = y_fragment(yr, yi, e >> 2, e & 3);
    const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
    Xr = mfma16(Ay, Gh[0], zero);
    Xr = mfma16(Ay, Gl[0], Xr);
    Xi = mfma16(Ay, Gh[1], zero);
    Xi = mfma16(Ay, Gl[1], Xi);
}

// ---------------------------------------------------------------------------
// The paper's own up-channelisation (Sec. 3, Sec. 3.2): a 128-point DFT of each
// 128-sample block, fine bin s' centre-shifted to q' = (s' + 64) mod 128 and
// its power summed into sub-channel q = ((q' + 4) div 8) mod 16 (the 8 fine
// channels nearest the sub-channel's centre).
//
// Still time first: the 128-point DFT runs on the raw samples, before E-W
// phasing and the N-S transform.  With s' = k + 16 r (k < 16, r < 8) and
// t = u + 8 tau (u < 8, tau < 16),
//   X[k + 16 r] = sum_u w8^(r u) w128^(u k) Y_u[k],  Y_u[k] = sum_tau x[u + 8 tau] w16^(k tau),
// so one bin k gives 8 fine "slices" r of all 2048 inputs (128 KB as FP32 in
// LDS), each of which then takes the same E-W and N-S transforms as a 16-point
// slice.  Fine bin k + 16 r lands in sub-channel q = (2 r + 8 + (k + 4) div 8)
// mod 16: its parity is fixed by k, so a workgroup of 8 waves takes the 8 bins
// k of one parity (par 1: k = 4..11, odd q; par 0: k = 0..3, 12..15, even q),
// and wave w always integrates the one sub-channel q_w = 2 w + 8 + par (mod 16)
// -- for every k exactly one of its 8 slices lands there.  No partial sums
// cross workgroups.
constexpr int kThreads128 = 512;

// Workgroup -> (channel-frame, parity).  The two workgroups of a channel-frame
// differ only in bit 3 of the id, so they run on the same XCD and share each
// raw block through its L2.
struct Work128 {
    int unit, par;
};
__device__ __forceinline__ Work128 work128_of_block()
{
    const int x = blockIdx.x;
    Work128 w;
    w.par = (x >> 3) & 1;
    w.unit = ((x >> 4) << 3) | (x & 7);
    return w;
}
inline dim3 grid128_for(int n_units) { return dim3(((n_units + 7) / 8) * 16); }

// Bin k of step i < 8 of a workgroup of parity par.
__device__ __forceinline__ int k128_of(int par, int i) { return par ? 4 + i : (i < 4 ? i : 8 + i); }
// Sub-channel of fine bin k + 16 r.
__device__ __forceinline__ int q128_of(int k, int r) { return ((((k + 16 * r + 64) & 127) + 4) >> 3) & 15; }
// The slice r of bin k whose fine channel lands in sub-channel q (q of the
// parity k serves).
__device__ __forceinline__ int r128_for(int k, int q)
{
    int r = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c)
        if (q128_of(k, c) == q) r = c;
    return r;
}
// Sub-channel integrated by wave w of a workgroup of parity par.
__device__ __forceinline__ int q128_of_wave(int par, int w) { return (2 * w + 8 + par) & 15; }

// The unit's samples are read through a buffer resource (base and size in
// SGPRs, bounds-checked by the hardware: reads past `bytes` return 0): one
// VGPR lane offset and scalar row offsets, where 64-bit per-row addresses
// would hold many VGPRs.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t unit_rsrc(const uint8_t* base, int bytes)
{
    // dword 3 of a raw (untyped) buffer descriptor on gfx9-family GPUs
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(base), 0, bytes, 0x00020000);
}
__device__ __forceinline__ uint2 load_pair(__amdgpu_buffer_rsrc_t r, int lane_off, int row_off)
{
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, row_off, 0);
    return make_uint2(v[0], v[1]);
}

// Float4 per fine slice in LDS: 1024 slots (slot = cyl * 256 + feed, float4 =
// both pols) and 1 of padding, so that the eight slices' writes of one
// instruction fall on different banks.
constexpr int kSlice128 = 1025;

// Bin k (class S0 = k mod 4) of the 128-point DFT of one 128-sample block for
// all 2048 inputs: the 8 fine slices r go to T[(r * kSlice128 + slot) * 4 +
// 2 pol + re/im].  With t = u + 8 t1 + 32 t2 within the block,
//   y_u[t1]    = sum_t2 x[t] (-i)^(S0 t2)      (exact integers, stride_sums128)
//   X[k + 16r] = sum_(u, t1) w128^(k (u + 8 t1)) w8^(r u) y_u[t1],
// the second a real 64 x 16 matrix per bin on the matrix cores (slices128; two
// K-steps of 32, kappa = u div 4; exact FP16 operands, FP32 results).  Each
// matrix entry is the single power w128^(k (u + 8 t1) + 16 r u) (w8 = w128^16),
// read from w128[] (FP32, LDS) and split into FP16 hi + lo in the lane that
// holds it (lane (g, n): K = (u = 4 kappa + g, t1, re/im), column n = slice
// r = n mod 8 of the real (n < 8) or imaginary output part): formed per bin in
// the kernel, so no table of per-bin matrices competes with the sample blocks
// for L2.  Wave w takes inputs 256 w .. 256 w + 255 as two sets of 128: lane
// (g, rr) reads the 8 bytes (inputs) at word column 64 w + 32 m + 2 rr of
// sample phases u = g and 4 + g (16 lanes: one whole 128-byte line of a row per
// load), forms their stride sums, and holds row rr of tile e (input
// 4 (64 w + 32 m + 2 rr) + e) for K-step kappa = u div 4.  A zero-valued input
// stays exactly zero.  Bins k and k + 4 (k and k + 12) share a class, hence
// their stride sums.

// The stride sums of one 128-sample block for this lane (two sets of 8 inputs,
// sample phases g and 4 + g, class S0): y[m][kappa] as time_y's words.
struct Y128 {
    uint32_t r[2][2][4][2], i[2][2][4][2];  // [set m][kappa][t1][word]
};
template <int S0>
__device__ __forceinline__ void stride_sums128(__amdgpu_buffer_rsrc_t src, int blk_off, Y128& y, int t)
{
    const int lane = t & 63, w = t >> 6, g = lane >> 4, rr = lane & 15;
    // this lane's sample phase g (+ 4 kappa) row and word columns, in bytes;
    // the rest of each row offset is uniform (scalar)
    const int lane_off = g * kInputs + 4 * (64 * w + 2 * rr);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int kap = 0; kap < 2; ++kap) {
            // one phase at a time: without the barrier the scheduler hoists
            // every phase's loads and runs out of registers
            __builtin_amdgcn_sched_barrier(0);
            uint2 raw[16];
#pragma unroll
            for (int tau = 0; tau < 16; ++tau)
                raw[tau] = load_pair(src, lane_off + 128 * m, blk_off + (4 * kap + 8 * tau) * kInputs);
            time_y<S0>(raw, y.r[m][kap], y.i[m][kap]);
        }
}
__device__ __forceinline__ void stride_sums128_class(int s0, __amdgpu_buffer_rsrc_t src, int blk_off,
                                                     Y128& y, int t)
{
    switch (s0) {
    case 0: stride_sums128<0>(src, blk_off, y, t); break;
    case 1: stride_sums128<1>(src, blk_off, y, t); break;
    case 2: stride_sums128<2>(src, blk_off, y, t); break;
    default: stride_sums128<3>(src, blk_off, y, t); break;
    }
}

// The 8 fine slices of bin k from the block's stride sums of class k mod 4
// (time_dft128): the bin's matrix in this lane's fragments, one tile per input
// e of each set, stores into T.
__device__ __forceinline__ void slices128(int k, const Y128& y, const float2* __restrict__ w128,
                                          float* __restrict__ T, int t)
{
    const int lane = t & 63, w = t >> 6, g = lane >> 4, rr = lane & 15;
    half8 Bh[2], Bl[2];
#pragma unroll
    for (int kap = 0; kap < 2; ++kap) {
        const int u = 4 * kap + g, r = rr & 7;
#pragma unroll
        for (int t1 = 0; t1 < 4; ++t1) {
            const float2 mv = w128[(k * (u + 8 * t1) + 16 * r * u) & 127];
            // real output: Re y Re M - Im y Im M; imaginary: Re y Im M + Im y Re M
            float x[2] = {rr < 8 ? mv.x : mv.y, rr < 8 ? -mv.y : mv.x};
#pragma unroll
            for (int ri = 0; ri < 2; ++ri) {
                // one FP32 value per entry, split once (see load_ew_mats)
                asm volatile("" : "+v"(x[ri]));
                const _Float16 hi = (_Float16)x[ri];
                Bh[kap][2 * t1 + ri] = hi;
                Bl[kap][2 * t1 + ri] = (_Float16)(x[ri] - (float)hi);
            }
        }
    }
    // output column of this lane: slice r = rr mod 8, real (nu = 0) or imaginary
    // part; its stores are this base plus compile-time offsets
    float* const Tl = T + (((rr & 7) * kSlice128 + 128 * w + 16 * g) * 4 + (rr >> 3));
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const half8 A0 = y_fragment(y.r[m][0], y.i[m][0], e >> 2, e & 3);
            const half8 A1 = y_fragment(y.r[m][1], y.i[m][1], e >> 2, e & 3);
            const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
            floatx4 X = mfma16(A0, Bh[0], zero);
            X = mfma16(A0, Bl[0], X);
            X = mfma16(A1, Bh[1], X);
            X = mfma16(A1, Bl[1], X);
            // row 4 g + i: input 4 (64 w + 32 m + 8 g + 2 i + (e >> 2)) + (e & 3),
            // i.e. slot 2 (64 w + 32 m + 8 g + 2 i + (e >> 2)) + ((e & 3) >> 1),
            // pol e & 1
#pragma unroll
            for (int i = 0; i < 4; ++i)
                Tl[(64 * m + 4 * i + 2 * (e >> 2) + ((e & 3) >> 1)) * 4 + 2 * (e & 1)] = X[i];
        }
}

// One bin, stride sums and slices together (the FP32 kernel, which has no
// registers to keep the sums across bins).
__device__ __forceinline__ void time_dft128_bin(int k, __amdgpu_buffer_rsrc_t src, int blk_off,
                                                const float2* w128, float* T, int t)
{
    Y128 y;
    stride_sums128_class(k & 3, src, blk_off, y, t);
    slices128(k, y, w128, T, t);
}

// End of frame, 128-point form: P[(w * 4 + j) * 512 + bin] holds wave w's
// integrated power of FFT bin `bin`, E-W beam j; beam (j, m) takes bin lut[m]
// into sub-channel q128_of_wave(par, w).
__device__ __forceinline__ void write_beams128(const float* __restrict__ P,
                                               const int32_t* __restrict__ lut,
                                               float* __restrict__ dst, int par, int t)
{
#pragma unroll 4
    for (int it = 0; it < 16; ++it) {
        const int u = it * kThreads128 + t;
        const int beam = u >> 3, w = u & 7;
        const int jj = beam >> 8, m = beam & 255;
        dst[beam * kUp + q128_of_wave(par, w)] = P[(w * 4 + jj) * 512 + lut[m]];
    }
}

// End of frame: P[(s2 * 4 + j) * 512 + k] holds the integrated power of FFT
// bin k for sub-channel s0 + 4 s2 and E-W beam j.  Beam (j, m) takes bin
// lut[m] (Eq. (1)); sub-channel q holds time-DFT bin (q + 8) mod 16.
__device__ __forceinline__ void write_beams(const float* __restrict__ P,
                                            const int32_t* __restrict__ lut,
                                            float* __restrict__ dst, int s0, int t)
{
#pragma unroll 4
    for (int it = 0; it < 16; ++it) {
        const int u = it * kThreads + t;
        const int beam = u >> 2, q2 = u & 3;
        const int jj = beam >> 8, m = beam & 255;
        const int ss2 = (q2 + 2) & 3;  // q = s0 + 4 q2 holds s = s0 + 4 ss2
        dst[beam * kUp + s0 + 4 * q2] = P[(ss2 * 4 + jj) * 512 + lut[m]];
    }
}

// 8-bit output of the same gather: code = clamp(rint(P scale + offset), 0, 255)
// in FP32 (one fused multiply-add, rint rounds half to even); scale and
// offset are this channel's [1024][16] rows.
__device__ __forceinline__ void write_beams_u8(const float* __restrict__ P,
                                               const int32_t* __restrict__ lut,
                                               const float* __restrict__ scale,
                                               const float* __restrict__ offset,
                                               uint8_t* __restrict__ dst, int s0, int t)
{
#pragma unroll 4
    for (int it = 0; it < 16; ++it) {
        const int u = it * kThreads + t;
        const int beam = u >> 2, q2 = u & 3;
        const int jj = beam >> 8, m = beam & 255;
        const int ss2 = (q2 + 2) & 3;
        const int o = beam * kUp + s0 + 4 * q2;
        const float x = rintf(fmaf(P[(ss2 * 4 + jj) * 512 + lut[m]], scale[o], offset[o]));
        dst[o] = (uint8_t)fminf(fmaxf(x, 0.f), 255.f);
    }
}

// End-of-frame output in the format the launch asks for.
__device__ __forceinline__ void write_output(const float* P, const LaunchArgs& a, const UnitIO& io,
                                             int s0, int t)
{
    const int32_t* lut = a.lut + (size_t)io.row * kBeamNS;
    if (io.out_u8)
        write_beams_u8(P, lut, a.scale + (size_t)io.row * kOutPerUnit,
                       a.offset + (size_t)io.row * kOutPerUnit, io.out_u8, s0, t);
    else
        write_beams(P, lut, io.out, s0, t);
}

}  // namespace dev
}  // namespace bf
