// Host side of libbeamform: argument validation, FP64 precompute of the
// per-channel tables, plan lifetime and the C ABI entry points.
//
// Tables (all computed in FP64, rounded once to FP32):
//   lut[chan][m]  Eq. (1)-(2) of the paper (Sec. 3.1): the FFT bin nearest
//                 desired pointing m, floor(N P f d sin(theta_m) / c + 0.5)
//                 reduced mod N P.  Eq. (2) is Eq. (1) at another frequency,
//                 so the formula is evaluated per channel.
//   ew[chan][j][c] E-W exact phasing (Sec. 3, Sec. 3.1):
//                 exp(-2 pi i f x_c sin(phi_j) / c).
//   tw[c][b]      Inter-stage twiddles of the 512-point N-S transform,
//                 exp(-2 pi i ((b c) mod 512) / 512), c < 32, b < 16.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "bf_plan.h"
#include "bf_trace.h"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
thread_local std::string g_init_error;

int32_t fail(bf_plan* p, int32_t status, const std::string& msg)
{
    if (p) p->err = msg;
    else g_init_error = msg;
    return status;
}

int32_t hip_fail(bf_plan* p, hipError_t e, const char* what)
{
    return fail(p, BF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Checks the sizes the kernels are specialised for.
int32_t check_config(const bf_config* c, std::string* msg)
{
    if (!c) { *msg = "cfg is NULL"; return BF_E_INVAL; }
    if (c->n_time <= 0 || c->n_time % bf::kUp != 0) {
        *msg = "n_time must be a positive multiple of 16";
        return BF_E_INVAL;
    }
    if (c->n_time > (1 << 20)) { *msg = "n_time too large"; return BF_E_INVAL; }
    if (c->n_cyl <= 0 || c->n_feed <= 0 || c->n_pol <= 0 || c->pad <= 0 ||
        c->n_beam_ns <= 0 || c->n_beam_ew <= 0 || c->n_upchan <= 0) {
        *msg = "sizes must be positive";
        return BF_E_INVAL;
    }
    if (!(c->feed_spacing_m > 0.0) || !(c->c0 > 0.0)) {
        *msg = "feed_spacing_m and c0 must be positive";
        return BF_E_INVAL;
    }
    if (c->reserved != 0) { *msg = "reserved must be 0"; return BF_E_INVAL; }
    if (c->precision != BF_FP32_FFT && c->precision != BF_FP16_MFMA &&
        c->precision != BF_FP32_MFMA) {
        *msg = "unknown precision";
        return BF_E_INVAL;
    }
    if (c->n_cyl != bf::kCyl || c->n_feed != bf::kFeed || c->n_pol != bf::kPol ||
        c->pad != bf::kPad || c->n_beam_ns != bf::kBeamNS || c->n_beam_ew != bf::kBeamEW ||
        c->n_upchan != bf::kUp) {
        *msg = "kernels are built for 4 cylinders x 256 feeds x 2 pols, P = 2, "
               "256 x 4 beams and a 16-point time DFT";
        return BF_E_UNSUPPORTED;
    }
    return BF_OK;
}

double default_cyl_x(int c) { return (c - 1.5) * 20.0; }
double default_sin_theta(int m) { return (m - 127.5) / 128.0; }
double default_sin_phi(int j) { return std::sin((j - 1.5) * 0.4 * kTwoPi / 360.0); }

// Eq. (1) of the paper evaluated in FP64, then floor and reduction mod N P;
// -1 when the argument is too large for an exact integer floor.
int32_t eq1_bin(const bf_config* c, double f_hz, double sin_theta)
{
    const int nb = c->n_feed * c->pad;
    const double t = (double)c->n_feed * (double)c->pad * f_hz * (c->feed_spacing_m / c->c0) *
                     sin_theta + 0.5;
    if (!(std::fabs(t) < 9.0e15)) return -1;  // beyond 2^53 floor is no longer exact
    long long k = (long long)std::floor(t);
    long long r = k % nb;
    if (r < 0) r += nb;
    return (int32_t)r;
}

int32_t fill_lut(const bf_config* c, const double* freqs, int32_t n_chan, int32_t* out,
                 std::string* msg)
{
    const int nb = c->n_feed * c->pad;
    for (int32_t ch = 0; ch < n_chan; ++ch) {
        const double f = freqs[ch];
        if (!std::isfinite(f) || !(f > 0.0)) { *msg = "channel frequency must be > 0"; return BF_E_INVAL; }
        for (int m = 0; m < c->n_beam_ns; ++m) {
            int32_t k;
            if (c->lut_override) {
                k = c->lut_override[(size_t)ch * c->n_beam_ns + m];
                if (k < 0 || k >= nb) { *msg = "lut_override entry out of [0, N P)"; return BF_E_INVAL; }
            } else {
                const double s = c->sin_theta_ns ? c->sin_theta_ns[m] : default_sin_theta(m);
                if (!std::isfinite(s)) { *msg = "sin_theta_ns must be finite"; return BF_E_INVAL; }
                k = eq1_bin(c, f, s);
                if (k < 0) { *msg = "Eq. (1) argument out of range (frequency x sin_theta too large)"; return BF_E_INVAL; }
            }
            out[(size_t)ch * c->n_beam_ns + m] = k;
        }
    }
    return BF_OK;
}

// E-W phases of one channel, W[j][c] = exp(-2 pi i f x_c sin(phi_j) / c0)
// (Sec. 3 first kernel, Sec. 3.1), in FP64 and rounded once to FP32.
void fill_ew(double f_hz, const double* cyl_x, const double* sin_phi, double c0, float2* w)
{
    for (int j = 0; j < bf::kBeamEW; ++j)
        for (int c = 0; c < bf::kCyl; ++c) {
            const double a = kTwoPi * f_hz * cyl_x[c] * sin_phi[j] / c0;
            w[j * bf::kCyl + c] = make_float2((float)std::cos(a), (float)-std::sin(a));
        }
}

// Mirror symmetry of the E-W geometry (the default layout has it): then
// W[j][3-c] = W[3-j][c] = conj(W[j][c]) exactly and the kernels use half the
// E-W multiply-adds.
bool mirror_symmetric(const double* cyl_x, const double* sin_phi)
{
    return cyl_x[3] == -cyl_x[0] && cyl_x[2] == -cyl_x[1] &&
           sin_phi[3] == -sin_phi[0] && sin_phi[2] == -sin_phi[1];
}
// Cylinder positions alone symmetric: W[j][3-c] = conj(W[j][c]) exactly for any
// direction (the phase is negated exactly in FP64), which the matrix-core
// kernels use for directions without mirror symmetry (tracking beams).
bool cylinders_symmetric(const double* cyl_x)
{
    return cyl_x[3] == -cyl_x[0] && cyl_x[2] == -cyl_x[1];
}

// Checks shared by the batch entry points, then one launch over all units.
int32_t launch_batch(bf_plan* p, const uint8_t* d_in, int32_t n_frames, float* d_out,
                     hipStream_t stream, const float2* ew, int32_t ew_by_unit, int32_t sym,
                     uint8_t* d_out_u8 = nullptr, const float* scale = nullptr,
                     const float* offset = nullptr)
{
    bf::LaunchArgs a{};
    a.in = d_in;
    a.out = d_out;
    a.lut = p->d_lut;
    a.ew = ew;
    a.tw = p->d_tw;
    a.mf = p->d_mf;
    a.n_chan = p->n_chan;
    a.n_units = n_frames * p->n_chan;
    a.n_blk = p->cfg.n_time / bf::kUp;
    a.n_time = p->cfg.n_time;
    a.st = nullptr;
    a.partial = nullptr;
    a.sym_ew = sym;
    a.cyl_sym = p->cyl_sym;
    a.split_v = p->cfg.precision == BF_FP32_MFMA ? 1 : 0;
    a.ew_by_unit = ew_by_unit;
    a.out_u8 = d_out_u8;
    a.scale = scale;
    a.offset = offset;
    hipError_t e = p->cfg.precision == BF_FP32_FFT ? bf::launch_fp32(a, stream)
                                                   : bf::launch_mfma(a, stream);
    if (e != hipSuccess) return hip_fail(p, e, "kernel launch");
    return BF_OK;
}

int32_t check_batch(bf_plan* p, const uint8_t* d_in, int32_t n_frames, const void* d_out)
{
    if (n_frames < 0) return fail(p, BF_E_INVAL, "n_frames < 0");
    if (n_frames == 0) return BF_OK;
    if (!d_in || !d_out) return fail(p, BF_E_INVAL, "NULL device buffer");
    if (((uintptr_t)d_in & 15) || ((uintptr_t)d_out & 15))
        return fail(p, BF_E_INVAL, "device buffers must be 16-byte aligned");
    if ((long long)n_frames * p->n_chan > (1LL << 26)) return fail(p, BF_E_INVAL, "batch too large");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(p, e, "hipGetDevice");
    if (dev != p->device) return fail(p, BF_E_STATE, "current device differs from the plan's device");
    return BF_OK;
}

// Per-frame E-W directions of a tracking call: finite, and whether every
// frame keeps the mirror symmetry the kernels' cheapest E-W form needs.
int32_t check_tracking(bf_plan* p, const double* sin_phi_ew, int32_t n_frames, bool* sym)
{
    if (!sin_phi_ew) return fail(p, BF_E_INVAL, "sin_phi_ew is NULL");
    *sym = true;
    for (int32_t f = 0; f < n_frames; ++f) {
        const double* s = sin_phi_ew + (size_t)f * bf::kBeamEW;
        for (int j = 0; j < bf::kBeamEW; ++j)
            if (!std::isfinite(s[j])) return fail(p, BF_E_INVAL, "sin_phi_ew must be finite");
        *sym = *sym && mirror_symmetric(p->cyl_x.data(), s);
    }
    return BF_OK;
}

// Weights of every channel-frame of a tracking call, FP64 rounded once:
// row f * n_chan + ch of out.
void fill_tracking(const bf_plan* p, const double* sin_phi_ew, int32_t n_frames, float2* out)
{
    for (int32_t f = 0; f < n_frames; ++f)
        for (int32_t ch = 0; ch < p->n_chan; ++ch)
            fill_ew(p->freqs[ch], p->cyl_x.data(), sin_phi_ew + (size_t)f * bf::kBeamEW, p->cfg.c0,
                    out + ((size_t)f * p->n_chan + ch) * bf::kBeamEW * bf::kCyl);
}

// Host staging of the allocation-free tracking entry point: pageable, fixed
// size, one table at a time (the mutex is held until the upload has read it).
std::mutex g_noalloc_stage_mutex;
float2 g_noalloc_stage[bf::kNoAllocRows * bf::kBeamEW * bf::kCyl];

}  // namespace

namespace bf {

// Stage-1 B fragments: lane (q, n) element i holds row K = 8q + i of the real
// form of the DFT-32 block, K = (a = 4q + i/2, re/im = i%2), column
// (c = n + 16 (tau & 1), re/im = tau >> 1); theta = 2 pi a c / 32.
// Stage-2 A fragments: lane (q, m) element i holds row (d = m, re/im = mu),
// K = (b = 4q + i/2, re/im = i%2); phi = 2 pi b d / 16.
// Complex product (cos - i sin)(xr + i xi): re = cos xr + sin xi,
// im = -sin xr + cos xi.  Each entry is FP64, split into FP16 hi + lo.
void build_mfma_tables(void* host_buf)
{
    _Float16* h = static_cast<_Float16*>(host_buf);
    auto put = [&](size_t frag, int lane, int i, double v) {
        const _Float16 hi = (_Float16)v;
        const _Float16 lo = (_Float16)(v - (double)hi);
        h[((frag * 2 + 0) * 64 + lane) * 8 + i] = hi;
        h[((frag * 2 + 1) * 64 + lane) * 8 + i] = lo;
    };
    for (int tau = 0; tau < 4; ++tau)
        for (int lane = 0; lane < 64; ++lane)
            for (int i = 0; i < 8; ++i) {
                const int q = lane >> 4, n = lane & 15;
                const int a = 4 * q + i / 2, ri = i & 1, c = n + 16 * (tau & 1), ro = tau >> 1;
                const double th = kTwoPi * (double)((a * c) % 32) / 32.0;
                const double v = ro == 0 ? (ri == 0 ? std::cos(th) : std::sin(th))
                                         : (ri == 0 ? -std::sin(th) : std::cos(th));
                put(tau, lane, i, v);
            }
    _Float16* h2 = h + 8 * 64 * 8;
    auto put2 = [&](int mu, int lane, int i, double v) {
        const _Float16 hi = (_Float16)v;
        const _Float16 lo = (_Float16)(v - (double)hi);
        h2[((mu * 2 + 0) * 64 + lane) * 8 + i] = hi;
        h2[((mu * 2 + 1) * 64 + lane) * 8 + i] = lo;
    };
    for (int mu = 0; mu < 2; ++mu)
        for (int lane = 0; lane < 64; ++lane)
            for (int i = 0; i < 8; ++i) {
                const int q = lane >> 4, d = lane & 15;
                const int b = 4 * q + i / 2, ri = i & 1;
                const double ph = kTwoPi * (double)((b * d) % 16) / 16.0;
                const double v = mu == 0 ? (ri == 0 ? std::cos(ph) : std::sin(ph))
                                         : (ri == 0 ? -std::sin(ph) : std::cos(ph));
                put2(mu, lane, i, v);
            }
    float2* tw = reinterpret_cast<float2*>(h2 + 4 * 64 * 8);
    for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 8; ++e) {
            const int q = lane >> 4, n = lane & 15;
            const int c = n + 16 * (e >> 2), b = 4 * q + (e & 3);
            const double a = kTwoPi * (double)((b * c) % kBins) / (double)kBins;
            tw[lane * 8 + e] = make_float2((float)std::cos(a), (float)-std::sin(a));
        }
}

}  // namespace bf

extern "C" {

int32_t beamform_default_config(bf_config* cfg)
{
    if (!cfg) return BF_E_INVAL;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->n_cyl = bf::kCyl;
    cfg->n_feed = bf::kFeed;
    cfg->n_pol = bf::kPol;
    cfg->pad = bf::kPad;
    cfg->n_beam_ns = bf::kBeamNS;
    cfg->n_beam_ew = bf::kBeamEW;
    cfg->n_upchan = bf::kUp;
    cfg->n_time = 384;
    cfg->feed_spacing_m = 0.3048;
    cfg->c0 = 299792458.0;
    cfg->precision = BF_FP32_FFT;
    return BF_OK;
}

int32_t beamform_compute_lut(const bf_config* cfg, const double* chan_freq_hz, int32_t n_chan,
                             int32_t* out)
{
    std::string msg;
    if (!cfg || !chan_freq_hz || !out || n_chan <= 0) return fail(nullptr, BF_E_INVAL, "bad arguments");
    if (cfg->n_feed <= 0 || cfg->pad <= 0 || cfg->n_beam_ns <= 0 || !(cfg->c0 > 0.0) ||
        !(cfg->feed_spacing_m > 0.0))
        return fail(nullptr, BF_E_INVAL, "bad geometry");
    int32_t r = fill_lut(cfg, chan_freq_hz, n_chan, out, &msg);
    return r == BF_OK ? BF_OK : fail(nullptr, r, msg);
}

int32_t beamform_init(const bf_config* cfg, const double* chan_freq_hz, int32_t n_chan,
                      void* stream, bf_plan** out_plan)
{
    bf::TraceRange trace_range("beamform_init");
    g_init_error.clear();
    if (!out_plan) return fail(nullptr, BF_E_INVAL, "out_plan is NULL");
    if (!chan_freq_hz || n_chan <= 0) return fail(nullptr, BF_E_INVAL, "need n_chan > 0 frequencies");
    std::string msg;
    int32_t st = check_config(cfg, &msg);
    if (st != BF_OK) return fail(nullptr, st, msg);

    bf_plan* p = new (std::nothrow) bf_plan();
    if (!p) return fail(nullptr, BF_E_NOMEM, "host allocation failed");
    p->cfg = *cfg;
    p->n_chan = n_chan;
    p->freqs.assign(chan_freq_hz, chan_freq_hz + n_chan);
    p->cyl_x.resize(bf::kCyl);
    p->sin_theta.resize(bf::kBeamNS);
    p->sin_phi.resize(bf::kBeamEW);
    for (int c = 0; c < bf::kCyl; ++c) p->cyl_x[c] = cfg->cyl_x_m ? cfg->cyl_x_m[c] : default_cyl_x(c);
    for (int m = 0; m < bf::kBeamNS; ++m)
        p->sin_theta[m] = cfg->sin_theta_ns ? cfg->sin_theta_ns[m] : default_sin_theta(m);
    for (int j = 0; j < bf::kBeamEW; ++j)
        p->sin_phi[j] = cfg->sin_phi_ew ? cfg->sin_phi_ew[j] : default_sin_phi(j);
    for (double v : p->cyl_x) if (!std::isfinite(v)) { delete p; return fail(nullptr, BF_E_INVAL, "cyl_x_m must be finite"); }
    for (double v : p->sin_phi) if (!std::isfinite(v)) { delete p; return fail(nullptr, BF_E_INVAL, "sin_phi_ew must be finite"); }

    p->sym_ew = mirror_symmetric(p->cyl_x.data(), p->sin_phi.data()) ? 1 : 0;
    p->cyl_sym = cylinders_symmetric(p->cyl_x.data()) ? 1 : 0;

    p->lut.resize((size_t)n_chan * bf::kBeamNS);
    bf_config tmp = *cfg;
    tmp.sin_theta_ns = p->sin_theta.data();
    st = fill_lut(&tmp, chan_freq_hz, n_chan, p->lut.data(), &msg);
    if (st != BF_OK) { delete p; return fail(nullptr, st, msg); }
    p->cfg.cyl_x_m = nullptr;
    p->cfg.sin_theta_ns = nullptr;
    p->cfg.sin_phi_ew = nullptr;
    p->cfg.lut_override = nullptr;

    // E-W weights and N-S twiddles in FP64, rounded once.
    std::vector<float2> ew((size_t)n_chan * bf::kBeamEW * bf::kCyl);
    for (int32_t ch = 0; ch < n_chan; ++ch)
        fill_ew(p->freqs[ch], p->cyl_x.data(), p->sin_phi.data(), cfg->c0,
                &ew[(size_t)ch * bf::kBeamEW * bf::kCyl]);
    std::vector<float2> tw(32 * 16);
    for (int c = 0; c < 32; ++c)
        for (int b = 0; b < 16; ++b) {
            const int r = (b * c) % bf::kBins;
            const double a = kTwoPi * (double)r / (double)bf::kBins;
            tw[c * 16 + b] = make_float2((float)std::cos(a), (float)-std::sin(a));
        }
    // w128^m, m < 128, of the 128-point up-channelisation (FP64 rounded once)
    std::vector<float2> tw128(128);
    for (int m = 0; m < 128; ++m) {
        const double a = kTwoPi * (double)m / 128.0;
        tw128[m] = make_float2((float)std::cos(a), (float)-std::sin(a));
    }

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { int32_t r = hip_fail(nullptr, e, "hipGetDevice"); delete p; return r; }
    // the fixed table of the allocation-free tracking entry point: its device
    // address is looked up here, once per device, with this device current
    if ((e = bf::noalloc_scratch(p->device, &p->d_scratch)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&p->noalloc_upload, hipEventDisableTiming)) != hipSuccess) {
        int32_t r = hip_fail(nullptr, e, "fixed tracking table");
        beamform_destroy(p);
        return r;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t lut_b = p->lut.size() * sizeof(int32_t), ew_b = ew.size() * sizeof(float2),
                 tw_b = tw.size() * sizeof(float2);
    std::vector<unsigned char> mf(bf::kMfmaTableBytes);
    bf::build_mfma_tables(mf.data());
    if ((e = hipMalloc(&p->d_lut, lut_b)) != hipSuccess ||
        (e = hipMalloc(&p->d_ew, ew_b)) != hipSuccess ||
        (e = hipMalloc(&p->d_tw, tw_b)) != hipSuccess ||
        (e = hipMalloc(&p->d_mf, mf.size())) != hipSuccess ||
        (e = hipMalloc(&p->d_tw128, tw128.size() * sizeof(float2))) != hipSuccess) {
        int32_t r = fail(nullptr, BF_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        beamform_destroy(p);
        return r;
    }
    if ((e = hipMemcpyAsync(p->d_lut, p->lut.data(), lut_b, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(p->d_ew, ew.data(), ew_b, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(p->d_tw, tw.data(), tw_b, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(p->d_mf, mf.data(), mf.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(p->d_tw128, tw128.data(), tw128.size() * sizeof(float2),
                            hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
        int32_t r = hip_fail(nullptr, e, "table upload");
        beamform_destroy(p);
        return r;
    }
    *out_plan = p;
    return BF_OK;
}

int32_t beamform_frame(bf_plan* p, const uint8_t* d_in, int32_t n_frames, float* d_out,
                       void* stream)
{
    bf::TraceRange trace_range("beamform_frame");
    if (!p) return BF_E_INVAL;
    p->err.clear();
    int32_t st = check_batch(p, d_in, n_frames, d_out);
    if (st != BF_OK || n_frames == 0) return st;
    return launch_batch(p, d_in, n_frames, d_out, (hipStream_t)stream, p->d_ew, 0, p->sym_ew);
}

int32_t beamform_frame_u8(bf_plan* p, const uint8_t* d_in, int32_t n_frames,
                          const float* d_scale, const float* d_offset, uint8_t* d_out,
                          void* stream)
{
    bf::TraceRange trace_range("beamform_frame_u8");
    if (!p) return BF_E_INVAL;
    p->err.clear();
    int32_t st = check_batch(p, d_in, n_frames, d_out);
    if (st != BF_OK || n_frames == 0) return st;
    if (!d_scale || !d_offset) return fail(p, BF_E_INVAL, "NULL scale or offset table");
    if (((uintptr_t)d_scale & 3) || ((uintptr_t)d_offset & 3))
        return fail(p, BF_E_INVAL, "scale and offset tables must be 4-byte aligned");
    return launch_batch(p, d_in, n_frames, nullptr, (hipStream_t)stream, p->d_ew, 0, p->sym_ew,
                        d_out, d_scale, d_offset);
}

int32_t beamform_frame_upchan128(bf_plan* p, const uint8_t* d_in, int32_t n_frames, float* d_out,
                                 void* stream)
{
    bf::TraceRange trace_range("beamform_frame_upchan128");
    if (!p) return BF_E_INVAL;
    p->err.clear();
    int32_t st = check_batch(p, d_in, n_frames, d_out);
    if (st != BF_OK || n_frames == 0) return st;
    if (p->cfg.n_time % 128 != 0)
        return fail(p, BF_E_UNSUPPORTED, "the 128-point up-channelisation needs n_time % 128 == 0");
    bf::LaunchArgs a{};
    a.in = d_in;
    a.out = d_out;
    a.lut = p->d_lut;
    a.ew = p->d_ew;
    a.tw = p->d_tw;
    a.mf = p->d_mf;
    a.tw128 = p->d_tw128;
    a.n_chan = p->n_chan;
    a.n_units = n_frames * p->n_chan;
    a.n_blk = p->cfg.n_time / bf::kUp;
    a.n_time = p->cfg.n_time;
    a.sym_ew = p->sym_ew;
    a.cyl_sym = p->cyl_sym;
    a.split_v = p->cfg.precision == BF_FP32_MFMA ? 1 : 0;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = p->cfg.precision == BF_FP32_FFT ? bf::launch_fp32_up128(a, s)
                                                   : bf::launch_mfma_up128(a, s);
    if (e != hipSuccess) return hip_fail(p, e, "kernel launch");
    return BF_OK;
}

int32_t beamform_debug_ns(bf_plan* p, const uint8_t* d_in, float* d_ns_out, void* stream)
{
    bf::TraceRange trace_range("beamform_debug_ns");
    if (!p) return BF_E_INVAL;
    p->err.clear();
    int32_t st = check_batch(p, d_in, 1, d_ns_out);
    if (st != BF_OK) return st;
    bf::LaunchArgs a{};
    a.in = d_in;
    a.lut = p->d_lut;
    a.ew = p->d_ew;
    a.tw = p->d_tw;
    a.mf = p->d_mf;
    a.n_chan = p->n_chan;
    a.n_units = p->n_chan;
    a.n_blk = p->cfg.n_time / bf::kUp;
    a.n_time = p->cfg.n_time;
    a.sym_ew = p->sym_ew;
    a.cyl_sym = p->cyl_sym;
    a.split_v = p->cfg.precision == BF_FP32_MFMA ? 1 : 0;
    a.fine = reinterpret_cast<float2*>(d_ns_out);
    hipError_t e = p->cfg.precision == BF_FP32_FFT ? bf::launch_fp32(a, (hipStream_t)stream)
                                                   : bf::launch_mfma(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(p, e, "kernel launch");
    return BF_OK;
}

int32_t beamform_frame_tracking(bf_plan* p, const uint8_t* d_in, int32_t n_frames,
                                const double* sin_phi_ew, float* d_out, void* stream)
{
    bf::TraceRange trace_range("beamform_frame_tracking");
    if (!p) return BF_E_INVAL;
    p->err.clear();
    int32_t st = check_batch(p, d_in, n_frames, d_out);
    if (st != BF_OK || n_frames == 0) return st;
    bool sym = true;
    if ((st = check_tracking(p, sin_phi_ew, n_frames, &sym)) != BF_OK) return st;
    const size_t rows = (size_t)n_frames * p->n_chan, row_b = bf::kBeamEW * bf::kCyl * sizeof(float2);
    bf_plan::EwTrack& t = p->ew_track[p->ew_track_next];
    hipError_t e = hipSuccess;
    if (!t.done && (e = hipEventCreateWithFlags(&t.done, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(p, e, "hipEventCreate");
    // The kernel of the call before last may still read this buffer pair and its
    // upload may still read the staging half: wait for it before reuse.
    if ((e = hipEventSynchronize(t.done)) != hipSuccess)
        return hip_fail(p, e, "previous tracking call");
    if (rows > t.cap) {
        if (t.d) (void)hipFree(t.d);
        if (t.h) (void)hipHostFree(t.h);
        t.d = nullptr;
        t.h = nullptr;
        t.cap = 0;
        if ((e = hipMalloc(&t.d, rows * row_b)) != hipSuccess ||
            (e = hipHostMalloc((void**)&t.h, rows * row_b, hipHostMallocDefault)) != hipSuccess) {
            if (t.d) (void)hipFree(t.d);
            t.d = nullptr;
            return fail(p, BF_E_NOMEM, std::string("tracking table: ") + hipGetErrorString(e));
        }
        t.cap = rows;
    }
    fill_tracking(p, sin_phi_ew, n_frames, t.h);
    hipStream_t s = (hipStream_t)stream;
    if ((e = hipMemcpyAsync(t.d, t.h, rows * row_b, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(p, e, "tracking table upload");
    st = launch_batch(p, d_in, n_frames, d_out, s, t.d, 1, sym ? 1 : 0);
    if ((e = hipEventRecord(t.done, s)) != hipSuccess && st == BF_OK)
        st = hip_fail(p, e, "hipEventRecord");
    p->ew_track_next ^= 1;
    return st;
}

int32_t beamform_frame_tracking_noalloc(bf_plan* p, const uint8_t* d_in, int32_t n_frames,
                                        const double* sin_phi_ew, float* d_out, void* stream)
{
    bf::TraceRange trace_range("beamform_frame_tracking_noalloc");
    if (!p) return BF_E_INVAL;
    p->err.clear();
    int32_t st = check_batch(p, d_in, n_frames, d_out);
    if (st != BF_OK || n_frames == 0) return st;
    bool sym = true;
    if ((st = check_tracking(p, sin_phi_ew, n_frames, &sym)) != BF_OK) return st;
    const long long rows = (long long)n_frames * p->n_chan;
    if (rows > bf::kNoAllocRows)
        return fail(p, BF_E_INVAL, "n_frames x n_chan = " + std::to_string(rows) +
                                       " exceeds the fixed tracking table of " +
                                       std::to_string(bf::kNoAllocRows) + " channel-frames");
    if (!p->d_scratch || !p->noalloc_upload) return fail(p, BF_E_STATE, "no fixed tracking table");
    const size_t bytes = (size_t)rows * bf::kBeamEW * bf::kCyl * sizeof(float2);
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(g_noalloc_stage_mutex);
    fill_tracking(p, sin_phi_ew, n_frames, g_noalloc_stage);
    hipError_t e = hipMemcpyAsync(p->d_scratch, g_noalloc_stage, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(p, e, "fixed tracking table upload");
    if ((e = hipEventRecord(p->noalloc_upload, s)) != hipSuccess)
        return hip_fail(p, e, "hipEventRecord");
    st = launch_batch(p, d_in, n_frames, d_out, s, p->d_scratch, 1, sym ? 1 : 0);
    // the staging table is reused by the next call: wait until the upload read it
    if ((e = hipEventSynchronize(p->noalloc_upload)) != hipSuccess && st == BF_OK)
        st = hip_fail(p, e, "fixed tracking table upload");
    return st;
}

int32_t beamform_get_lut(const bf_plan* p, int32_t* host_out)
{
    if (!p || !host_out) return BF_E_INVAL;
    std::memcpy(host_out, p->lut.data(), p->lut.size() * sizeof(int32_t));
    return BF_OK;
}

int32_t beamform_plan_info(const bf_plan* p, int32_t* n_chan, int32_t* n_time, int32_t* precision)
{
    if (!p) return BF_E_INVAL;
    if (n_chan) *n_chan = p->n_chan;
    if (n_time) *n_time = p->cfg.n_time;
    if (precision) *precision = p->cfg.precision;
    return BF_OK;
}

int32_t beamform_destroy(bf_plan* p)
{
    bf::TraceRange trace_range("beamform_destroy");
    if (!p) return BF_OK;
    int32_t st = BF_OK;
    int prev = -1;
    if (hipGetDevice(&prev) == hipSuccess && prev != p->device) (void)hipSetDevice(p->device);
    if (hipDeviceSynchronize() != hipSuccess) st = BF_E_DEVICE;
    if (p->d_lut) (void)hipFree(p->d_lut);
    if (p->d_ew) (void)hipFree(p->d_ew);
    if (p->d_tw) (void)hipFree(p->d_tw);
    if (p->d_mf) (void)hipFree(p->d_mf);
    if (p->d_tw128) (void)hipFree(p->d_tw128);
    if (p->noalloc_upload) (void)hipEventDestroy(p->noalloc_upload);
    for (bf_plan::EwTrack& t : p->ew_track) {
        if (t.d) (void)hipFree(t.d);
        if (t.h) (void)hipHostFree(t.h);
        if (t.done) (void)hipEventDestroy(t.done);
    }
    if (prev >= 0 && prev != p->device) (void)hipSetDevice(prev);
    delete p;
    return st;
}

const char* beamform_strerror(int32_t status)
{
    switch (status) {
    case BF_OK: return "ok";
    case BF_E_INVAL: return "invalid argument";
    case BF_E_NOMEM: return "out of memory";
    case BF_E_DEVICE: return "device error";
    case BF_E_STATE: return "invalid state";
    case BF_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char* beamform_last_error(const bf_plan* p)
{
    return p ? p->err.c_str() : g_init_error.c_str();
}

}  // extern "C"
