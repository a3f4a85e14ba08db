// Serving loop: frames for a varying set of channels, beamformed from a
// device input ring into a device output ring, one launch per chunk of every
// frame (paper Sec. 2: each frequency channel is an endless stream of 2.56 us
// samples; Sec. 3 and Table 1: 0.983 ms output cadence).
//
// Host side per launch: apply the frame's join/leave events (slot assignment,
// admission by memory), copy a small StreamState (ring entry, chunk, active
// slots) host -> device, replay the captured kernel graph, record an event.
// A completion thread waits on those events in order and timestamps them;
// frame latency = completion of the frame's last launch - availability of its
// last chunk.  Host-paced, the host waits for each chunk's availability before
// launching it, and latency is taken on the host clock.  Device-gated, the
// availability times are kept on the device's constant-rate wall clock (the
// schedule's start aligned once to the host clock): the host queues launches
// ahead, a one-wave gate kernel in front of each launch holds the stream until
// the chunk's time, and a one-wave stamp after each frame's last launch gives
// its completion on the same clock, so latency is the device's own (the data
// arrive as from a receiver writing into HBM at line rate, whatever the host
// threads do, and the two clocks' drift does not enter).  The HIP runtime's launch calls now and
// then block for milliseconds, which a host-paced loop passes on to every frame
// behind the stall and a queue of gated launches absorbs (a host thread that
// published arrivals was no better: it could share a CPU with the runtime's
// busy wait on events and then ran only every few milliseconds).  All device
// state is allocated when the loop starts and freed before it returns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "bf_gate.h"
#include "bf_plan.h"
#include "bf_trace.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr double kSampleS = 2.56e-6;
constexpr int kInFlight = BF_STREAM_RUN_AHEAD;  // launches the host may run ahead of the device
constexpr int32_t kGateTimeoutMs = 1000;        // default bound of one gated wait, plus two
                                                // chunk periods
constexpr int kClockProbes = 5;                 // host/device clock alignment attempts
constexpr size_t kTabBytes = bf::kBeamNS * sizeof(int32_t) + bf::kBeamEW * bf::kCyl * sizeof(float2);

// Channel slots, admission and event application (pure host; no device).
struct Scheduler {
    int max_slots, capacity;
    bf_config geo;  // geometry and pointings a joining channel's Eq. (1) bins use
    std::vector<int32_t> slot_chan;
    std::vector<double> slot_freq;
    int n_active = 0;
    int64_t joins = 0, leaves = 0, rejected = 0, ignored = 0;

    Scheduler(int max_slots_, int capacity_, const bf_config& geo_)
        : max_slots(max_slots_), capacity(capacity_), geo(geo_), slot_chan(max_slots_, -1),
          slot_freq(max_slots_, 0.0) {}

    // The channel's Eq. (1) bin table can be formed (finite, positive frequency
    // whose argument stays within an exact integer floor).
    bool freq_ok(double f)
    {
        int32_t bins[bf::kBeamNS];
        return std::isfinite(f) && f > 0.0 && beamform_compute_lut(&geo, &f, 1, bins) == BF_OK;
    }

    int find(int32_t chan) const
    {
        for (int s = 0; s < max_slots; ++s)
            if (slot_chan[s] == chan) return s;
        return -1;
    }
    // Returns the slot a JOIN filled, else -1.
    int apply(const bf_stream_event& e)
    {
        if (e.op == BF_STREAM_JOIN) {
            if (e.channel_id < 0 || find(e.channel_id) >= 0 || !freq_ok(e.freq_hz)) {
                ++ignored;
                return -1;
            }
            if (n_active >= capacity) {
                ++rejected;
                return -1;
            }
            for (int s = 0; s < max_slots; ++s)
                if (slot_chan[s] < 0) {
                    slot_chan[s] = e.channel_id;
                    slot_freq[s] = e.freq_hz;
                    ++n_active;
                    ++joins;
                    return s;
                }
            ++rejected;  // unreachable while capacity <= max_slots
            return -1;
        }
        if (e.op == BF_STREAM_LEAVE) {
            const int s = e.channel_id >= 0 ? find(e.channel_id) : -1;
            if (s < 0) {
                ++ignored;
                return -1;
            }
            slot_chan[s] = -1;
            --n_active;
            ++leaves;
            return -1;
        }
        ++ignored;
        return -1;
    }
    int active(int32_t* slots) const
    {
        int n = 0;
        for (int s = 0; s < max_slots; ++s)
            if (slot_chan[s] >= 0) slots[n++] = s;
        return n;
    }
};

int32_t check_desc(const bf_stream_desc* d, std::string* msg)
{
    if (!d) { *msg = "desc is NULL"; return BF_E_INVAL; }
    if (d->depth < 1) { *msg = "depth must be >= 1"; return BF_E_INVAL; }
    if (d->max_slots < 1 || d->max_slots > BF_STREAM_MAX_SLOTS) {
        *msg = "max_slots must be in [1, BF_STREAM_MAX_SLOTS]";
        return BF_E_INVAL;
    }
    if (d->n_frames < 0) { *msg = "n_frames < 0"; return BF_E_INVAL; }
    if (d->n_events < 0 || (d->n_events > 0 && !d->events)) { *msg = "bad events"; return BF_E_INVAL; }
    if (d->warmup_frames < 0 || d->warmup_frames > d->n_frames) {
        *msg = "warmup_frames must be in [0, n_frames]";
        return BF_E_INVAL;
    }
    if (d->pacing != BF_STREAM_PACE_NONE && d->pacing != BF_STREAM_PACE_HOST &&
        d->pacing != BF_STREAM_PACE_GATED) {
        *msg = "pacing must be 0, 1 or 2";
        return BF_E_INVAL;
    }
    if (d->gate_timeout_ms < 0 || d->reserved2 != 0) {
        *msg = "gate_timeout_ms must be >= 0 and reserved2 0";
        return BF_E_INVAL;
    }
    if (d->mem_cap_bytes < 0) { *msg = "mem_cap_bytes < 0"; return BF_E_INVAL; }
    for (int32_t i = 1; i < d->n_events; ++i)
        if (d->events[i].frame < d->events[i - 1].frame) {
            *msg = "events must be sorted by frame";
            return BF_E_INVAL;
        }
    return BF_OK;
}

int64_t per_slot_bytes(int depth, int n_time, bool partial_sums)
{
    // the slot's share of both rings, its partial sums (chunked ingest only) and
    // its table rows
    return (int64_t)depth * ((int64_t)n_time * bf::kInputs + (int64_t)bf::kOutPerUnit * 4) +
           (partial_sums ? (int64_t)4 * bf::kPartialPerWg * 4 : 0) + (int64_t)kTabBytes;
}

// Default geometry for the host-only dry run's Eq. (1) check.
bf_config default_geometry()
{
    bf_config c;
    beamform_default_config(&c);
    return c;
}

// Active slots of frame i for the launches: the slot indices, each marked
// missing when the ingest did not deliver that channel-frame.  Returns the
// number of missing ones.
int mark_missing(const bf_stream_desc* d, int32_t i, const int32_t* act, int n_act, int32_t* out)
{
    int missing = 0;
    for (int u = 0; u < n_act; ++u) {
        const bool ok = !d->ingest_ok || d->ingest_ok[(size_t)i * d->max_slots + act[u]] != 0;
        out[u] = ok ? act[u] : (act[u] | bf::kSlotMissing);
        missing += ok ? 0 : 1;
    }
    return missing;
}

double quantile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

// Bin table and E-W weights of one channel (FP64, rounded once), as in
// beamform_init; false if the bin table cannot be formed (the scheduler admits
// no such channel).
bool channel_tables(const bf_plan* p, double f, unsigned char* dst)
{
    int32_t* lut = reinterpret_cast<int32_t*>(dst);
    float2* ew = reinterpret_cast<float2*>(dst + bf::kBeamNS * sizeof(int32_t));
    bf_config c = p->cfg;
    c.sin_theta_ns = p->sin_theta.data();
    c.lut_override = nullptr;
    if (beamform_compute_lut(&c, &f, 1, lut) != BF_OK) return false;
    const double two_pi = 6.283185307179586476925286766559;
    for (int j = 0; j < bf::kBeamEW; ++j)
        for (int cy = 0; cy < bf::kCyl; ++cy) {
            const double a = two_pi * f * p->cyl_x[cy] * p->sin_phi[j] / p->cfg.c0;
            ew[j * bf::kCyl + cy] = make_float2((float)std::cos(a), (float)-std::sin(a));
        }
    return true;
}

struct LaunchRec {
    int32_t frame;
    bool last_chunk;
    Clock::time_point avail;
    uint64_t arrival_tick;  // device-gated: availability on the device wall clock
};

}  // namespace

extern "C" {

int32_t beamform_stream_schedule(const bf_stream_desc* d, int64_t psb, int64_t cap,
                                 bf_stream_stats* st)
{
    std::string msg;
    if (check_desc(d, &msg) != BF_OK || psb <= 0 || cap < 0 || !st) return BF_E_INVAL;
    std::memset(st, 0, sizeof(*st));
    const int capacity = (int)std::min<int64_t>(d->max_slots, cap / psb);
    Scheduler sch(d->max_slots, capacity, default_geometry());
    std::vector<int32_t> act(d->max_slots), marked(d->max_slots);
    int32_t ev = 0;
    st->min_active = d->n_frames > 0 ? d->max_slots : 0;
    for (int32_t i = 0; i < d->n_frames; ++i) {
        while (ev < d->n_events && d->events[ev].frame <= i) sch.apply(d->events[ev++]);
        if (d->slot_log)
            std::memcpy(d->slot_log + (size_t)i * d->max_slots, sch.slot_chan.data(),
                        sizeof(int32_t) * d->max_slots);
        const int n_act = sch.active(act.data());
        st->missing_frames += mark_missing(d, i, act.data(), n_act, marked.data());
        st->channel_frames += sch.n_active;
        st->max_active = std::max(st->max_active, sch.n_active);
        st->min_active = std::min(st->min_active, sch.n_active);
    }
    st->frames = d->n_frames;
    st->joins = sch.joins;
    st->leaves = sch.leaves;
    st->rejected_joins = sch.rejected;
    st->ignored_events = sch.ignored + (d->n_events - ev);
    st->per_slot_bytes = psb;
    st->slot_capacity = capacity;
    return BF_OK;
}

int32_t beamform_stream(bf_plan* p, const bf_stream_desc* d, bf_stream_stats* st, void* stream)
{
    bf::TraceRange trace_range("beamform_stream");
    if (!p || !st) return BF_E_INVAL;
    p->err.clear();
    std::string msg;
    int32_t rc = check_desc(d, &msg);
    if (rc != BF_OK) { p->err = msg; return rc; }
    const int n_time = p->cfg.n_time;
    const int chunk = d->chunk ? d->chunk : n_time;
    if (chunk <= 0 || chunk % bf::kUp != 0 || n_time % chunk != 0) {
        p->err = "chunk must be a multiple of 16 dividing n_time";
        return BF_E_INVAL;
    }
    if (d->n_frames > 0 && (!d->d_in_ring || !d->d_out_ring)) {
        p->err = "NULL ring";
        return BF_E_INVAL;
    }
    if (((uintptr_t)d->d_in_ring & 15) || ((uintptr_t)d->d_out_ring & 15)) {
        p->err = "rings must be 16-byte aligned";
        return BF_E_INVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
        p->err = "current device differs from the plan's device";
        return BF_E_STATE;
    }
    const int n_chunks = n_time / chunk;
    std::memset(st, 0, sizeof(*st));
    const int64_t psb = per_slot_bytes(d->depth, n_time, n_chunks > 1);
    int64_t cap = d->mem_cap_bytes;
    if (cap == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            p->err = "hipMemGetInfo failed";
            return BF_E_DEVICE;
        }
        cap = (int64_t)free_b;
    }
    const int capacity = (int)std::min<int64_t>(d->max_slots, cap / psb);
    st->per_slot_bytes = psb;
    st->slot_capacity = capacity;

    // ---- device and pinned state ----
    hipError_t e = hipSuccess;
    const int S = d->max_slots;
    int32_t* d_lut = nullptr;
    float2* d_ew = nullptr;
    float* d_partial = nullptr;
    bf::StreamState* d_state = nullptr;
    bf::StreamState* h_state = nullptr;  // [kInFlight] launch states, coherent pinned memory
    bf::StreamState* d_hstate = nullptr; // their device address (the gates read them)
    unsigned char* h_tab = nullptr;
    const bool gated = d->pacing == BF_STREAM_PACE_GATED;
    uint64_t* d_gate = nullptr;        // [0] low word: set by a gate that timed out; [1] clock probe
    uint64_t* h_stamp = nullptr;       // [kInFlight] completion stamps, coherent pinned memory
    uint64_t* d_stamp = nullptr;       // their device address
    hipStream_t s = nullptr;
    hipEvent_t ev_start[kInFlight] = {}, ev_end[kInFlight] = {}, ev_sync = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto cleanup = [&]() {
        if (s) (void)hipStreamSynchronize(s);  // queued gates end by their arrival ticks
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (int k = 0; k < kInFlight; ++k) {
            if (ev_start[k]) (void)hipEventDestroy(ev_start[k]);
            if (ev_end[k]) (void)hipEventDestroy(ev_end[k]);
        }
        if (ev_sync) (void)hipEventDestroy(ev_sync);
        if (s) (void)hipStreamDestroy(s);
        if (d_lut) (void)hipFree(d_lut);
        if (d_ew) (void)hipFree(d_ew);
        if (d_partial) (void)hipFree(d_partial);
        if (d_state) (void)hipFree(d_state);
        if (h_state) (void)hipHostFree(h_state);
        if (h_tab) (void)hipHostFree(h_tab);
        if (d_gate) (void)hipFree(d_gate);
        if (h_stamp) (void)hipHostFree(h_stamp);
    };
    auto fail = [&](const char* what) -> int32_t {
        p->err = std::string(what) + ": " + hipGetErrorString(e);
        cleanup();
        return BF_E_DEVICE;
    };
    if ((e = hipMalloc(&d_lut, (size_t)S * bf::kBeamNS * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&d_ew, (size_t)S * bf::kBeamEW * bf::kCyl * sizeof(float2))) != hipSuccess ||
        (e = hipMalloc(&d_state, sizeof(bf::StreamState))) != hipSuccess)
        return fail("hipMalloc");
    if (n_chunks > 1 &&
        (e = hipMalloc(&d_partial, (size_t)S * 4 * bf::kPartialPerWg * sizeof(float))) != hipSuccess)
        return fail("hipMalloc partial sums");
    if ((e = hipHostMalloc((void**)&h_state, sizeof(bf::StreamState) * kInFlight, hipHostMallocCoherent)) !=
            hipSuccess ||
        (e = hipHostGetDevicePointer((void**)&d_hstate, h_state, 0)) != hipSuccess ||
        (e = hipHostMalloc((void**)&h_tab, kTabBytes * S, 0)) != hipSuccess)
        return fail("hipHostMalloc");
    uint64_t gate_ticks = 0;
    int khz = 0;
    if (gated) {
        if ((e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess)
            return fail("wall clock rate");
        if (khz <= 0 || khz > 10000000) {  // a rate in kHz, 10 GHz at most
            e = hipErrorInvalidValue;
            return fail("wall clock rate");
        }
        const double bound_ms = d->gate_timeout_ms ? (double)d->gate_timeout_ms
                                                   : kGateTimeoutMs + 2e3 * chunk * kSampleS;
        gate_ticks = (uint64_t)((double)khz * bound_ms);
        if ((e = hipMalloc(&d_gate, 2 * sizeof(uint64_t))) != hipSuccess ||
            (e = hipHostMalloc((void**)&h_stamp, kInFlight * sizeof(uint64_t), hipHostMallocCoherent)) !=
                hipSuccess ||
            (e = hipHostGetDevicePointer((void**)&d_stamp, h_stamp, 0)) != hipSuccess)
            return fail("gate state");
    }
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return fail("stream");
    for (int k = 0; k < kInFlight; ++k)
        if ((e = hipEventCreate(&ev_start[k])) != hipSuccess ||
            (e = hipEventCreate(&ev_end[k])) != hipSuccess)
            return fail("hipEventCreate");
    if ((e = hipEventCreateWithFlags(&ev_sync, hipEventDisableTiming)) != hipSuccess) return fail("event");
    // start after the caller's stream has reached this point
    if ((e = hipEventRecord(ev_sync, (hipStream_t)stream)) != hipSuccess ||
        (e = hipStreamWaitEvent(s, ev_sync, 0)) != hipSuccess)
        return fail("stream ordering");

    bf::LaunchArgs a{};
    a.in = d->d_in_ring;
    a.out = d->d_out_ring;
    a.lut = d_lut;
    a.ew = d_ew;
    a.tw = p->d_tw;
    a.mf = p->d_mf;
    a.st = d_state;
    a.partial = d_partial;
    a.n_chan = 1;
    a.n_units = S;
    a.n_blk = chunk / bf::kUp;
    a.n_time = n_time;
    a.max_slots = S;
    a.sym_ew = p->sym_ew;
    a.cyl_sym = p->cyl_sym;
    a.split_v = p->cfg.precision == BF_FP32_MFMA ? 1 : 0;
    auto launch = [&](hipStream_t on) {
        return p->cfg.precision == BF_FP32_FFT ? bf::launch_fp32(a, on) : bf::launch_mfma(a, on);
    };
    if (d->use_graph) {
        if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return fail("hipStreamBeginCapture");
        hipError_t le = launch(s);
        e = hipStreamEndCapture(s, &graph);
        if (le != hipSuccess) { e = le; return fail("captured launch"); }
        if (e != hipSuccess) return fail("hipStreamEndCapture");
        if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess)
            return fail("hipGraphInstantiate");
    }
    // Warm start: one launch with no active slot (every workgroup returns at
    // once), and one gate that passes at once, before the clock starts, so that
    // the first paced frame does not pay the first replay's one-time setup.
    {
        std::memset(&h_state[0], 0, bf::kStreamStateHeader);
        if ((gated && ((e = hipMemsetAsync(d_gate, 0, 2 * sizeof(uint64_t), s)) != hipSuccess ||
                       (e = bf::launch_ingest_gate(0, gate_ticks, reinterpret_cast<int32_t*>(d_gate), nullptr,
                                                   nullptr, 0, s)) != hipSuccess)) ||
            (e = hipMemcpyAsync(d_state, &h_state[0], bf::kStreamStateHeader, hipMemcpyHostToDevice,
                                s)) != hipSuccess ||
            (e = (d->use_graph ? hipGraphLaunch(exec, s) : launch(s))) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return fail("warm-up launch");
    }
    // Device-gated: align the device wall clock with the host clock.  Each probe
    // reads the device clock between two host readings ta < tb; the probe with
    // the shortest round trip is kept and its reading taken as made at ta, so
    // that a gate opens at its chunk's availability or at most that round trip
    // (tens of microseconds) after it, never before.
    uint64_t clk0 = 0;
    Clock::time_point clk0_host{};
    if (gated) {
        Clock::duration best = Clock::duration::max();
        for (int k = 0; k < kClockProbes; ++k) {
            uint64_t v = 0;
            const Clock::time_point ta = Clock::now();
            if ((e = bf::launch_wall_clock_probe(d_gate + 1, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return fail("clock probe");
            const Clock::time_point tb = Clock::now();
            if ((e = hipMemcpyAsync(&v, d_gate + 1, sizeof v, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return fail("clock probe");
            if (tb - ta < best) {
                best = tb - ta;
                clk0 = v;
                clk0_host = ta;
            }
        }
    }

    // ---- completion thread ----
    std::vector<LaunchRec> recs(kInFlight);
    std::vector<double> lat_ms((size_t)d->n_frames, 0.0), svc_ms((size_t)d->n_frames, 0.0),
        issue_ms((size_t)d->n_frames, 0.0);
    std::atomic<int64_t> launched{0}, completed{0};
    std::atomic<bool> stop{false};
    std::atomic<int> thread_err{0};
    const int device = p->device;
    std::thread waiter([&]() {
        (void)hipSetDevice(device);
        for (int64_t L = 0;; ++L) {
            while (L >= launched.load(std::memory_order_acquire)) {
                if (stop.load(std::memory_order_acquire) && L >= launched.load()) return;
                std::this_thread::yield();
            }
            const int k = (int)(L % kInFlight);
            if (hipEventSynchronize(ev_end[k]) != hipSuccess) thread_err.store(1);
            const Clock::time_point now = Clock::now();
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev_start[k], ev_end[k]);
            const LaunchRec r = recs[k];
            svc_ms[r.frame] += ms;
            if (r.last_chunk && gated) {
                const uint64_t done = __atomic_load_n(&h_stamp[k], __ATOMIC_ACQUIRE);
                lat_ms[r.frame] = (double)(int64_t)(done - r.arrival_tick) / (double)khz;
            } else if (r.last_chunk) {
                lat_ms[r.frame] = std::chrono::duration<double, std::milli>(now - r.avail).count();
            }
            completed.store(L + 1, std::memory_order_release);
        }
    });
    auto wait_completed = [&](int64_t n) {
        while (completed.load(std::memory_order_acquire) < n && !thread_err.load())
            std::this_thread::yield();
    };

    // ---- main loop ----
    bf_config geo = p->cfg;
    geo.sin_theta_ns = p->sin_theta.data();
    geo.lut_override = nullptr;
    Scheduler sch(S, capacity, geo);
    std::vector<int64_t> tab_launch(S, -1);
    std::vector<int32_t> act(S), act_launch(S);
    int32_t evi = 0;
    int64_t L = 0;
    st->min_active = d->n_frames > 0 ? S : 0;
    // The schedule starts once frame 0's events (the initial channel set) have
    // been applied: t0 = that moment + 0.5 ms, so that their table uploads do not
    // count against the first frame.
    Clock::time_point t_start = Clock::now();
    Clock::time_point t0 = t_start + std::chrono::microseconds(500);
    // availability of chunk c of frame i (the last sample's arrival)
    auto avail_at = [&](int64_t i, int c) {
        return t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(
                        ((double)i * n_time + (double)(c + 1) * chunk) * kSampleS));
    };
    // the same on the device wall clock (device-gated): t0 mapped through the
    // probe, the schedule itself in device ticks
    const double ticks_per_s = (double)khz * 1e3;
    double t0_ticks = 0.0;
    auto start_schedule = [&]() {
        t_start = Clock::now();
        t0 = t_start + std::chrono::microseconds(500);
        t0_ticks = (double)clk0 +
                   std::max(0.0, std::chrono::duration<double>(t0 - clk0_host).count()) * ticks_per_s;
    };
    start_schedule();
    auto arrival_tick = [&](int64_t i, int c) {
        return (uint64_t)std::ceil(t0_ticks +
                                   ((double)i * n_time + (double)(c + 1) * chunk) * kSampleS * ticks_per_s);
    };
    // wait on the host clock until `when` (sleeping while far, yielding near)
    auto wait_until = [](Clock::time_point when) {
        for (;;) {
            const auto now = Clock::now();
            if (now >= when) return;
            if (when - now > std::chrono::microseconds(300))
                std::this_thread::sleep_for(std::chrono::microseconds(100));
            else
                std::this_thread::yield();
        }
    };
    int32_t status = BF_OK;
    for (int32_t i = 0; i < d->n_frames && status == BF_OK; ++i) {
        while (evi < d->n_events && d->events[evi].frame <= i) {
            const int slot = sch.apply(d->events[evi++]);
            if (slot < 0) continue;
            // the staging row may still feed an earlier copy: queued copies are
            // read when they execute, so wait for it (drain the stream when that
            // copy's launch has not even been issued, i.e. same-frame reuse)
            if (tab_launch[slot] >= 0) {
                if (tab_launch[slot] >= launched.load(std::memory_order_acquire)) {
                    if ((e = hipStreamSynchronize(s)) != hipSuccess) { status = BF_E_DEVICE; break; }
                } else {
                    wait_completed(tab_launch[slot] + 1);
                }
            }
            unsigned char* row = h_tab + kTabBytes * slot;
            if (!channel_tables(p, sch.slot_freq[slot], row)) {
                status = BF_E_STATE;
                e = hipErrorInvalidValue;
                break;
            }
            if ((e = hipMemcpyAsync(d_lut + (size_t)slot * bf::kBeamNS, row,
                                    bf::kBeamNS * sizeof(int32_t), hipMemcpyHostToDevice, s)) != hipSuccess ||
                (e = hipMemcpyAsync(d_ew + (size_t)slot * bf::kBeamEW * bf::kCyl,
                                    row + bf::kBeamNS * sizeof(int32_t),
                                    bf::kBeamEW * bf::kCyl * sizeof(float2), hipMemcpyHostToDevice,
                                    s)) != hipSuccess) {
                status = BF_E_DEVICE;
                break;
            }
            tab_launch[slot] = L;
        }
        if (status != BF_OK) break;
        if (i == 0) start_schedule();
        const int n_act = sch.active(act.data());
        if (d->slot_log)
            std::memcpy(d->slot_log + (size_t)i * S, sch.slot_chan.data(), sizeof(int32_t) * S);
        const int n_missing = mark_missing(d, i, act.data(), n_act, act_launch.data());
        st->missing_frames += n_missing;
        st->channel_frames += n_act;
        st->max_active = std::max(st->max_active, n_act);
        st->min_active = std::min(st->min_active, n_act);
        for (int c = 0; c < n_chunks; ++c, ++L) {
            Clock::time_point avail = avail_at(i, c);
            if (d->pacing == BF_STREAM_PACE_HOST) wait_until(avail);
            wait_completed(L - kInFlight + 1);  // slot k of the state/event rings is free
            if (thread_err.load()) { status = BF_E_DEVICE; break; }
            if (d->pacing == BF_STREAM_PACE_NONE) avail = Clock::now();
            const int k = (int)(L % kInFlight);
            bf::StreamState& hs = h_state[k];
            hs.ring_index = i % d->depth;
            hs.chunk_index = c;
            hs.n_chunks = n_chunks;
            hs.n_active = n_act;
            std::memcpy(hs.slot, act_launch.data(), sizeof(int32_t) * n_act);
            const uint64_t tick = gated ? arrival_tick(i, c) : 0;
            recs[k] = LaunchRec{i, c == n_chunks - 1, avail, tick};
            // the state goes to the device by a copy, or (device-gated) inside the
            // gate kernel, which reads it from the pinned ring entry
            const size_t state_bytes = bf::kStreamStateHeader + sizeof(int32_t) * n_act;
            if ((!gated && (e = hipMemcpyAsync(d_state, &hs, state_bytes, hipMemcpyHostToDevice, s)) !=
                               hipSuccess) ||
                (gated && (e = bf::launch_ingest_gate(tick, gate_ticks, reinterpret_cast<int32_t*>(d_gate),
                                                      reinterpret_cast<const uint32_t*>(d_hstate + k),
                                                      reinterpret_cast<uint32_t*>(d_state),
                                                      (uint32_t)(state_bytes / 4), s)) != hipSuccess) ||
                (e = hipEventRecord(ev_start[k], s)) != hipSuccess ||
                (e = (d->use_graph ? hipGraphLaunch(exec, s) : launch(s))) != hipSuccess ||
                (c == n_chunks - 1 && (n_missing > 0 || d->d_out_valid) &&
                 (e = bf::launch_stream_flags(d_state, d->d_out_ring, d->d_out_valid, S, n_act, s)) !=
                     hipSuccess) ||
                (gated && c == n_chunks - 1 && (e = bf::launch_wall_clock_probe(d_stamp + k, s)) != hipSuccess) ||
                (e = hipEventRecord(ev_end[k], s)) != hipSuccess) {
                status = BF_E_DEVICE;
                break;
            }
            if (c == n_chunks - 1)
                issue_ms[i] = std::chrono::duration<double, std::milli>(Clock::now() - avail).count();
            launched.store(L + 1, std::memory_order_release);
        }
    }
    stop.store(true, std::memory_order_release);
    waiter.join();
    const Clock::time_point t_end = Clock::now();
    if (status == BF_OK && thread_err.load()) {
        status = BF_E_DEVICE;
        e = hipErrorUnknown;
    }
    if (status != BF_OK) return fail("stream launch");
    if (gated) {
        int32_t timed_out = 0;
        if ((e = hipMemcpyAsync(&timed_out, d_gate, sizeof(int32_t), hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return fail("gate status");
        if (timed_out) {
            e = hipErrorLaunchTimeOut;
            return fail("a device-gated wait for a chunk's arrival exceeded gate_timeout_ms");
        }
    }
    if ((e = hipEventRecord(ev_sync, s)) != hipSuccess ||
        (e = hipStreamWaitEvent((hipStream_t)stream, ev_sync, 0)) != hipSuccess)
        return fail("stream ordering");

    // ---- statistics ----
    const double budget_ms = n_time * kSampleS * 1e3;
    st->frames = d->n_frames;
    st->launches = L;
    st->joins = sch.joins;
    st->leaves = sch.leaves;
    st->rejected_joins = sch.rejected;
    st->ignored_events = sch.ignored + (d->n_events - evi);
    if (d->latency_log_ms && !lat_ms.empty())
        std::memcpy(d->latency_log_ms, lat_ms.data(), sizeof(double) * lat_ms.size());
    if (d->service_log_ms && !svc_ms.empty())
        std::memcpy(d->service_log_ms, svc_ms.data(), sizeof(double) * svc_ms.size());
    if (d->issue_log_ms && !issue_ms.empty())
        std::memcpy(d->issue_log_ms, issue_ms.data(), sizeof(double) * issue_ms.size());
    // latency and service statistics over the frames after the warm-up
    lat_ms.erase(lat_ms.begin(), lat_ms.begin() + d->warmup_frames);
    svc_ms.erase(svc_ms.begin(), svc_ms.begin() + d->warmup_frames);
    for (double v : lat_ms) if (v > budget_ms) ++st->late_frames;
    st->latency_p50_ms = quantile(lat_ms, 0.50);
    st->latency_p99_ms = quantile(lat_ms, 0.99);
    st->latency_max_ms = lat_ms.empty() ? 0.0 : *std::max_element(lat_ms.begin(), lat_ms.end());
    double sum = 0.0, ssum = 0.0;
    for (double v : lat_ms) sum += v;
    for (double v : svc_ms) ssum += v;
    st->latency_mean_ms = lat_ms.empty() ? 0.0 : sum / (double)lat_ms.size();
    st->service_mean_ms = svc_ms.empty() ? 0.0 : ssum / (double)svc_ms.size();
    st->service_p99_ms = quantile(svc_ms, 0.99);
    st->wall_s = std::chrono::duration<double>(t_end - t_start).count();
    if (st->wall_s > 0) {
        st->channels_realtime = (double)st->channel_frames / st->wall_s * n_time * kSampleS;
        st->input_gb_s = (double)st->channel_frames * n_time * bf::kInputs / st->wall_s / 1e9;
    }
    cleanup();
    return BF_OK;
}

}  // extern "C"
