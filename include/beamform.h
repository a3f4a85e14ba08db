/*
 * beamform.h -- C ABI of the MI355X hybrid FFT beamformer (libbeamform.so).
 *
 * Implements the CHIME/FRB fan-beam hot path of Ng et al., "CHIME FRB: An
 * application of FFT beamforming for a radio telescope" (arXiv:1702.04728):
 * per frequency channel and per 0.983 ms frame of 384 samples,
 *   - decode 4+4-bit complex voltages of 2048 inputs (Sec. 2, Table 1);
 *   - N-S beams: 256-feed lines zero-padded to 512 and Fourier transformed,
 *     keeping per channel the 256 bins nearest the desired pointings
 *     (Sec. 3.1, Eqs. (1)-(2));
 *   - 4 E-W beams by exact phasing across the 4 cylinders (Sec. 3, Sec. 3.1);
 *   - up-channelisation by a 16-point DFT in time, 390.625 kHz -> 24.4 kHz
 *     (Sec. 3, Sec. 3.2);
 *   - Stokes I (|X|^2 + |Y|^2) integrated over the 24 16-sample blocks of the
 *     frame (Sec. 3, Table 1).
 *
 * Conventions (readings of what the paper leaves open):
 *   input  u8 in[frame][chan][t < n_time][i < 2048], i = (cyl*256+feed)*2+pol,
 *          byte = ((re + 8) << 4) | (im + 8)  (high nibble real);
 *   output f32 out[frame][chan][beam < 1024][q < 16], beam = j*256 + m
 *          (E-W beam j, N-S beam m), sub-channel q holds time-DFT bin
 *          s = (q + 8) mod 16, so q = 8 is the channel centre; no normalisation;
 *   Eq. (1) index k_m = floor(512 f d sin(theta_m) / c + 0.5) mod 512 (FP64);
 *   E-W weight W[j][c] = exp(-2 pi i f x_c sin(phi_j) / c), forward
 *   transforms exp(-2 pi i ...).
 *
 * Memory and ownership: all data pointers passed to beamform_frame are DEVICE
 * pointers owned by the caller; the library never frees them.  Arrays inside
 * bf_config are HOST pointers, copied during beamform_init (the caller may
 * free them afterwards).  The plan owns its device tables; beamform_destroy
 * synchronises the plan's device and frees them.
 *
 * Streams: `stream` arguments are hipStream_t values passed as void* (NULL is
 * the null stream).  Work is enqueued asynchronously; outputs are valid once
 * the stream reaches the enqueued work.
 *
 * Errors: every call returns an int32 status (BF_OK = 0, negative on error).
 * No exception or process exit crosses this interface.  Launch failures are
 * reported by the call that launched; asynchronous device faults surface as
 * BF_E_DEVICE from a later call.  beamform_strerror() gives a static string,
 * beamform_last_error() the plan's last detailed message.  A plan is not
 * thread-safe: use one plan per host thread.
 */
#ifndef BEAMFORM_H
#define BEAMFORM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BF_OK 0
#define BF_E_INVAL (-1)       /* bad argument, size or pointer */
#define BF_E_NOMEM (-2)       /* host or device allocation failed */
#define BF_E_DEVICE (-3)      /* HIP runtime / kernel failure */
#define BF_E_STATE (-4)       /* call not valid for the plan's state */
#define BF_E_UNSUPPORTED (-5) /* valid request the library does not implement */

typedef struct bf_plan bf_plan; /* opaque, library-owned */

/* Arithmetic of the N-S transform.
 *   BF_FP32_FFT:  FP32 radix FFT (the baseline, <= 1e-5 relative power error
 *                 against an FP64 evaluation).
 *   BF_FP16_MFMA: four-step 512 = 32 x 16 DFT on FP16 matrix cores with FP32
 *                 accumulation (<= 2e-3; DFT matrices and the inter-stage data
 *                 carried as FP16 hi + lo pairs, the E-W output rounded once).
 *   BF_FP32_MFMA: the same matrix-core transform with every operand carried as
 *                 FP16 hi + lo (about 22 significant bits): FP32-class error,
 *                 <= 1e-5 like BF_FP32_FFT. */
typedef enum { BF_FP32_FFT = 0, BF_FP16_MFMA = 1, BF_FP32_MFMA = 2 } bf_precision;

typedef struct {
    int32_t n_cyl;      /* cylinders: must be 4 */
    int32_t n_feed;     /* N-S feeds per cylinder (N): must be 256 */
    int32_t n_pol;      /* polarisations: must be 2 */
    int32_t pad;        /* zero-padding factor P: must be 2 (Sec. 3.1) */
    int32_t n_beam_ns;  /* kept N-S beams: must be 256 */
    int32_t n_beam_ew;  /* E-W beams: must be 4 */
    int32_t n_upchan;   /* time-DFT length: must be 16 */
    int32_t n_time;     /* samples per frame: a positive multiple of 16 (384 = 0.983 ms) */
    double feed_spacing_m;      /* N-S feed spacing d (0.3048 m, Sec. 1) */
    double c0;                  /* speed of light in m/s (299792458) */
    const double *cyl_x_m;      /* [n_cyl] E-W cylinder positions; NULL: (c - 1.5) * 20 m */
    const double *sin_theta_ns; /* [n_beam_ns] desired N-S pointings sin(theta_m);
                                   NULL: (m - 127.5) / 128 */
    const double *sin_phi_ew;   /* [n_beam_ew] E-W beam directions sin(phi_j);
                                   NULL: sin((j - 1.5) * 0.4 deg) */
    const int32_t *lut_override;/* [n_chan][n_beam_ns] bins in [0, 512) used instead of
                                   Eq. (1), or NULL */
    int32_t precision;          /* bf_precision */
    int32_t reserved;           /* must be 0 */
} bf_config;

/* Fill *cfg with the defaults above (sizes 4/256/2/2/256/4/16/384, d = 0.3048 m,
 * c0 = 299792458, NULL tables, BF_FP32_FFT).  Host only, no device call. */
int32_t beamform_default_config(bf_config *cfg);

/* Eq. (1)-(2) (Sec. 3.1): the kept FFT bin of every desired N-S pointing for
 * each channel, k_m = floor(N P f d sin(theta_m) / c + 0.5) mod (N P),
 * evaluated in FP64 (or cfg->lut_override copied).  chan_freq_hz: host
 * [n_chan]; out: host int32 [n_chan][n_beam_ns].  Host only, no device call. */
int32_t beamform_compute_lut(const bf_config *cfg, const double *chan_freq_hz,
                             int32_t n_chan, int32_t *out);

/* Create a plan for n_chan channels with centre frequencies chan_freq_hz
 * (host FP64 [n_chan], Hz) on the current HIP device: validates cfg, computes
 * in FP64 the Eq. (1) bin table, the E-W phases W[chan][j][c] and the FFT
 * twiddles, rounds each once to the kernel precision and uploads them on
 * `stream`.  *out_plan is set only on success. */
int32_t beamform_init(const bf_config *cfg, const double *chan_freq_hz, int32_t n_chan,
                      void *stream, bf_plan **out_plan);

/* Beamform n_frames frames of all the plan's channels (the full hot path:
 * decode, N-S beams, E-W beams, 16-point up-channelisation, Stokes I,
 * integration over the frame).
 *   d_in : device u8  [n_frames][n_chan][n_time][2048], 16-byte aligned;
 *   d_out: device f32 [n_frames][n_chan][1024][16], 16-byte aligned, fully
 *          overwritten (no accumulation across calls).
 * n_frames = 0 is a valid no-op.  Asynchronous on `stream`. */
int32_t beamform_frame(bf_plan *plan, const uint8_t *d_in, int32_t n_frames, float *d_out,
                       void *stream);

/* The paper's own up-channelisation (Sec. 3: fine channelisation by 128 times
 * to 3 kHz, Stokes I integrated to 16 sub-channels of 24.4 kHz per 0.983 ms;
 * Sec. 3.2: every 128 samples transformed).  As beamform_frame, with the
 * 16-point DFT of 16-sample blocks replaced by a 128-point DFT of each
 * 128-sample block: fine bin s' (centre-shifted q' = (s' + 64) mod 128) is
 * squared and summed over both pols and the frame's blocks into sub-channel
 * q = ((q' + 4) / 8) mod 16, the 8 fine channels nearest its centre.
 * One pass, still time first: the 128-point DFT of each block runs on the raw
 * samples (16 points over the stride-8 samples, twiddles, 8 points over the
 * sample phase), bin by bin into on-chip slices that then take E-W phasing,
 * the N-S transform and detection in the plan's precision; nothing but the
 * input and the output touches device memory, and the call allocates nothing.
 *   d_in, d_out: as beamform_frame (d_out fully overwritten).
 * Needs n_time % 128 == 0 (else BF_E_UNSUPPORTED). */
int32_t beamform_frame_upchan128(bf_plan *plan, const uint8_t *d_in, int32_t n_frames,
                                 float *d_out, void *stream);

/* Test aid: the complex beams before detection (Sec. 3: the beamforming
 * kernel's output, here already up-channelised) for one frame of every
 * channel: for channel c, 16-sample block b, time-DFT bin s (not centre-
 * shifted), pol p, E-W beam j and N-S beam m,
 *   U = sum_{tau < 16} B[16 b + tau] exp(-2 pi i s tau / 16),
 * B the beam (j, m) of pol p (N-S bin from Eq. (1), E-W exact phasing), in
 * the plan's precision.
 *   d_in:     device u8 [n_chan][n_time][2048] (one frame), 16-byte aligned;
 *   d_ns_out: device f32 [n_chan][n_time / 16][16][2][4][256][2] (re, im),
 *             16-byte aligned, fully overwritten (6.3 MB per channel).
 * Squaring, summing the pols and the blocks and centre-shifting s gives
 * beamform_frame's output. */
int32_t beamform_debug_ns(bf_plan *plan, const uint8_t *d_in, float *d_ns_out, void *stream);

/* 8-bit output (Sec. 3 and Table 1: the integrated Stokes I beams leave the
 * beamformer rescaled to 8-bit integers; the rule is not given, this is an
 * affine rescale per channel, beam and sub-channel).  As beamform_frame, but
 * each integrated power P (FP32, as beamform_frame computes it) is written as
 *   code = min(255, max(0, rint(fmaf(P, scale, offset))))
 * in FP32, rint rounding half to even.
 *   d_scale, d_offset: device f32 [n_chan][1024][16], caller-owned, read only;
 *   d_out: device u8 [n_frames][n_chan][1024][16], 16-byte aligned, fully
 *          overwritten (a quarter of beamform_frame's output bytes).
 * n_frames = 0 is a valid no-op.  Errors: BF_E_INVAL for NULL or misaligned
 * buffers. */
int32_t beamform_frame_u8(bf_plan *plan, const uint8_t *d_in, int32_t n_frames,
                          const float *d_scale, const float *d_offset, uint8_t *d_out,
                          void *stream);

/* Tracking E-W beams (Sec. 3.1: the E-W beams may be static or tracking).  As
 * beamform_frame, with the E-W directions given per frame instead of the
 * plan's static ones:
 *   sin_phi_ew: host FP64 [n_frames][n_beam_ew], sin(phi_j) of each frame.
 * W[frame][chan][j][c] = exp(-2 pi i f_chan x_c sin(phi_{frame,j}) / c) is
 * evaluated on the host in FP64, rounded once to FP32 and uploaded on `stream`
 * into one of two plan-owned device tables used in turn (128 B per
 * channel-frame each, grown when a call needs more: the first calls of a given
 * size allocate); each channel-frame reads its own row.  N-S beams, bins and
 * output layout are those of beamform_frame.  sin_phi_ew is read before the
 * call returns.  A call blocks until the kernel of the call before last has
 * finished (it reuses that call's table), so the host computes one table
 * while the previous kernel runs; calls on one plan must be issued from one
 * host thread.  Errors: BF_E_INVAL
 * (NULL or non-finite sin_phi_ew, bad buffers), BF_E_NOMEM, BF_E_DEVICE. */
int32_t beamform_frame_tracking(bf_plan *plan, const uint8_t *d_in, int32_t n_frames,
                                const double *sin_phi_ew, float *d_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and arguments as beamform_frame_tracking, with results equal to
 * it bit for bit, but the per-channel-frame weight table is a fixed device
 * array of the library (BF_NOALLOC_MAX_ROWS channel-frames, 2 MiB, one per
 * GPU, held until the process ends) and its host staging a fixed host array.
 * The call makes no device or host allocation (the array's device address is
 * looked up once per device by beamform_init).  It uploads the weights on
 * `stream`, launches, and returns once the upload has read the staging table,
 * i.e. after all work enqueued on `stream` before the call has finished.
 * Every call on one GPU shares that GPU's table and keeps it until the next
 * call: calls that overlap on one GPU (other streams, other plans, other host
 * threads) race, so issue them on one stream.
 * Errors: BF_E_INVAL when n_frames x n_chan > BF_NOALLOC_MAX_ROWS and for the
 * arguments beamform_frame_tracking rejects; BF_E_DEVICE. */
#define BF_NOALLOC_MAX_ROWS 16384
int32_t beamform_frame_tracking_noalloc(bf_plan *plan, const uint8_t *d_in, int32_t n_frames,
                                        const double *sin_phi_ew, float *d_out, void *stream);

/* ---------------------------------------------------------------------------
 * Streaming (serving) loop.  Frames of 0.983 ms arrive for a varying set of
 * channels (channels join and leave); each launch beamforms the active
 * channels' newest chunk straight from a device input ring into a device
 * output ring.  Per-bin partial integrations of a frame stay in HBM between
 * chunks; a captured hipGraph is replayed per launch; frame latency is measured
 * against each frame's availability time.  Paper Sec. 2 (one channel per GPU
 * stream of 2.56 us samples), Sec. 3 (0.983 ms integration), Table 1.
 * ------------------------------------------------------------------------- */

#define BF_STREAM_JOIN 1
#define BF_STREAM_LEAVE 2
#define BF_STREAM_MAX_SLOTS 1024
#define BF_STREAM_PACE_NONE 0
#define BF_STREAM_PACE_HOST 1
#define BF_STREAM_PACE_GATED 2
#define BF_STREAM_RUN_AHEAD 48 /* launches queued and not yet completed, at most (16 frames
                                  of 128-sample chunks) */

typedef struct {
    int32_t frame;       /* applied before frame `frame` is processed */
    int32_t op;          /* BF_STREAM_JOIN or BF_STREAM_LEAVE */
    int32_t channel_id;  /* caller's channel identifier */
    int32_t reserved;    /* must be 0 */
    double freq_hz;      /* centre frequency (JOIN only) */
} bf_stream_event;

typedef struct {
    const uint8_t *d_in_ring; /* device u8 [depth][max_slots][n_time][2048]: frame i of the
                                 channel in slot s is read from entry (i mod depth, s) */
    float *d_out_ring;        /* device f32 [depth][max_slots][1024][16]: result of frame i,
                                 slot s, written to entry (i mod depth, s) */
    int32_t depth;            /* ring entries (>= 1) */
    int32_t max_slots;        /* channel slots, 1 .. BF_STREAM_MAX_SLOTS */
    int32_t n_frames;         /* frames to run (>= 0) */
    int32_t chunk;            /* samples per launch: a multiple of 16 dividing n_time
                                 (0 = n_time, whole frames) */
    int32_t pacing;           /* BF_STREAM_PACE_*: 0 launch as fast as possible; 1 real
                                 time, host-paced: chunk c of frame i becomes available at
                                 t0 + (i n_time + (c+1) chunk) x 2.56 us and the host
                                 launches it then; 2 real time, device-gated: the same
                                 availability times, kept on the device's constant-rate
                                 wall clock (aligned to the host clock at start, a gate
                                 opening at most one probe round trip late, never early):
                                 the host queues launches ahead of their data (up to
                                 BF_STREAM_RUN_AHEAD launches not yet completed) and a
                                 one-wave kernel in front of each holds the stream until
                                 its chunk's availability, so a host or HIP-runtime stall
                                 shorter than the queued work delays no frame */
    int32_t use_graph;        /* 1: replay one captured hipGraph per launch; 0: plain launches */
    int64_t mem_cap_bytes;    /* device bytes the stream may use for channel state and its
                                 share of the rings (0: free memory at start); a JOIN that
                                 would exceed it, or find no free slot, is rejected (a JOIN
                                 of an active id, or with a frequency whose Eq. (1) bins
                                 cannot be formed, is ignored) */
    const bf_stream_event *events; /* host, sorted by frame; may be NULL if n_events = 0 */
    int32_t n_events;
    int32_t warmup_frames;         /* frames at the start left out of the latency, late-frame
                                      and service statistics (0 .. n_frames) */
    int32_t *slot_log;        /* optional host int32 [n_frames][max_slots]: channel id held
                                 by each slot during each frame, -1 when empty */
    const uint8_t *ingest_ok; /* optional host u8 [n_frames][max_slots], set by the ingest
                                 (the paper's data arrive over lossy links): nonzero when
                                 frame i of slot s arrived complete by its availability
                                 time; read when the frame's first chunk is launched
                                 (queued, with device-gated pacing).  A
                                 zero (empty or late ring entry) skips that channel-frame:
                                 its output entry is written as zeros, flagged invalid in
                                 d_out_valid and counted in missing_frames.  NULL: every
                                 frame arrived */
    uint8_t *d_out_valid;     /* optional device u8 [depth][max_slots]: written with the
                                 output entry of every active slot, 1 = beamformed,
                                 0 = zeros for a missing frame */
    double *latency_log_ms;   /* optional host [n_frames]: each frame's latency in ms
                                 (warm-up frames included), filled before returning */
    double *service_log_ms;   /* optional host [n_frames]: device time of each frame's
                                 launches in ms (event to event), filled before returning */
    double *issue_log_ms;     /* optional host [n_frames]: host time at which each frame's
                                 last launch had been issued, minus the availability of
                                 its last chunk, in ms (with pacing: how late the host
                                 issued it; a latency well above the service time with a
                                 small issue lag means the frame queued behind earlier
                                 ones on the device; negative: queued ahead of its data,
                                 device-gated pacing), filled before returning */
    int32_t gate_timeout_ms;  /* device-gated pacing: longest wait of one gate for its
                                 chunk's arrival (a bound on the device-side wait) before
                                 the loop fails with BF_E_DEVICE; 0 = 1000 ms plus two
                                 chunk periods */
    int32_t reserved2;        /* must be 0 */
} bf_stream_desc;

typedef struct {
    int64_t frames;           /* frames run */
    int64_t launches;         /* kernel launches (frames x chunks) */
    int64_t channel_frames;   /* sum over frames of active channels */
    int64_t late_frames;      /* frames whose latency exceeded n_time x 2.56 us (latency,
                                 late-frame and service figures cover the frames after
                                 desc->warmup_frames; the counts cover every frame) */
    int64_t joins, leaves, rejected_joins, ignored_events;
    int32_t max_active, min_active;
    double latency_p50_ms, latency_p99_ms, latency_max_ms, latency_mean_ms;
    double service_mean_ms, service_p99_ms; /* device time of a frame's launches */
    double wall_s;
    double channels_realtime;  /* channel_frames / wall_s x n_time x 2.56 us */
    double input_gb_s;         /* channel_frames x n_time x 2048 B / wall_s */
    int64_t per_slot_bytes;    /* device bytes one active channel costs */
    int32_t slot_capacity;     /* slots admissible under mem_cap_bytes */
    int32_t reserved;
    int64_t missing_frames;    /* active channel-frames skipped (ingest_ok zero), output
                                  zeroed and flagged; all frames, warm-up included */
} bf_stream_stats;

/* Run the serving loop on the plan's geometry and precision (the plan's own
 * channel list is not used; channels come from JOIN events).  Frame i:
 * apply its events; (host-paced) wait for each chunk's availability, or
 * (device-gated) queue a wait for it on the device; launch the beamformer for
 * every active slot; the last chunk writes the frame's output.  Latency of
 * frame i = time its last launch completes - availability of its last chunk
 * (host steady clock).  Blocks until all frames completed; `stream` is
 * synchronised with before the first launch and after the last.  Library
 * state (slot tables, partial accumulators, graph, the receiver's pinned
 * words and thread) is allocated at start and freed before returning.
 * Errors: BF_E_INVAL for a bad descriptor, BF_E_DEVICE for HIP failures and
 * for a device-gated wait that exceeded gate_timeout_ms. */
int32_t beamform_stream(bf_plan *plan, const bf_stream_desc *desc, bf_stream_stats *stats,
                        void *stream);

/* The loop's host scheduler alone, without a device (test aid): applies the
 * events frame by frame with the admission rule of beamform_stream, given the
 * per-slot byte cost and the byte cap, and fills stats (joins, leaves,
 * rejections, active counts, channel_frames) and desc->slot_log.  Launches
 * nothing; desc device pointers are ignored. */
int32_t beamform_stream_schedule(const bf_stream_desc *desc, int64_t per_slot_bytes,
                                 int64_t cap_bytes, bf_stream_stats *stats);

/* Copy the plan's bin table to host int32 [n_chan][n_beam_ns] (synchronous). */
int32_t beamform_get_lut(const bf_plan *plan, int32_t *host_out);

/* Number of channels and samples per frame of a plan. */
int32_t beamform_plan_info(const bf_plan *plan, int32_t *n_chan, int32_t *n_time,
                           int32_t *precision);

/* Synchronise the plan's device, free its tables and the plan.  NULL is a no-op. */
int32_t beamform_destroy(bf_plan *plan);

/* Static description of a status code. */
const char *beamform_strerror(int32_t status);

/* The plan's last error message ("" if none); NULL plan: the last error of a
 * failed beamform_init on this thread. */
const char *beamform_last_error(const bf_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* BEAMFORM_H */
