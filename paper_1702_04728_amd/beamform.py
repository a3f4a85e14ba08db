"""ctypes binding over libbeamform.so (argument marshalling only).

Every step of the hot path runs in the library's HIP kernels.  PyTorch is
used only for device memory (tensors whose data pointers are passed through)
and for the current HIP stream.  If the library is not built this module
raises; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbeamform.so")

BF_OK = 0
FP32_FFT = 0
FP16_MFMA = 1
FP32_MFMA = 2
_PRECISION = {"fp32": FP32_FFT, "fp16": FP16_MFMA, "fp32_mfma": FP32_MFMA,
              FP32_FFT: FP32_FFT, FP16_MFMA: FP16_MFMA, FP32_MFMA: FP32_MFMA}

N_INPUTS = 2048
PACING = {"none": 0, "host": 1, "gated": 2}  # bf_stream_desc.pacing
N_BEAMS = 1024
N_UPCHAN = 16
N_BEAM_NS = 256

# Every symbol include/beamform.h declares.
EXPORTED = (
    "beamform_default_config", "beamform_compute_lut", "beamform_init", "beamform_frame",
    "beamform_frame_upchan128", "beamform_frame_u8", "beamform_frame_tracking",
    "beamform_frame_tracking_noalloc", "beamform_debug_ns",
    "beamform_stream", "beamform_stream_schedule", "beamform_get_lut", "beamform_plan_info",
    "beamform_destroy", "beamform_strerror", "beamform_last_error",
)

STREAM_JOIN = 1
STREAM_LEAVE = 2
STREAM_MAX_SLOTS = 1024


class BeamformError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (_strerror(status), status, msg))
        self.status = status


class BfConfig(ctypes.Structure):
    _fields_ = [
        ("n_cyl", ctypes.c_int32), ("n_feed", ctypes.c_int32), ("n_pol", ctypes.c_int32),
        ("pad", ctypes.c_int32), ("n_beam_ns", ctypes.c_int32), ("n_beam_ew", ctypes.c_int32),
        ("n_upchan", ctypes.c_int32), ("n_time", ctypes.c_int32),
        ("feed_spacing_m", ctypes.c_double), ("c0", ctypes.c_double),
        ("cyl_x_m", ctypes.POINTER(ctypes.c_double)),
        ("sin_theta_ns", ctypes.POINTER(ctypes.c_double)),
        ("sin_phi_ew", ctypes.POINTER(ctypes.c_double)),
        ("lut_override", ctypes.POINTER(ctypes.c_int32)),
        ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class BfStreamEvent(ctypes.Structure):
    _fields_ = [("frame", ctypes.c_int32), ("op", ctypes.c_int32),
                ("channel_id", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("freq_hz", ctypes.c_double)]


class BfStreamDesc(ctypes.Structure):
    _fields_ = [("d_in_ring", ctypes.c_void_p), ("d_out_ring", ctypes.c_void_p),
                ("depth", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("n_frames", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("pacing", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("mem_cap_bytes", ctypes.c_int64),
                ("events", ctypes.POINTER(BfStreamEvent)), ("n_events", ctypes.c_int32),
                ("warmup_frames", ctypes.c_int32),
                ("slot_log", ctypes.POINTER(ctypes.c_int32)),
                ("ingest_ok", ctypes.POINTER(ctypes.c_uint8)),
                ("d_out_valid", ctypes.c_void_p),
                ("latency_log_ms", ctypes.POINTER(ctypes.c_double)),
                ("service_log_ms", ctypes.POINTER(ctypes.c_double)),
                ("issue_log_ms", ctypes.POINTER(ctypes.c_double)),
                ("gate_timeout_ms", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


class BfStreamStats(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("channel_frames", ctypes.c_int64), ("late_frames", ctypes.c_int64),
                ("joins", ctypes.c_int64), ("leaves", ctypes.c_int64),
                ("rejected_joins", ctypes.c_int64), ("ignored_events", ctypes.c_int64),
                ("max_active", ctypes.c_int32), ("min_active", ctypes.c_int32),
                ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("latency_max_ms", ctypes.c_double), ("latency_mean_ms", ctypes.c_double),
                ("service_mean_ms", ctypes.c_double), ("service_p99_ms", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("channels_realtime", ctypes.c_double),
                ("input_gb_s", ctypes.c_double), ("per_slot_bytes", ctypes.c_int64),
                ("slot_capacity", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("missing_frames", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


def _events_array(events):
    """events: iterable of (frame, op, channel_id, freq_hz), sorted by frame."""
    ev = list(events)
    arr = (BfStreamEvent * max(1, len(ev)))()
    for i, (fr, op, cid, f) in enumerate(ev):
        arr[i] = BfStreamEvent(int(fr), int(op), int(cid), 0, float(f))
    return arr, len(ev)


def _pacing(p):
    """pacing as False/True (none/host-paced), "none"/"host"/"gated", or the C value."""
    if isinstance(p, str):
        if p not in PACING:
            raise ValueError("pacing must be one of %s" % sorted(PACING))
        return PACING[p]
    return int(p)


def _stream_desc(depth, max_slots, n_frames, chunk, pacing, use_graph, mem_cap_bytes, events,
                 slot_log, d_in=None, d_out=None, warmup_frames=0, ingest_ok=None,
                 d_out_valid=None):
    arr, n_ev = _events_array(events)
    d = BfStreamDesc()
    d.d_in_ring = d_in
    d.d_out_ring = d_out
    d.depth, d.max_slots, d.n_frames, d.chunk = int(depth), int(max_slots), int(n_frames), int(chunk)
    d.pacing, d.use_graph, d.mem_cap_bytes = _pacing(pacing), int(use_graph), int(mem_cap_bytes)
    d.events = arr
    d.n_events = n_ev
    d.warmup_frames = int(warmup_frames)
    if slot_log is not None:
        d.slot_log = slot_log.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    keep = [arr]
    if ingest_ok is not None:
        ok = np.ascontiguousarray(ingest_ok, dtype=np.uint8)
        if ok.shape != (n_frames, max_slots):
            raise ValueError("ingest_ok must be [n_frames][max_slots] = %s, got %s"
                             % ((n_frames, max_slots), ok.shape))
        keep.append(ok)
        d.ingest_ok = ok.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    d.d_out_valid = d_out_valid
    return d, keep


def stream_schedule(events, n_frames, max_slots, per_slot_bytes, cap_bytes, depth=1,
                    warmup_frames=0, ingest_ok=None, pacing=0, gate_timeout_ms=0):
    """Host-only dry run of the serving loop's scheduler: (stats dict, slot_log).  The
    descriptor (pacing and gate_timeout_ms included) is validated as beamform_stream
    validates it."""
    lib = load_library()
    log = np.full((n_frames, max_slots), -1, dtype=np.int32)
    d, keep = _stream_desc(depth, max_slots, n_frames, 0, pacing, 0, 0, events, log,
                           warmup_frames=warmup_frames, ingest_ok=ingest_ok)
    d.gate_timeout_ms = int(gate_timeout_ms)
    st = BfStreamStats()
    _check(lib.beamform_stream_schedule(ctypes.byref(d), int(per_slot_bytes), int(cap_bytes),
                                        ctypes.byref(st)))
    del keep
    return st.as_dict(), log


_lib = None


def load_library():
    """Load libbeamform.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbeamform.so is not built (run paper_1702_04728_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    cp = ctypes.POINTER(BfConfig)
    sig = {
        "beamform_default_config": ([cp], i32),
        "beamform_compute_lut": ([cp, vp, i32, vp], i32),
        "beamform_init": ([cp, vp, i32, vp, ctypes.POINTER(vp)], i32),
        "beamform_frame": ([vp, vp, i32, vp, vp], i32),
        "beamform_frame_tracking": ([vp, vp, i32, vp, vp, vp], i32),
        "beamform_frame_tracking_noalloc": ([vp, vp, i32, vp, vp, vp], i32),
        "beamform_frame_u8": ([vp, vp, i32, vp, vp, vp, vp], i32),
        "beamform_frame_upchan128": ([vp, vp, i32, vp, vp], i32),
        "beamform_debug_ns": ([vp, vp, vp, vp], i32),
        "beamform_stream": ([vp, ctypes.POINTER(BfStreamDesc), ctypes.POINTER(BfStreamStats), vp],
                            i32),
        "beamform_stream_schedule": ([ctypes.POINTER(BfStreamDesc), ctypes.c_int64,
                                      ctypes.c_int64, ctypes.POINTER(BfStreamStats)], i32),
        "beamform_get_lut": ([vp, vp], i32),
        "beamform_plan_info": ([vp, vp, vp, vp], i32),
        "beamform_destroy": ([vp], i32),
        "beamform_strerror": ([i32], ctypes.c_char_p),
        "beamform_last_error": ([vp], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _strerror(status: int) -> str:
    try:
        return load_library().beamform_strerror(status).decode()
    except Exception:
        return "status"


def _check(status: int, plan=None):
    if status != BF_OK:
        msg = load_library().beamform_last_error(plan).decode()
        raise BeamformError(status, msg)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _Config:
    """BfConfig plus the host arrays it points at (kept alive together)."""

    def __init__(self, n_time=384, precision="fp32", sin_theta_ns=None, sin_phi_ew=None,
                 cyl_x_m=None, lut_override=None, feed_spacing_m=None, c0=None):
        lib = load_library()
        self.c = BfConfig()
        _check(lib.beamform_default_config(ctypes.byref(self.c)))
        self.c.n_time = int(n_time)
        self.c.precision = _PRECISION[precision]
        if feed_spacing_m is not None:
            self.c.feed_spacing_m = float(feed_spacing_m)
        if c0 is not None:
            self.c.c0 = float(c0)
        self._keep = []
        if sin_theta_ns is not None:
            a = np.ascontiguousarray(sin_theta_ns, dtype=np.float64)
            assert a.shape == (N_BEAM_NS,)
            self._keep.append(a)
            self.c.sin_theta_ns = _dptr(a)
        if sin_phi_ew is not None:
            a = np.ascontiguousarray(sin_phi_ew, dtype=np.float64)
            assert a.shape == (4,)
            self._keep.append(a)
            self.c.sin_phi_ew = _dptr(a)
        if cyl_x_m is not None:
            a = np.ascontiguousarray(cyl_x_m, dtype=np.float64)
            assert a.shape == (4,)
            self._keep.append(a)
            self.c.cyl_x_m = _dptr(a)
        if lut_override is not None:
            a = np.ascontiguousarray(lut_override, dtype=np.int32)
            self._keep.append(a)
            self.c.lut_override = a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def compute_lut(freqs_hz, **cfg) -> np.ndarray:
    """Host-only Eq. (1) bin table [n_chan][256] as the library computes it."""
    lib = load_library()
    f = np.ascontiguousarray(freqs_hz, dtype=np.float64)
    c = _Config(**cfg)
    out = np.empty((f.size, N_BEAM_NS), dtype=np.int32)
    _check(lib.beamform_compute_lut(ctypes.byref(c.c), ctypes.c_void_p(f.ctypes.data), f.size,
                                    ctypes.c_void_p(out.ctypes.data)))
    return out


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Beamformer:
    """One plan: a fixed set of channels (centre frequencies in Hz) on the current device.

    ``frame(raw, out)`` beamforms raw u8 [n_frames][n_chan][n_time][2048] into f32
    [n_frames][n_chan][1024][16] on the current stream (both CUDA tensors).
    """

    def __init__(self, freqs_hz, precision="fp32", n_time=384, sin_theta_ns=None,
                 sin_phi_ew=None, cyl_x_m=None, lut_override=None, feed_spacing_m=None,
                 c0=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Beamformer needs a GPU")
        self.lib = load_library()
        self.freqs = np.ascontiguousarray(freqs_hz, dtype=np.float64).reshape(-1)
        self.n_chan = int(self.freqs.size)
        self.n_time = int(n_time)
        self.precision = precision
        self.device = torch.cuda.current_device()
        cfg = _Config(n_time, precision, sin_theta_ns, sin_phi_ew, cyl_x_m, lut_override,
                      feed_spacing_m, c0)
        plan = ctypes.c_void_p()
        st = self.lib.beamform_init(ctypes.byref(cfg.c), ctypes.c_void_p(self.freqs.ctypes.data),
                                    self.n_chan, _stream_handle(stream), ctypes.byref(plan))
        _check(st, None)
        self._plan = plan

    def out_shape(self, n_frames: int):
        return (n_frames, self.n_chan, N_BEAMS, N_UPCHAN)

    def frame(self, raw, out=None, stream=None, sin_phi_ew=None, upchan=16, noalloc=False):
        """Beamform raw [n_frames][n_chan][n_time][2048] (CUDA uint8) into out
        [n_frames][n_chan][1024][16] (CUDA float32).  sin_phi_ew: None for the plan's
        static E-W beams, or [n_frames][4] E-W directions per frame (tracking beams).
        upchan: 16 (16-point DFT of 16-sample blocks) or 128 (the 128-point
        up-channelisation integrated to the same 16 sub-channels).  noalloc (tracking
        beams only): use the entry point whose weight table is the library's fixed
        device array (no allocation in the call)."""
        import torch
        if self._plan is None:
            raise BeamformError(-4, "plan destroyed")
        if not (isinstance(raw, torch.Tensor) and raw.is_cuda and raw.dtype == torch.uint8):
            raise TypeError("raw must be a CUDA uint8 tensor")
        if raw.dim() != 4 or raw.shape[1:] != (self.n_chan, self.n_time, N_INPUTS):
            raise ValueError("raw must be [n_frames][%d][%d][%d], got %s"
                             % (self.n_chan, self.n_time, N_INPUTS, tuple(raw.shape)))
        if not raw.is_contiguous():
            raise ValueError("raw must be contiguous")
        n_frames = int(raw.shape[0])
        if out is None:
            out = torch.empty(self.out_shape(n_frames), dtype=torch.float32, device=raw.device)
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float32
                and out.is_contiguous() and tuple(out.shape) == self.out_shape(n_frames)):
            raise ValueError("out must be a contiguous CUDA float32 tensor of shape %s"
                             % (self.out_shape(n_frames),))
        if upchan not in (16, 128):
            raise ValueError("upchan must be 16 or 128")
        if noalloc and sin_phi_ew is None:
            raise ValueError("noalloc applies to tracking beams (sin_phi_ew)")
        if upchan == 128:
            if sin_phi_ew is not None:
                raise ValueError("tracking beams use the 16-point up-channelisation")
            st = self.lib.beamform_frame_upchan128(self._plan, ctypes.c_void_p(raw.data_ptr()),
                                                   n_frames, ctypes.c_void_p(out.data_ptr()),
                                                   _stream_handle(stream))
        elif sin_phi_ew is None:
            st = self.lib.beamform_frame(self._plan, ctypes.c_void_p(raw.data_ptr()), n_frames,
                                         ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
        else:
            phi = np.ascontiguousarray(sin_phi_ew, dtype=np.float64)
            if phi.shape != (n_frames, 4):
                raise ValueError("sin_phi_ew must be [n_frames][4], got %s" % (phi.shape,))
            fn = (self.lib.beamform_frame_tracking_noalloc if noalloc
                  else self.lib.beamform_frame_tracking)
            st = fn(self._plan, ctypes.c_void_p(raw.data_ptr()), n_frames,
                ctypes.c_void_p(phi.ctypes.data), ctypes.c_void_p(out.data_ptr()),
                _stream_handle(stream))
        _check(st, self._plan)
        return out

    def debug_ns(self, raw, stream=None):
        """Test aid: complex beams before detection for one frame, raw CUDA uint8
        [n_chan][n_time][2048] -> CUDA complex64 [n_chan][n_time/16][16 (bin s,
        not centre-shifted)][2 pols][4 E-W][256 N-S]."""
        import torch
        if self._plan is None:
            raise BeamformError(-4, "plan destroyed")
        if not (isinstance(raw, torch.Tensor) and raw.is_cuda and raw.dtype == torch.uint8
                and raw.is_contiguous() and tuple(raw.shape) == (self.n_chan, self.n_time, N_INPUTS)):
            raise ValueError("raw must be a contiguous CUDA uint8 [%d][%d][%d]"
                             % (self.n_chan, self.n_time, N_INPUTS))
        out = torch.empty((self.n_chan, self.n_time // 16, 16, 2, 4, N_BEAM_NS, 2),
                          dtype=torch.float32, device=raw.device)
        st = self.lib.beamform_debug_ns(self._plan, ctypes.c_void_p(raw.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
        _check(st, self._plan)
        return torch.view_as_complex(out)

    def frame_u8(self, raw, scale, offset, out=None, stream=None):
        """8-bit output: code = clamp(rint(P * scale + offset), 0, 255) per output,
        scale/offset CUDA float32 [n_chan][1024][16]; returns CUDA uint8
        [n_frames][n_chan][1024][16]."""
        import torch
        if self._plan is None:
            raise BeamformError(-4, "plan destroyed")
        if not (isinstance(raw, torch.Tensor) and raw.is_cuda and raw.dtype == torch.uint8
                and raw.is_contiguous() and raw.dim() == 4
                and raw.shape[1:] == (self.n_chan, self.n_time, N_INPUTS)):
            raise ValueError("raw must be a contiguous CUDA uint8 [n_frames][%d][%d][%d]"
                             % (self.n_chan, self.n_time, N_INPUTS))
        tab = (self.n_chan, N_BEAMS, N_UPCHAN)
        for name, x in (("scale", scale), ("offset", offset)):
            if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32
                    and x.is_contiguous() and tuple(x.shape) == tab):
                raise ValueError("%s must be a contiguous CUDA float32 tensor of shape %s"
                                 % (name, tab))
        n_frames = int(raw.shape[0])
        shape = self.out_shape(n_frames)
        if out is None:
            out = torch.empty(shape, dtype=torch.uint8, device=raw.device)
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.uint8
                and out.is_contiguous() and tuple(out.shape) == shape):
            raise ValueError("out must be a contiguous CUDA uint8 tensor of shape %s" % (shape,))
        st = self.lib.beamform_frame_u8(self._plan, ctypes.c_void_p(raw.data_ptr()), n_frames,
                                        ctypes.c_void_p(scale.data_ptr()),
                                        ctypes.c_void_p(offset.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
        _check(st, self._plan)
        return out

    def stream(self, in_ring, out_ring, events, n_frames, chunk=0, pacing=False, use_graph=True,
               mem_cap_bytes=0, stream=None, log_slots=True, warmup_frames=0, ingest_ok=None,
               out_valid=None, latency_log=None, service_log=None, issue_log=None,
               gate_timeout_ms=0):
        """Run the serving loop (blocking).  in_ring: CUDA uint8 [depth][max_slots][n_time][2048];
        out_ring: CUDA float32 [depth][max_slots][1024][16]; events: (frame, op, channel_id,
        freq_hz) tuples sorted by frame; pacing: False / "none" (as fast as possible),
        True / "host" (host-paced real time) or "gated" (device-gated real time: launches
        queued ahead of their data and held on the device clock until it arrives,
        gate_timeout_ms bounding one wait, 0 = 1 s plus two chunk periods);
        latency and service statistics leave out the first
        warmup_frames frames.  ingest_ok: host uint8 [n_frames][max_slots], 0 where a
        channel-frame did not arrive (its output is zeroed and flagged); out_valid: CUDA
        uint8 [depth][max_slots] receiving those flags; latency_log: host float64
        [n_frames] receiving each frame's latency in ms; service_log, issue_log: the same
        for each frame's device time and for how late its last launch was issued after
        its availability.  Returns (stats dict, slot_log [n_frames][max_slots])."""
        import torch
        if not (isinstance(in_ring, torch.Tensor) and in_ring.is_cuda and in_ring.dtype == torch.uint8
                and in_ring.is_contiguous() and in_ring.dim() == 4
                and tuple(in_ring.shape[2:]) == (self.n_time, N_INPUTS)):
            raise ValueError("in_ring must be a contiguous CUDA uint8 [depth][slots][%d][%d]"
                             % (self.n_time, N_INPUTS))
        depth, max_slots = int(in_ring.shape[0]), int(in_ring.shape[1])
        if not (isinstance(out_ring, torch.Tensor) and out_ring.is_cuda
                and out_ring.dtype == torch.float32 and out_ring.is_contiguous()
                and tuple(out_ring.shape) == (depth, max_slots, N_BEAMS, N_UPCHAN)):
            raise ValueError("out_ring must be a contiguous CUDA float32 [%d][%d][%d][%d]"
                             % (depth, max_slots, N_BEAMS, N_UPCHAN))
        if out_valid is not None and not (
                isinstance(out_valid, torch.Tensor) and out_valid.is_cuda
                and out_valid.dtype == torch.uint8 and out_valid.is_contiguous()
                and tuple(out_valid.shape) == (depth, max_slots)):
            raise ValueError("out_valid must be a contiguous CUDA uint8 [%d][%d]"
                             % (depth, max_slots))
        log = np.full((n_frames, max_slots), -1, dtype=np.int32) if log_slots else None
        d, keep = _stream_desc(depth, max_slots, n_frames, chunk, pacing, use_graph,
                               mem_cap_bytes, events, log, ctypes.c_void_p(in_ring.data_ptr()),
                               ctypes.c_void_p(out_ring.data_ptr()), warmup_frames, ingest_ok,
                               ctypes.c_void_p(out_valid.data_ptr()) if out_valid is not None
                               else None)
        for name, arr in (("latency_log", latency_log), ("service_log", service_log),
                          ("issue_log", issue_log)):
            if arr is None:
                continue
            if not (isinstance(arr, np.ndarray) and arr.dtype == np.float64
                    and arr.flags.c_contiguous and arr.shape == (n_frames,)):
                raise ValueError("%s must be a contiguous float64 array [%d]" % (name, n_frames))
            setattr(d, name + "_ms", arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        d.gate_timeout_ms = int(gate_timeout_ms)
        st = BfStreamStats()
        rc = self.lib.beamform_stream(self._plan, ctypes.byref(d), ctypes.byref(st),
                                      _stream_handle(stream))
        del keep
        _check(rc, self._plan)
        return st.as_dict(), log

    def lut(self) -> np.ndarray:
        out = np.empty((self.n_chan, N_BEAM_NS), dtype=np.int32)
        _check(self.lib.beamform_get_lut(self._plan, ctypes.c_void_p(out.ctypes.data)), self._plan)
        return out

    def close(self):
        if getattr(self, "_plan", None) is not None:
            st = self.lib.beamform_destroy(self._plan)
            self._plan = None
            _check(st)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
