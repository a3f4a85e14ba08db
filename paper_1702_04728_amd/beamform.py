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
_PRECISION = {"fp32": FP32_FFT, "fp16": FP16_MFMA, FP32_FFT: FP32_FFT, FP16_MFMA: FP16_MFMA}

N_INPUTS = 2048
N_BEAMS = 1024
N_UPCHAN = 16
N_BEAM_NS = 256

# Every symbol include/beamform.h declares.
EXPORTED = (
    "beamform_default_config", "beamform_compute_lut", "beamform_init", "beamform_frame",
    "beamform_get_lut", "beamform_plan_info", "beamform_destroy", "beamform_strerror",
    "beamform_last_error",
)


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

    def frame(self, raw, out=None, stream=None):
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
        st = self.lib.beamform_frame(self._plan, ctypes.c_void_p(raw.data_ptr()), n_frames,
                                     ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
        _check(st, self._plan)
        return out

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
