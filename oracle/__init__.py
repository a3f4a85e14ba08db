"""FP64 CPU oracle for the hybrid FFT beamformer -- TEST INFRASTRUCTURE ONLY.

Thin ctypes binding over ``oracle.c`` (plain C, FP64, OpenMP over channel-
frames).  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never imports, links or
calls anything here, and this package imports nothing from the library.

The paper (Ng et al., arXiv:1702.04728) fixes what is computed: Sec. 2 and
Table 1 (inputs), Sec. 3 (kernel order, Stokes I, integration), Sec. 3.1 with
Eqs. (1)-(2) (zero-padded N-S FFT beams clamped to the desired pointings,
static E-W beams by exact phasing), Sec. 3.2 (up-channelisation).  The
conventions it leaves open are the ones documented in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Instrument constants (Sec. 1: 256 feeds per cylinder at 0.3048 m, four
# cylinders 20 m wide; Sec. 3.1: N = 256, P = 2).
C0 = 299_792_458.0
FEED_SPACING_M = 0.3048
CYL_SPACING_M = 20.0


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [
        ("n_feed", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("n_cyl", ctypes.c_int32), ("n_pol", ctypes.c_int32),
        ("n_beam_ns", ctypes.c_int32), ("n_beam_ew", ctypes.c_int32),
        ("n_dft", ctypes.c_int32), ("n_time", ctypes.c_int32),
        ("feed_spacing_m", ctypes.c_double), ("c0", ctypes.c_double),
        ("cyl_x_m", ctypes.POINTER(ctypes.c_double)),
        ("sin_theta_ns", ctypes.POINTER(ctypes.c_double)),
        ("sin_phi_ew", ctypes.POINTER(ctypes.c_double)),
    ]


def default_sin_theta(n_beam_ns: int = 256) -> np.ndarray:
    """Desired N-S pointings, uniform in sin(theta) over the whole N-S sky.

    Sec. 3.1 asks for 256 desired pointings with a tunable tiling but gives no
    values; this reading spaces them uniformly in sin(theta) across [-1, 1].
    """
    m = np.arange(n_beam_ns, dtype=np.float64)
    return (m - (n_beam_ns - 1) / 2.0) / (n_beam_ns / 2.0)


def default_sin_phi(n_beam_ew: int = 4) -> np.ndarray:
    """Static E-W beams 0.4 deg apart, centred on the meridian (Sec. 3.1)."""
    j = np.arange(n_beam_ew, dtype=np.float64)
    return np.sin(np.deg2rad((j - (n_beam_ew - 1) / 2.0) * 0.4))


@dataclass
class Geometry:
    n_feed: int = 256
    pad: int = 2
    n_cyl: int = 4
    n_pol: int = 2
    n_beam_ns: int = 256
    n_beam_ew: int = 4
    n_dft: int = 16
    n_time: int = 384
    feed_spacing_m: float = FEED_SPACING_M
    c0: float = C0
    cyl_x_m: np.ndarray | None = None
    sin_theta_ns: np.ndarray | None = None
    sin_phi_ew: np.ndarray | None = None
    _keep: list = field(default_factory=list, repr=False)

    def __post_init__(self):
        if self.cyl_x_m is None:
            self.cyl_x_m = (np.arange(self.n_cyl) - (self.n_cyl - 1) / 2.0) * CYL_SPACING_M
        if self.sin_theta_ns is None:
            self.sin_theta_ns = default_sin_theta(self.n_beam_ns)
        if self.sin_phi_ew is None:
            self.sin_phi_ew = default_sin_phi(self.n_beam_ew)
        self.cyl_x_m = np.ascontiguousarray(self.cyl_x_m, dtype=np.float64)
        self.sin_theta_ns = np.ascontiguousarray(self.sin_theta_ns, dtype=np.float64)
        self.sin_phi_ew = np.ascontiguousarray(self.sin_phi_ew, dtype=np.float64)
        assert self.cyl_x_m.shape == (self.n_cyl,)
        assert self.sin_theta_ns.shape == (self.n_beam_ns,)
        assert self.sin_phi_ew.shape == (self.n_beam_ew,)

    @property
    def n_inputs(self) -> int:
        return self.n_cyl * self.n_feed * self.n_pol

    @property
    def n_beams(self) -> int:
        return self.n_beam_ew * self.n_beam_ns

    def _c(self) -> _Geom:
        dp = ctypes.POINTER(ctypes.c_double)
        return _Geom(self.n_feed, self.pad, self.n_cyl, self.n_pol, self.n_beam_ns,
                     self.n_beam_ew, self.n_dft, self.n_time, self.feed_spacing_m, self.c0,
                     self.cyl_x_m.ctypes.data_as(dp), self.sin_theta_ns.ctypes.data_as(dp),
                     self.sin_phi_ew.ctypes.data_as(dp))


_lib = None


def build_variant(src_text: str, out_path: str, extra_flags=()) -> str:
    """Compile another oracle source (e.g. a deliberately broken copy used to check
    that the pins detect mistakes, or the oracle itself with sanitizer flags) into
    out_path."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared"]
                          + list(extra_flags) + ["-o", out_path, src, "-lm"])
    return out_path


class use_library:
    """Context manager: route every oracle call through the library at `path`."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _bind(ctypes.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved


def _load():
    """The oracle library: liboracle.so, or the build named by ORACLE_LIB (a
    sanitizer build of the same source, for the CPU hygiene runs)."""
    global _lib
    if _lib is None:
        alt = os.environ.get("ORACLE_LIB")
        _lib = _bind(ctypes.CDLL(alt if alt else build()))
    return _lib


def _bind(lib):
    """Declare the C signatures on a loaded oracle library."""
    vp = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    gp = ctypes.POINTER(_Geom)
    lib.orc_decode.argtypes = [vp, i64, vp]
    lib.orc_decode.restype = None
    lib.orc_lut.argtypes = [gp, f64, vp]
    lib.orc_lut.restype = None
    lib.orc_ns_beams.argtypes = [i32, i32, vp, i32, vp, vp]
    lib.orc_ns_beams.restype = None
    lib.orc_ew_weights.argtypes = [gp, f64, vp]
    lib.orc_ew_weights.restype = None
    lib.orc_ew_beams.argtypes = [i32, i32, vp, vp, vp]
    lib.orc_ew_beams.restype = None
    lib.orc_upchan.argtypes = [i32, vp, vp]
    lib.orc_upchan.restype = None
    lib.orc_beamform_unit.argtypes = [gp, f64, vp, vp, vp]
    lib.orc_beamform_unit.restype = ctypes.c_int
    lib.orc_beamform_units.argtypes = [gp, vp, i32, vp, vp, i32, vp, i32, vp, i32]
    lib.orc_beamform_units.restype = ctypes.c_int
    lib.orc_beamform.argtypes = [gp, vp, i32, vp, vp, i32, vp, i32]
    lib.orc_beamform.restype = ctypes.c_int
    lib.orc_max_threads.argtypes = []
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_rescale_u8.argtypes = [vp, vp, vp, i64, vp]
    lib.orc_rescale_u8.restype = None
    lib.orc_group_bins.argtypes = [vp, i64, i32, i32, vp]
    lib.orc_group_bins.restype = None
    lib.orc_beams_unit.argtypes = [gp, f64, vp, vp, vp]
    lib.orc_beams_unit.restype = ctypes.c_int
    return lib


def _ptr(a: np.ndarray | None):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _cplx(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def group_bins(fine, group: int) -> np.ndarray:
    """Sum centre-shifted fine bins (last axis, length L) into L / group coarse
    sub-channels, each the `group` fine bins nearest its centre."""
    fine = np.ascontiguousarray(fine, dtype=np.float64)
    L = fine.shape[-1]
    if L % group:
        raise ValueError("group must divide the fine bin count")
    out = np.empty(fine.shape[:-1] + (L // group,), np.float64)
    _load().orc_group_bins(_ptr(fine), fine.size // L, L, group, _ptr(out))
    return out


def beamform_upchan128(g: Geometry, freqs, raw, lut_override=None, n_threads: int = 0,
                       units=None) -> np.ndarray:
    """The paper's up-channelisation (Sec. 3, Sec. 3.2): 128-point DFTs of every 128
    samples, Stokes I, integrated over the frame into 16 sub-channels of 8 fine
    channels each.  Output [.., beams, 16] like beamform."""
    g128 = Geometry(**{k: getattr(g, k) for k in ("n_feed", "pad", "n_cyl", "n_pol",
                                                  "n_beam_ns", "n_beam_ew", "n_time",
                                                  "feed_spacing_m", "c0", "cyl_x_m",
                                                  "sin_theta_ns", "sin_phi_ew")}, n_dft=128)
    fine = beamform(g128, freqs, raw, lut_override=lut_override, n_threads=n_threads,
                    units=units)
    return group_bins(fine, 8)


def rescale_u8(P, scale, offset) -> np.ndarray:
    """8-bit output codes clamp(rint(P * scale + offset), 0, 255), decided in FP32
    (Sec. 3, Table 1; the rule is a reading).  P: FP64 powers; scale, offset:
    broadcast to P's shape and rounded to FP32."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    sc = np.ascontiguousarray(np.broadcast_to(np.asarray(scale, np.float32), P.shape))
    of = np.ascontiguousarray(np.broadcast_to(np.asarray(offset, np.float32), P.shape))
    out = np.empty(P.shape, np.uint8)
    _load().orc_rescale_u8(_ptr(P), _ptr(sc), _ptr(of), P.size, _ptr(out))
    return out


def decode(raw) -> np.ndarray:
    """4+4-bit bytes -> complex128 (same shape)."""
    raw = np.ascontiguousarray(raw, dtype=np.uint8)
    out = np.empty(raw.shape, dtype=np.complex128)
    _load().orc_decode(_ptr(raw), raw.size, _ptr(out))
    return out


def lut(geom: Geometry, f_hz: float) -> np.ndarray:
    """Eq. (1) kept-bin index per desired N-S pointing."""
    g = geom._c()
    out = np.empty(geom.n_beam_ns, dtype=np.int32)
    _load().orc_lut(ctypes.byref(g), float(f_hz), _ptr(out))
    return out


def ns_beams(x, k, n_bins: int) -> np.ndarray:
    """Bins k of the n_bins-point DFT of the zero-padded line x (direct sums)."""
    x = _cplx(x)
    k = np.ascontiguousarray(k, dtype=np.int32)
    y = np.empty(k.shape, dtype=np.complex128)
    _load().orc_ns_beams(x.size, n_bins, _ptr(x), k.size, _ptr(k), _ptr(y))
    return y


def ew_weights(geom: Geometry, f_hz: float) -> np.ndarray:
    g = geom._c()
    w = np.empty((geom.n_beam_ew, geom.n_cyl), dtype=np.complex128)
    _load().orc_ew_weights(ctypes.byref(g), float(f_hz), _ptr(w))
    return w


def ew_beams(w, y) -> np.ndarray:
    w = _cplx(w)
    y = _cplx(y)
    n_ew, n_cyl = w.shape
    b = np.empty(n_ew, dtype=np.complex128)
    _load().orc_ew_beams(n_cyl, n_ew, _ptr(w), _ptr(y), _ptr(b))
    return b


def upchan(b) -> np.ndarray:
    b = _cplx(b)
    u = np.empty(b.size, dtype=np.complex128)
    _load().orc_upchan(b.size, _ptr(b), _ptr(u))
    return u


def beams_unit(geom: Geometry, f_hz: float, raw_unit, lut_override=None) -> np.ndarray:
    """Complex beams before detection for one channel-frame: complex128
    [n_time/n_dft][n_dft (bin s, not centre-shifted)][n_pol][n_beam_ew][n_beam_ns]."""
    raw_unit = np.ascontiguousarray(raw_unit, dtype=np.uint8)
    assert raw_unit.size == geom.n_time * geom.n_inputs
    lo = None if lut_override is None else np.ascontiguousarray(lut_override, dtype=np.int32)
    out = np.empty((geom.n_time // geom.n_dft, geom.n_dft, geom.n_pol, geom.n_beam_ew,
                    geom.n_beam_ns), dtype=np.complex128)
    g = geom._c()
    r = _load().orc_beams_unit(ctypes.byref(g), float(f_hz), _ptr(lo), _ptr(raw_unit), _ptr(out))
    if r != 0:
        raise RuntimeError("orc_beams_unit failed (%d)" % r)
    return out


def beamform_unit(geom: Geometry, f_hz: float, raw_unit, lut_override=None) -> np.ndarray:
    """One channel-frame: raw [n_time][n_inputs] u8 -> [n_beams][n_dft] float64."""
    raw_unit = np.ascontiguousarray(raw_unit, dtype=np.uint8)
    assert raw_unit.size == geom.n_time * geom.n_inputs
    lo = None if lut_override is None else np.ascontiguousarray(lut_override, dtype=np.int32)
    out = np.empty((geom.n_beams, geom.n_dft), dtype=np.float64)
    g = geom._c()
    r = _load().orc_beamform_unit(ctypes.byref(g), float(f_hz), _ptr(lo), _ptr(raw_unit), _ptr(out))
    if r != 0:
        raise RuntimeError("orc_beamform_unit failed (%d)" % r)
    return out


def beamform(geom: Geometry, freqs_hz, raw, lut_override=None, n_threads: int = 0,
             units=None) -> np.ndarray:
    """Batch oracle.

    raw: u8 [n_frames][n_chan][n_time][n_inputs].  Returns float64
    [n_frames][n_chan][n_beams][n_dft], or [n_units][n_beams][n_dft] when
    ``units`` (a sequence of (frame, chan) pairs) selects channel-frames.
    """
    raw = np.ascontiguousarray(raw, dtype=np.uint8)
    freqs = np.ascontiguousarray(freqs_hz, dtype=np.float64)
    n_frames, n_chan = raw.shape[0], raw.shape[1]
    assert freqs.shape == (n_chan,)
    assert raw.shape[2:] == (geom.n_time, geom.n_inputs), raw.shape
    lo = None
    if lut_override is not None:
        lo = np.ascontiguousarray(lut_override, dtype=np.int32)
        assert lo.shape == (n_chan, geom.n_beam_ns)
    g = geom._c()
    lib = _load()
    if units is None:
        out = np.empty((n_frames, n_chan, geom.n_beams, geom.n_dft), dtype=np.float64)
        r = lib.orc_beamform(ctypes.byref(g), _ptr(freqs), n_chan, _ptr(lo), _ptr(raw),
                             n_frames, _ptr(out), int(n_threads))
    else:
        u = np.ascontiguousarray(np.asarray(units, dtype=np.int32).reshape(-1, 2))
        out = np.empty((u.shape[0], geom.n_beams, geom.n_dft), dtype=np.float64)
        r = lib.orc_beamform_units(ctypes.byref(g), _ptr(freqs), n_chan, _ptr(lo), _ptr(raw),
                                   n_frames, _ptr(u), u.shape[0], _ptr(out), int(n_threads))
    if r != 0:
        raise RuntimeError("oracle beamform failed (%d)" % r)
    return out


__all__ = ["Geometry", "C0", "FEED_SPACING_M", "CYL_SPACING_M", "build", "decode", "lut",
           "ns_beams", "ew_weights", "ew_beams", "upchan", "beamform_unit", "beamform",
           "default_sin_theta", "default_sin_phi", "max_threads"]

