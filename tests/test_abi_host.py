"""Host-side checks of libbeamform.so that need no GPU: it loads, exports every
symbol the header declares, and its FP64 host precompute (the Eq. (1) bin
table) agrees with the oracle's independent evaluation."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1702_04728_amd as bf
from paper_1702_04728_amd import beamform as bfm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "beamform.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(beamform_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return bf.load_library()


def test_exports_every_declared_symbol(lib):
    declared = _declared_symbols()
    assert len(declared) >= 9
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(bf.EXPORTED) == declared


def test_default_config(lib):
    c = bfm.BfConfig()
    assert lib.beamform_default_config(ctypes.byref(c)) == 0
    assert (c.n_cyl, c.n_feed, c.n_pol, c.pad, c.n_beam_ns, c.n_beam_ew, c.n_upchan, c.n_time) == \
        (4, 256, 2, 2, 256, 4, 16, 384)
    assert c.feed_spacing_m == 0.3048 and c.c0 == 299792458.0
    assert c.precision == bf.FP32_FFT and c.reserved == 0
    assert lib.beamform_default_config(None) == -1


def test_strerror(lib):
    assert lib.beamform_strerror(0) == b"ok"
    for s in (-1, -2, -3, -4, -5):
        assert lib.beamform_strerror(s) not in (b"ok", b"unknown status")
    assert lib.beamform_strerror(-99) == b"unknown status"


def test_lut_matches_oracle_all_channels(oracle_mod):
    freqs = 400e6 + np.arange(1024) * 390625.0
    lib_lut = bf.compute_lut(freqs)
    g = oracle_mod.Geometry()
    for c in range(1024):
        np.testing.assert_array_equal(lib_lut[c], oracle_mod.lut(g, freqs[c]))


def test_lut_custom_pointings_and_override(oracle_mod):
    rng = np.random.default_rng(1)
    st = np.sort(rng.uniform(-1, 1, 256))
    freqs = np.array([412.5e6, 733.1e6])
    g = oracle_mod.Geometry(sin_theta_ns=st)
    got = bf.compute_lut(freqs, sin_theta_ns=st)
    for c in range(2):
        np.testing.assert_array_equal(got[c], oracle_mod.lut(g, freqs[c]))
    ov = rng.integers(0, 512, (2, 256)).astype(np.int32)
    np.testing.assert_array_equal(bf.compute_lut(freqs, lut_override=ov), ov)
    ov[1, 7] = 512
    with pytest.raises(bf.BeamformError):
        bf.compute_lut(freqs, lut_override=ov)


def test_lut_rejects_out_of_range_argument():
    """A finite but huge frequency or pointing is refused instead of overflowing the
    integer floor of Eq. (1)."""
    with pytest.raises(bf.BeamformError):
        bf.compute_lut([1e300])
    with pytest.raises(bf.BeamformError):
        bf.compute_lut([600e6], sin_theta_ns=np.full(256, 1e200))


def test_lut_rejects_bad_frequency():
    with pytest.raises(bf.BeamformError):
        bf.compute_lut([600e6, -1.0])
    with pytest.raises(bf.BeamformError):
        bf.compute_lut([float("nan")])


def _init_status(lib, **fields):
    c = bfm.BfConfig()
    lib.beamform_default_config(ctypes.byref(c))
    for k, v in fields.items():
        setattr(c, k, v)
    f = np.array([600e6])
    plan = ctypes.c_void_p()
    return lib.beamform_init(ctypes.byref(c), ctypes.c_void_p(f.ctypes.data), 1, None,
                             ctypes.byref(plan))


def test_init_rejects_bad_config_before_touching_device(lib):
    """Configuration errors are reported before any HIP call (so also on a CPU host)."""
    assert _init_status(lib, n_time=100) == -1
    assert _init_status(lib, n_time=0) == -1
    assert _init_status(lib, reserved=1) == -1
    assert _init_status(lib, precision=7) == -1
    assert _init_status(lib, feed_spacing_m=0.0) == -1
    assert _init_status(lib, n_feed=128) == -5
    assert _init_status(lib, n_upchan=128) == -5
    assert b"16" in lib.beamform_last_error(None) or lib.beamform_last_error(None)


def test_null_arguments(lib):
    assert lib.beamform_frame(None, None, 1, None, None) == -1
    assert lib.beamform_destroy(None) == 0
    assert lib.beamform_get_lut(None, None) == -1
    assert lib.beamform_plan_info(None, None, None, None) == -1
