"""GPU tests of the pre-detection beams (beamform_debug_ns): complex values against
the oracle's beams before |.|^2, which pins the phases that power parity cannot see,
and detection of those beams against beamform_frame, for all three precisions."""
import numpy as np
import pytest

import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

# amplitude tolerance relative to the largest beam of the same (block, sub-channel):
# the power tolerances 1e-5 and 2e-3 halved, as amplitudes
TOL = {"fp32": 5e-6, "fp16": 1e-3, "fp32_mfma": 5e-6}
PRECISIONS = ["fp32", "fp16", "fp32_mfma"]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    torch.cuda.init()
    return torch


@pytest.fixture(scope="module")
def bfm():
    import paper_1702_04728_amd as bf
    bf.load_library()
    return bf


def _beams(torch_mod, bfm, raw1, freqs, precision):
    """raw1: one frame [n_chan][384][2048]."""
    print("debug_ns: %s precision %s" % (raw1.shape, precision), flush=True)
    with bfm.Beamformer(freqs, precision=precision) as b:
        d = torch_mod.from_numpy(np.ascontiguousarray(raw1)).cuda()
        u = b.debug_ns(d)
        p = b.frame(d[None])
        torch_mod.cuda.synchronize()
        return u.cpu().numpy().astype(np.complex128), p.cpu().numpy()[0]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_complex_beams_against_oracle(torch_mod, bfm, oracle_mod, precision):
    c = synth.config0()
    raw1 = np.concatenate([c["raw"][0], synth.uniform_bytes(51, (1, 384, 2048))])
    freqs = np.array([c["freqs"][0], float(synth.chan_freq_hz(870))])
    got, _ = _beams(torch_mod, bfm, raw1, freqs, precision)
    assert got.shape == (2, 24, 16, 2, 4, 256)
    g = oracle_mod.Geometry()
    for ch in range(2):
        ref = oracle_mod.beams_unit(g, freqs[ch], raw1[ch])       # [24][16][2][4][256]
        scale = np.abs(ref).reshape(24, 16, -1).max(axis=-1)[..., None, None, None]
        err = (np.abs(got[ch] - ref) / scale).max()
        print("debug_ns %s channel %d: max |dU| / max|U| per (block, s) %.3e" % (precision, ch, err))
        assert err <= TOL[precision]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_detected_beams_equal_frame_output(torch_mod, bfm, precision):
    raw1 = synth.noise_frames(52, 1, 3)[0]
    freqs = synth.chan_freq_hz([5, 333, 1010])
    u, p = _beams(torch_mod, bfm, raw1, freqs, precision)
    pw = (np.abs(u) ** 2).sum(axis=(1, 3))                          # [ch][s][j][m]
    for s in range(16):
        q = (s + 8) % 16
        ref = p[:, :, q].astype(np.float64).reshape(3, 4, 256)
        lut = bfm.compute_lut(freqs)
        # outputs gather bins through the Eq. (1) table; the beams hold them per m
        assert np.allclose(pw[:, s], ref, rtol=1e-5, atol=0), (s, lut.shape)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_ns_stage_alone_against_numpy_fft(torch_mod, bfm, precision):
    """The N-S stage on its own (Sec. 3.1): only cylinder 0 carries signal, constant
    over one 16-sample block, and all E-W directions are 0 (every weight exactly 1), so
    every E-W beam is cylinder 0's line and the time DFT is 16 x the sample in bin 0 and
    exactly 0 elsewhere.  Bin 0's beams must equal 16 x the zero-padded 512-point FFT of
    the 256 feeds (numpy's, a library routine independent of both the oracle and the
    kernels) at the Eq. (1) bins of every channel."""
    rng = np.random.default_rng(55)
    freqs = synth.chan_freq_hz([40, 512, 990])
    n_chan = len(freqs)
    x = rng.integers(-8, 8, (n_chan, 256, 2)) + 1j * rng.integers(-8, 8, (n_chan, 256, 2))
    raw1 = np.full((n_chan, 16, 2048), 0x88, dtype=np.uint8)
    code = (((x.real + 8).astype(np.uint8) << 4) | (x.imag + 8).astype(np.uint8)).reshape(n_chan, 512)
    raw1[:, :, :512] = code[:, None, :]                     # inputs (0 * 256 + n) * 2 + p
    print("debug_ns N-S alone: %s precision %s" % (raw1.shape, precision), flush=True)
    with bfm.Beamformer(freqs, precision=precision, n_time=16, sin_phi_ew=np.zeros(4)) as b:
        u = b.debug_ns(torch_mod.from_numpy(raw1).cuda()).cpu().numpy().astype(np.complex128)
    assert u.shape == (n_chan, 1, 16, 2, 4, 256)
    assert not np.any(u[:, :, 1:])                          # time-DFT bins s != 0: exactly 0
    sin_m = (np.arange(256) - 127.5) / 128
    for c, f in enumerate(freqs):
        k = np.mod(np.floor(512 * f * 0.3048 * sin_m / 299_792_458.0 + 0.5).astype(np.int64), 512)
        for p in range(2):
            ref = 16 * np.fft.fft(x[c, :, p], 512)[k]
            got = u[c, 0, 0, p]                             # [j][m]
            for j in range(4):
                err = np.abs(got[j] - ref).max() / np.abs(ref).max()
                assert err <= TOL[precision], (c, p, j, err)
            assert np.array_equal(got[0], got[3]) and np.array_equal(got[1], got[2])


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("directions", ["default", "tracking_tie"])
def test_impulse_beams_equal_weight_times_phase(torch_mod, bfm, oracle_mod, precision, directions):
    """Time DFT and E-W phasing together (Sec. 3, Sec. 3.1), closed form: block k holds a
    single sample of value 7 at sample t1 = k mod 4 of cylinder c = k div 4, feed 0, pol 0,
    so every kept beam of sub-channel s and E-W beam j must be 7 W[j][c] w16^(s t1) (feed 0
    has N-S phase 1 in every bin), pol 1 and the empty blocks exactly 0.  The tracking
    directions are the bench's last frame, whose weights at 650 MHz put an entry of
    W[3][c] w16^(s t1) on an FP16 rounding tie (0.46838...): the matrix-core paths carry
    those products as FP16 hi + lo pairs, which must come from one FP32 value."""
    freqs = np.array([450e6, 550e6, 650e6, 750e6])
    if directions == "default":
        sin_phi = None
        geom = oracle_mod.Geometry()
    else:
        phi = 0.3 + (15.0 / 3600.0) * 384 * 2.56e-6 * 127
        sin_phi = synth.tracking_pointings([phi])[0]
        geom = oracle_mod.Geometry(sin_phi_ew=sin_phi)
    raw1 = np.full((4, 384, 2048), 0x88, dtype=np.uint8)
    for k in range(16):
        raw1[:, 16 * k + (k & 3), (k >> 2) * 512] = 0xF8       # value 7 + 0i
    print("debug_ns impulses: %s directions, precision %s" % (directions, precision), flush=True)
    with bfm.Beamformer(freqs, precision=precision, sin_phi_ew=sin_phi) as b:
        u = b.debug_ns(torch_mod.from_numpy(raw1).cuda()).cpu().numpy().astype(np.complex128)
    assert not np.any(u[:, 16:]) and not np.any(u[:, :, :, 1])
    s = np.arange(16)
    for ch, f in enumerate(freqs):
        W = oracle_mod.ew_weights(geom, f)                       # [j][c]
        for k in range(16):
            ref = 7 * W[None, :, k >> 2] * np.exp(-2j * np.pi * s * (k & 3) / 16)[:, None]
            err = np.abs(u[ch, k, :, 0] - ref[:, :, None]).max() / 7
            assert err <= TOL[precision], (ch, k, err)
