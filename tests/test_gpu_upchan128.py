"""GPU tests of the paper's 128-point up-channelisation (beamform_frame_upchan128;
Sec. 3 and Sec. 3.2), all three precisions: per-output parity with the oracle (128-point DFTs of
128-sample blocks, fine bins grouped 8 to a sub-channel), the closed-form
relations to the 16-point path (a channel-centre tone: same sub-channel, 8 times
the power; any input: 8 times the total power), large and split batches, and
the unsupported configurations."""
import numpy as np
import pytest

import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-5


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


def _run(torch_mod, bfm, raw, freqs, upchan, **kw):
    print("upchan%d run: raw %s %s" % (upchan, raw.shape, kw), flush=True)
    with bfm.Beamformer(freqs, n_time=raw.shape[2], **kw) as b:
        out = b.frame(torch_mod.from_numpy(np.ascontiguousarray(raw)).cuda(), upchan=upchan)
        torch_mod.cuda.synchronize()
        return out.cpu().numpy().astype(np.float64)


TOLS = {"fp32": 1e-5, "fp16": 2e-3, "fp32_mfma": 1e-5}


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
def test_config0_parity(torch_mod, bfm, oracle_mod, precision):
    c = synth.config0()
    got = _run(torch_mod, bfm, c["raw"], c["freqs"], 128, precision=precision)
    ref = oracle_mod.beamform_upchan128(oracle_mod.Geometry(), c["freqs"], c["raw"])
    err = np.abs(got - ref) / ref
    print("upchan128 config0 %s max rel err %.3e" % (precision, err.max()))
    assert err.max() <= TOLS[precision]
    b, q = np.unravel_index(np.argmax(got[0, 0]), got[0, 0].shape)
    assert (b, q) == (3 * 256 + 171, 8)


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
@pytest.mark.parametrize("n_frames,n_chan,seed", [(3, 2, 41), (1, 5, 42)])
def test_uniform_bytes_parity(torch_mod, bfm, oracle_mod, n_frames, n_chan, seed, precision):
    raw = synth.uniform_bytes(seed, (n_frames, n_chan, 384, 2048))
    freqs = synth.chan_freq_hz(np.random.default_rng(seed).integers(0, 1024, n_chan))
    got = _run(torch_mod, bfm, raw, freqs, 128, precision=precision)
    ref = oracle_mod.beamform_upchan128(oracle_mod.Geometry(), freqs, raw)
    err = np.abs(got - ref) / ref
    print("upchan128 %dx%d %s max rel err %.3e" % (n_frames, n_chan, precision, err.max()))
    assert err.max() <= TOLS[precision]


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
@pytest.mark.parametrize("n_time", [128, 640])
def test_other_frame_lengths(torch_mod, bfm, oracle_mod, n_time, precision):
    """One 128-sample block per frame (the smallest the 128-point form takes) and five
    (a frame longer than the paper's): the kernel's block loop at both ends.  As for the
    16-point form, frames shorter than 0.983 ms integrate few terms, so the FP16 error is
    normalised by max(P_ref, median P_ref) there (R17)."""
    raw = synth.uniform_bytes(47 + n_time, (2, 2, n_time, 2048))
    freqs = synth.chan_freq_hz([150, 930])
    got = _run(torch_mod, bfm, raw, freqs, 128, precision=precision)
    ref = oracle_mod.beamform_upchan128(oracle_mod.Geometry(n_time=n_time), freqs, raw)
    den = ref if (precision != "fp16" or n_time >= 384) else np.maximum(ref, np.median(ref))
    err = np.abs(got - ref) / den
    print("upchan128 n_time %d %s max rel err %.3e" % (n_time, precision, err.max()))
    assert err.max() <= TOLS[precision]


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
@pytest.mark.parametrize("cyl_x", [None, (-31.0, -9.5, 10.25, 29.0)])
def test_general_geometry_parity(torch_mod, bfm, oracle_mod, precision, cyl_x):
    """E-W directions without mirror symmetry, with the default (symmetric) cylinders
    or asymmetric ones: the kernels' other E-W forms."""
    raw = synth.uniform_bytes(45, (1, 2, 384, 2048))
    freqs = synth.chan_freq_hz([300, 800])
    sphi = np.sin(np.deg2rad([-0.5, -0.1, 0.25, 0.7]))
    kw = {} if cyl_x is None else {"cyl_x_m": np.array(cyl_x)}
    got = _run(torch_mod, bfm, raw, freqs, 128, precision=precision, sin_phi_ew=sphi, **kw)
    ref = oracle_mod.beamform_upchan128(oracle_mod.Geometry(sin_phi_ew=sphi, **kw), freqs, raw)
    err = np.abs(got - ref) / ref
    assert err.max() <= TOLS[precision]


def test_many_channels_sampled(torch_mod, bfm, oracle_mod):
    """300 channels x 3 frames in one call; seeded channel-frames against the
    oracle."""
    n_frames, n_chan = 3, 300
    raw = synth.noise_frames(43, 1, 1)
    raw = np.ascontiguousarray(np.broadcast_to(raw, (n_frames, n_chan, 384, 2048)))
    rng = np.random.default_rng(43)
    freqs = synth.chan_freq_hz(rng.permutation(1024)[:n_chan])
    got = _run(torch_mod, bfm, raw, freqs, 128)
    units = [(int(f), int(c)) for f, c in zip(rng.integers(0, n_frames, 6), rng.integers(0, n_chan, 6))]
    ref = oracle_mod.beamform_upchan128(oracle_mod.Geometry(), freqs, raw, units=units)
    for i, (f, c) in enumerate(units):
        err = np.abs(got[f, c] - ref[i]) / ref[i]
        assert err.max() <= TOL, (f, c, err.max())


def test_batch_split_matches_one_call(torch_mod, bfm, oracle_mod):
    """4 channels x 66 frames: frames 62-65 of one call equal, bit for bit, the
    same frames beamformed in a call of their own (each channel-frame is
    independent of the batch around it), and two of them match the oracle."""
    n_frames, n_chan = 66, 4
    raw = synth.uniform_bytes(46, (n_frames, n_chan, 384, 2048))
    freqs = synth.chan_freq_hz([100, 400, 700, 1000])
    whole = _run(torch_mod, bfm, raw, freqs, 128)
    part = _run(torch_mod, bfm, raw[62:], freqs, 128)
    assert np.array_equal(whole[62:], part)
    units = [(63, 1), (65, 2)]
    ref = oracle_mod.beamform_upchan128(oracle_mod.Geometry(), freqs, raw, units=units)
    for i, (f, c) in enumerate(units):
        err = np.abs(whole[f, c] - ref[i]) / ref[i]
        assert err.max() <= TOL, (f, c, err.max())


def test_closed_form_relations_to_16_point(torch_mod, bfm):
    """Channel-centre tone (exact integer samples): sub-channel 8 only, 8 times the
    16-point power (3 x 128^2 against 24 x 16^2); uniform bytes: total power 8 times
    the 16-point total (Parseval).  The tone's beams span 100 dB (2e-10 of the peak
    power at the weakest), and the two forms round differently before the N-S
    transform (FP32 E-W sums against matrix-core products), so beyond the relative
    bound the relation holds to FP32 rounding of the peak: 1e-6 of the peak power."""
    tone = np.empty((1, 1, 384, 2048), np.uint8)
    synth.channel_frames(None, 600e6, 1, [synth.Source(0.3, 0.2, 3.0)], tone[:, 0], sigma=0.0)
    a16 = _run(torch_mod, bfm, tone, [600e6], 16)[0, 0]
    a128 = _run(torch_mod, bfm, tone, [600e6], 128)[0, 0]
    assert np.allclose(a128[:, 8], 8 * a16[:, 8], rtol=TOL, atol=1e-6 * a128[:, 8].max())
    strong = a128[:, 8] >= 1e-3 * a128[:, 8].max()
    assert np.allclose(a128[strong, 8], 8 * a16[strong, 8], rtol=TOL, atol=0)
    assert np.abs(np.delete(a128, 8, axis=1)).max() <= 1e-6 * a128.max()
    rnd = synth.uniform_bytes(44, (2, 3, 384, 2048))
    f = synth.chan_freq_hz([10, 500, 1000])
    t16 = _run(torch_mod, bfm, rnd, f, 16).sum(axis=-1)
    t128 = _run(torch_mod, bfm, rnd, f, 128).sum(axis=-1)
    assert np.allclose(t128, 8 * t16, rtol=TOL, atol=0)


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
def test_full_scale_coherent_input(torch_mod, bfm, oracle_mod, precision):
    """Every input at the most negative code (-8 - 8i) in every sample: the largest
    beams any frame can produce (N-S bin 0 of a coherent line, about 2^17.5 in
    amplitude before detection), all in the channel-centre sub-channel, stay exact
    to the path's tolerance; the other sub-channels stay at rounding level."""
    raw = np.zeros((1, 2, 384, 2048), np.uint8)
    freqs = synth.chan_freq_hz([20, 1000])
    got = _run(torch_mod, bfm, raw, freqs, 128, precision=precision)
    assert np.isfinite(got).all()
    ref = oracle_mod.beamform_upchan128(oracle_mod.Geometry(), freqs, raw)
    big = ref >= 1e-3 * ref.max()
    err = np.abs(got[big] - ref[big]) / ref[big]
    print("upchan128 full scale %s: max rel err %.3e over %d outputs" % (precision, err.max(), big.sum()))
    assert err.max() <= TOLS[precision]
    assert big[..., 8].any() and not big[..., np.arange(16) != 8].any()
    assert np.abs(got[..., np.arange(16) != 8]).max() <= 1e-5 * ref.max()


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
def test_config4_sky_parity(torch_mod, bfm, oracle_mod, precision):
    """Config-4 inputs (noise, DM-500 pulse, RFI tones identical on every input) in the
    128-point form: a strong tone concentrates into one fine channel, and any rounding
    applied before the 8-point DFT over sample phases would leak it into the
    noise-only fine channels of the neighbouring sub-channels (FP16-rounded
    intermediate beams of an earlier two-pass form reached 2.3e-3 here)."""
    c_idx = synth.sweep_c_idx(64)[[20, 31, 50]]
    raw = synth.config4_frames(1004, c_idx, [0], sky=synth.config4_sky(1004, c_idx))
    freqs = synth.chan_freq_hz(c_idx)
    got = _run(torch_mod, bfm, raw, freqs, 128, precision=precision)
    ref = oracle_mod.beamform_upchan128(oracle_mod.Geometry(), freqs, raw)
    err = np.abs(got - ref) / ref
    print("upchan128 config4 %s max rel err %.3e" % (precision, err.max()))
    assert err.max() <= TOLS[precision]


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
def test_tone_grouping_parity(torch_mod, bfm, oracle_mod, precision):
    """Noiseless tones on exact fine-channel frequencies, -5 .. +12 fine channels from
    several sub-channel centres (Sec. 3, Sec. 3.2): each lands in the sub-channel
    whose 8-fine-channel group holds its frequency (the group nearest the tone,
    its centre 1.5 kHz below the sub-channel's nominal centre), as the oracle pin
    derives from frequencies alone, and every output matches the oracle.  The
    frames hold exact Dirichlet-like nulls, so the error is taken against the
    frame's largest power."""
    import test_oracle_pins as pins
    f = 600e6
    raw = pins.tone_frames(pins.TONE_CASES, f)
    freqs = [f] * len(pins.TONE_CASES)
    got = _run(torch_mod, bfm, raw, freqs, 128, precision=precision)
    ref = oracle_mod.beamform_upchan128(oracle_mod.Geometry(), freqs, raw)
    err = np.abs(got - ref) / ref.max(axis=(2, 3), keepdims=True)
    print("upchan128 tones %s: max err / frame max %.3e" % (precision, err.max()))
    assert err.max() <= TOLS[precision]
    tot = got[0].sum(axis=1)
    for i, (q, off) in enumerate(pins.TONE_CASES):
        want = pins.expected_subchannel((q - 8) * synth.SUBCHAN_HZ + off * pins.FINE_HZ)
        assert int(np.argmax(tot[i])) == want, (q, off)
        assert tot[i, want] >= 0.99 * tot[i].sum(), (q, off)


def test_unsupported_configurations(torch_mod, bfm):
    short = torch_mod.zeros((1, 1, 48, 2048), dtype=torch_mod.uint8, device="cuda")
    with bfm.Beamformer([600e6], n_time=48) as b:
        with pytest.raises(bfm.BeamformError):
            b.frame(short, upchan=128)
        with pytest.raises(ValueError):
            b.frame(short, upchan=64)
