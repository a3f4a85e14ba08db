"""The bench's other steps at full size, in the launch configuration the bench times
(config 1: 4 channels x 128 frames, one call over all 512 channel-frames): tracking E-W
beams (Sec. 3.1), 8-bit output (Table 1) and the 128-point up-channelisation (Sec. 3,
Sec. 3.2).  Seeded samples of channel-frames are checked against the oracle.  The
8-bit codes are checked on every output against the same path's FP32 powers."""
import numpy as np
import pytest

import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = {"fp32": 1e-5, "fp16": 2e-3, "fp32_mfma": 1e-5}
PRECISIONS = ["fp32", "fp16", "fp32_mfma"]
FRAME_S = 384 * 2.56e-6


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


@pytest.fixture(scope="module")
def workload(torch_mod):
    c = synth.config1()
    print("bench workload: raw %s" % (c["raw"].shape,), flush=True)
    return c["raw"], c["freqs"], torch_mod.from_numpy(c["raw"]).cuda()


def _units(seed, n=4):
    """Seeded (frame, channel) pairs, the first and last frames always among them."""
    rng = np.random.default_rng(seed)
    fr = [0, 127] + list(rng.integers(1, 127, n - 2))
    return [(int(f), int(c)) for f, c in zip(fr, rng.integers(0, 4, n))]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_tracking_full_size_sampled(torch_mod, bfm, oracle_mod, workload, precision):
    """Beam 2 follows a source drifting from 0.3 deg at the sidereal rate, as in the
    bench: every frame has its own (non-mirrored) E-W directions."""
    raw, freqs, d = workload
    phi = 0.3 + (15.0 / 3600.0) * FRAME_S * np.arange(raw.shape[0])
    track = synth.tracking_pointings(phi)
    print("tracking full size %s" % precision, flush=True)
    with bfm.Beamformer(freqs, precision=precision) as b:
        got = b.frame(d, sin_phi_ew=track)
        torch_mod.cuda.synchronize()
        got = got.cpu().numpy().astype(np.float64)
    for f, c in _units(71):
        ref = oracle_mod.beamform(oracle_mod.Geometry(sin_phi_ew=track[f]), freqs,
                                  raw[f:f + 1], units=[(0, c)])[0]
        err = np.abs(got[f, c] - ref) / ref
        print("tracking %s frame %d channel %d max rel err %.3e" % (precision, f, c, err.max()))
        assert err.max() <= TOL[precision]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_u8_full_size(torch_mod, bfm, oracle_mod, workload, precision):
    """The bench's tables (noise mean to code 64, no offset).  Every code equals the
    rule applied in FP32 to the same path's FP32 powers, and the sampled
    channel-frames' codes equal the oracle's, a neighbour being accepted where the
    scaled power lies within the path's tolerance of a rounding tie."""
    raw, freqs, d = workload
    scale = np.full((len(freqs), 1024, 16), 64.0 / 9.874e6, np.float32)
    offset = np.zeros_like(scale)
    print("u8 full size %s" % precision, flush=True)
    with bfm.Beamformer(freqs, precision=precision) as b:
        u8 = b.frame_u8(d, torch_mod.from_numpy(scale).cuda(), torch_mod.from_numpy(offset).cuda())
        p32 = b.frame(d)
        torch_mod.cuda.synchronize()
        u8, p32 = u8.cpu().numpy(), p32.cpu().numpy()
    codes = np.clip(np.rint(p32 * scale[None] + offset[None]), 0, 255).astype(np.uint8)
    assert np.array_equal(u8, codes)
    assert 0 < np.median(u8) < 255
    for f, c in _units(72):
        P = oracle_mod.beamform(oracle_mod.Geometry(), freqs, raw, units=[(f, c)])[0]
        ref = oracle_mod.rescale_u8(P, scale[c], offset[c])
        t = P * scale[c].astype(np.float64) + offset[c].astype(np.float64)
        near_tie = np.abs(t - (np.floor(t) + 0.5)) <= TOL[precision] * t + 1e-6
        diff = u8[f, c].astype(np.int64) - ref.astype(np.int64)
        bad = (diff != 0) & ~(near_tie & (np.abs(diff) == 1))
        print("u8 %s frame %d channel %d: %d codes differ at ties, %d wrong"
              % (precision, f, c, int((diff != 0).sum()), int(bad.sum())))
        assert not bad.any()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_upchan128_full_size_sampled(torch_mod, bfm, oracle_mod, workload, precision):
    """The bench's one-launch 128-point step at full size, sampled against the oracle."""
    raw, freqs, d = workload
    print("upchan128 full size %s" % precision, flush=True)
    with bfm.Beamformer(freqs, precision=precision) as b:
        got = b.frame(d, upchan=128)
        torch_mod.cuda.synchronize()
        got = got.cpu().numpy().astype(np.float64)
    assert np.isfinite(got).all() and (got > 0).all()
    units = _units(73)
    ref = oracle_mod.beamform_upchan128(oracle_mod.Geometry(), freqs, raw, units=units)
    for i, (f, c) in enumerate(units):
        err = np.abs(got[f, c] - ref[i]) / ref[i]
        print("upchan128 %s frame %d channel %d max rel err %.3e" % (precision, f, c, err.max()))
        assert err.max() <= TOL[precision]
