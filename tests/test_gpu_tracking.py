"""GPU tests of tracking E-W beams (beamform_frame_tracking; Sec. 3.1: the E-W
beams may be static or tracking): per-frame E-W directions against the FP64
oracle run with each frame's geometry, equality with static plans, a drifting
source held in its tracking beam, the plan's table regrowing, argument errors."""
import numpy as np
import pytest

import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = {"fp32": 1e-5, "fp16": 2e-3, "fp32_mfma": 1e-5}
PRECISIONS = ["fp32", "fp16", "fp32_mfma"]
FREQS = [float(synth.chan_freq_hz(200)), float(synth.chan_freq_hz(512)),
         float(synth.chan_freq_hz(937))]


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
def drift():
    # phi0 = 0.25 deg: no frame's directions are mirror-symmetric
    raw, phi = synth.drifting_source(61, FREQS, 3, phi0_deg=0.25)
    return raw, phi, synth.tracking_pointings(phi)


def _track(torch_mod, bfm, raw, freqs, sin_phi, precision, **kw):
    print("tracking run: raw %s precision %s sin_phi %s" % (raw.shape, precision,
                                                            np.round(sin_phi, 5).tolist()),
          flush=True)
    with bfm.Beamformer(freqs, precision=precision, **kw) as b:
        out = b.frame(torch_mod.from_numpy(np.ascontiguousarray(raw)).cuda(), sin_phi_ew=sin_phi)
        torch_mod.cuda.synchronize()
        return out.cpu().numpy()


def _static(torch_mod, bfm, raw, freqs, precision, **kw):
    with bfm.Beamformer(freqs, precision=precision, **kw) as b:
        out = b.frame(torch_mod.from_numpy(np.ascontiguousarray(raw)).cuda())
        torch_mod.cuda.synchronize()
        return out.cpu().numpy()


@pytest.mark.parametrize("precision", PRECISIONS)
def test_tracking_parity_vs_oracle(torch_mod, bfm, oracle_mod, drift, precision):
    raw, _, track = drift
    got = _track(torch_mod, bfm, raw, FREQS, track, precision).astype(np.float64)
    for fr in range(raw.shape[0]):
        ref = oracle_mod.beamform(oracle_mod.Geometry(sin_phi_ew=track[fr]), FREQS,
                                  raw[fr:fr + 1])[0]
        err = np.abs(got[fr] - ref) / ref
        print("tracking %s frame %d max rel err %.3e" % (precision, fr, err.max()))
        assert err.max() <= TOL[precision]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_tracking_equals_static_plan_per_frame(torch_mod, bfm, drift, precision):
    """Frame f of a tracking call equals a static plan built with frame f's
    directions, bit for bit (both take the general E-W form here)."""
    raw, _, track = drift
    got = _track(torch_mod, bfm, raw, FREQS, track, precision)
    for fr in range(raw.shape[0]):
        ref = _static(torch_mod, bfm, raw[fr:fr + 1], FREQS, precision, sin_phi_ew=track[fr])
        np.testing.assert_array_equal(got[fr], ref[0])


@pytest.mark.parametrize("precision", PRECISIONS)
def test_static_directions_every_frame_equal_beamform_frame(torch_mod, bfm, drift, precision):
    """A static plan's (mirror-symmetric) directions repeated in every frame
    reproduce that plan's beamform_frame exactly."""
    raw, _, _ = drift
    sphi = np.sin(np.deg2rad((np.arange(4) - 1.5) * 0.4))
    got = _track(torch_mod, bfm, raw, FREQS, np.tile(sphi, (raw.shape[0], 1)), precision,
                 sin_phi_ew=sphi)
    ref = _static(torch_mod, bfm, raw, FREQS, precision, sin_phi_ew=sphi)
    np.testing.assert_array_equal(got, ref)


def test_drifting_source_held_in_tracked_beam(torch_mod, bfm, drift):
    """The source stays at the peak of E-W beam 2 in every frame when tracked."""
    raw, _, track = drift
    got = _track(torch_mod, bfm, raw, FREQS, track, "fp32")
    ci = FREQS.index(600e6)
    peaks = []
    for fr in range(raw.shape[0]):
        b, q = np.unravel_index(np.argmax(got[fr, ci]), got[fr, ci].shape)
        assert b // 256 == 2 and q == 8
        peaks.append(got[fr, ci, b, q])
    assert max(peaks) / min(peaks) < 1.05


def test_tracking_table_regrows_and_shrinks(torch_mod, bfm, oracle_mod):
    """Calls of 1, 4 and 2 frames on one plan (the device table grows once and is
    reused); each matches the oracle."""
    freqs = FREQS[:2]
    raw, phi = synth.drifting_source(62, freqs, 4, rate_deg=-0.2)
    track = synth.tracking_pointings(phi, lead_beam=1)
    with bfm.Beamformer(freqs, precision="fp32") as b:
        for n in (1, 4, 2):
            print("tracking regrow: %d frames" % n, flush=True)
            out = b.frame(torch_mod.from_numpy(raw[:n].copy()).cuda(), sin_phi_ew=track[:n])
            got = out.cpu().numpy().astype(np.float64)
            for fr in range(n):
                ref = oracle_mod.beamform(oracle_mod.Geometry(sin_phi_ew=track[fr]), freqs,
                                          raw[fr:fr + 1])[0]
                assert (np.abs(got[fr] - ref) / ref).max() <= TOL["fp32"]


def test_tracking_argument_errors(torch_mod, bfm):
    raw = torch_mod.zeros((2, 1, 384, 2048), dtype=torch_mod.uint8, device="cuda")
    with bfm.Beamformer([600e6]) as b:
        bad = np.zeros((2, 4))
        bad[1, 2] = np.nan
        with pytest.raises(bfm.BeamformError):
            b.frame(raw, sin_phi_ew=bad)
        with pytest.raises(ValueError):
            b.frame(raw, sin_phi_ew=np.zeros((3, 4)))
        out = b.frame(raw[:0], sin_phi_ew=np.zeros((0, 4)))
        assert out.shape[0] == 0
