"""GPU test of the allocation-free tracking entry point
(beamform_frame_tracking_noalloc): through the C ABI its output equals
beamform_frame_tracking's bit for bit on two calls in a row, the second with a
smaller input (so the fixed table keeps rows of the first call that the second
must not read), and sizes beyond the fixed table are rejected before any
device work."""
import ctypes

import numpy as np
import pytest

import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

FREQS = [float(synth.chan_freq_hz(c)) for c in (130, 512, 901)]


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


def _run(torch_mod, b, raw_t, phi, noalloc):
    print("tracking noalloc=%s raw %s" % (noalloc, tuple(raw_t.shape)), flush=True)
    out = b.frame(raw_t, sin_phi_ew=phi, noalloc=noalloc)
    torch_mod.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
def test_noalloc_equals_tracking_two_calls(torch_mod, bfm, precision):
    raw, phi = synth.drifting_source(71, FREQS, 4, phi0_deg=0.25)
    track = synth.tracking_pointings(phi)
    raw_t = torch_mod.from_numpy(np.ascontiguousarray(raw)).cuda()
    with bfm.Beamformer(FREQS, precision=precision) as b:
        # first call: 4 frames x 3 channels; second: the last 2 frames only, with
        # other directions, so stale rows of the first call would show
        first_ref = _run(torch_mod, b, raw_t, track, noalloc=False)
        first = _run(torch_mod, b, raw_t, track, noalloc=True)
        np.testing.assert_array_equal(first, first_ref)
        track2 = track[2:] + 1e-3
        raw2 = raw_t[2:].contiguous()
        second = _run(torch_mod, b, raw2, track2, noalloc=True)
        second_ref = _run(torch_mod, b, raw2, track2, noalloc=False)
        np.testing.assert_array_equal(second, second_ref)
        assert not np.array_equal(second, first[2:])


def test_noalloc_rejects_oversized_call(torch_mod, bfm):
    """A call whose channel-frames exceed the fixed table fails with BF_E_INVAL
    from the host-side check; nothing is launched."""
    lib = bfm.load_library()
    n_chan = 128
    freqs = [float(synth.chan_freq_hz(c)) for c in range(n_chan)]
    n_frames = 16384 // n_chan + 1
    phi = np.zeros((n_frames, 4))
    with bfm.Beamformer(freqs) as b:
        # buffers of the full size the call names (13 GB in, 1.1 GB out), so that
        # even a launch would stay in bounds; the size check comes first
        raw = torch_mod.empty((n_frames, n_chan, 384, 2048), dtype=torch_mod.uint8, device="cuda")
        out = torch_mod.empty((n_frames, n_chan, 1024, 16), dtype=torch_mod.float32, device="cuda")
        st = lib.beamform_frame_tracking_noalloc(
            b._plan, ctypes.c_void_p(raw.data_ptr()), n_frames,
            ctypes.c_void_p(phi.ctypes.data), ctypes.c_void_p(out.data_ptr()), None)
        assert st == -1
        assert b"exceeds the fixed tracking table" in lib.beamform_last_error(b._plan)
        del raw, out
        torch_mod.cuda.empty_cache()
