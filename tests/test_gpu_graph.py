"""beamform_frame and beamform_frame_u8 recorded into a HIP graph (through a torch
CUDA graph on its capture stream) and replayed several times, with the program's own
eager work and synchronisations between the replays: every replay equals the eager
result bit for bit.  The calls enqueue only kernels (no memset, no copy), so a caller
can capture them."""
import numpy as np
import pytest

import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


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


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
def test_captured_frame_replays_equal_eager(torch_mod, bfm, precision):
    torch = torch_mod
    cfg = synth.config1(n_frames=2)
    raw = torch.from_numpy(cfg["raw"]).cuda()
    other = torch.from_numpy(synth.noise_frames(61, 2, 4)).cuda()
    print("graph capture: %s %s" % (tuple(raw.shape), precision), flush=True)
    with bfm.Beamformer(cfg["freqs"], precision=precision) as b:
        eager = b.frame(raw).clone()
        eager_other = b.frame(other).clone()
        tab = (4, 1024, 16)
        scale = torch.full(tab, 64.0 / 9.874e6, dtype=torch.float32, device="cuda")
        offset = torch.full(tab, 3.0, dtype=torch.float32, device="cuda")
        eager_u8 = b.frame_u8(raw, scale, offset).clone()
        src = torch.empty_like(raw)
        out = torch.empty_like(eager)
        out_u8 = torch.empty_like(eager_u8)
        src.copy_(raw)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            b.frame(src, out, stream=s)             # warm-up on the capture stream
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            b.frame(src, out, stream=s)
            b.frame_u8(src, scale, offset, out_u8, stream=s)
        for rep in range(4):
            inp, ref = (raw, eager) if rep % 2 == 0 else (other, eager_other)
            src.copy_(inp)                           # eager work between replays
            out.fill_(-1.0)
            out_u8.fill_(0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, ref), rep
            if rep % 2 == 0:
                assert torch.equal(out_u8, eager_u8), rep
            _ = b.frame(other)                      # the plan used eagerly in between
            torch.cuda.synchronize()
