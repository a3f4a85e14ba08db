"""GPU tests of the 8-bit output (beamform_frame_u8; Sec. 3 and Table 1: the integrated
beams leave the beamformer as 8-bit integers): codes against the oracle's codes,
decided in FP32 from the oracle's FP64 powers; codes against the same launch's FP32
powers; argument errors.

Several codes are correct where P scale + offset lies within the path's power
tolerance of a rounding tie (k + 0.5): there either neighbour is accepted and
everything else must match exactly."""
import numpy as np
import pytest

import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = {"fp32": 1e-5, "fp16": 2e-3, "fp32_mfma": 1e-5}
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


@pytest.fixture(scope="module")
def case():
    """Config-1 sources and noise on 3 channels, 2 frames; per-output scales around
    64 / (noise mean) and offsets in [-40, 40], so codes span 0 .. 255 (both ends
    saturate)."""
    c = synth.config1(n_frames=2)
    raw, freqs = c["raw"][:, :3], c["freqs"][:3]
    rng = np.random.default_rng(91)
    scale = rng.uniform(0.5, 3.0, (3, 1024, 16)).astype(np.float32) * np.float32(64 / 9.874e6)
    offset = rng.uniform(-40, 40, (3, 1024, 16)).astype(np.float32)
    return np.ascontiguousarray(raw), freqs, scale, offset


def _run_u8(torch_mod, bfm, raw, freqs, scale, offset, precision):
    print("u8 run: raw %s precision %s" % (raw.shape, precision), flush=True)
    with bfm.Beamformer(freqs, precision=precision) as b:
        d = torch_mod.from_numpy(raw).cuda()
        u8 = b.frame_u8(d, torch_mod.from_numpy(scale).cuda(), torch_mod.from_numpy(offset).cuda())
        p32 = b.frame(d)
        torch_mod.cuda.synchronize()
        return u8.cpu().numpy(), p32.cpu().numpy()


def _check_codes(got, P, scale, offset, rel_tol):
    """got == codes of P except within rel_tol of a tie, where a neighbour is allowed."""
    t = np.float32(P).astype(np.float64) * scale.astype(np.float64) + offset.astype(np.float64)
    ref = np.clip(np.rint(t.astype(np.float32)), 0, 255).astype(np.int64)
    band = rel_tol * np.abs(np.float32(P).astype(np.float64) * scale) + 1e-6
    near_tie = np.abs(t - (np.floor(t) + 0.5)) <= band
    diff = got.astype(np.int64) - ref
    bad = (diff != 0) & ~(near_tie & (np.abs(diff) == 1))
    return int(bad.sum()), int(((diff != 0) & near_tie).sum()), ref


@pytest.mark.parametrize("precision", PRECISIONS)
def test_u8_codes_against_oracle(torch_mod, bfm, oracle_mod, case, precision):
    raw, freqs, scale, offset = case
    got, _ = _run_u8(torch_mod, bfm, raw, freqs, scale, offset, precision)
    P = oracle_mod.beamform(oracle_mod.Geometry(), freqs, raw)
    sc = np.broadcast_to(scale, P.shape)
    of = np.broadcast_to(offset, P.shape)
    ref_oracle = oracle_mod.rescale_u8(P, sc, of)
    n_bad, n_tie, ref = _check_codes(got, P, sc, of, TOL[precision])
    assert np.array_equal(ref.astype(np.uint8), ref_oracle)   # same rule on both sides
    print("u8 %s: %d codes, %d at 0, %d at 255, %d differ at ties, %d wrong"
          % (precision, got.size, (got == 0).sum(), (got == 255).sum(), n_tie, n_bad))
    assert (got == 0).sum() > 0 and (got == 255).sum() > 0
    assert n_bad == 0


@pytest.mark.parametrize("precision", PRECISIONS)
def test_u8_codes_equal_rescaled_fp32_output(torch_mod, bfm, case, precision):
    """The 8-bit epilogue applies the rule to exactly the powers beamform_frame writes."""
    raw, freqs, scale, offset = case
    got, p32 = _run_u8(torch_mod, bfm, raw, freqs, scale, offset, precision)
    sc = np.broadcast_to(scale, p32.shape)
    of = np.broadcast_to(offset, p32.shape)
    n_bad, n_tie, _ = _check_codes(got, p32.astype(np.float64), sc, of, 0.0)
    assert n_bad == 0 and n_tie == 0


def test_u8_argument_errors(torch_mod, bfm):
    raw = torch_mod.zeros((1, 1, 384, 2048), dtype=torch_mod.uint8, device="cuda")
    tab = torch_mod.zeros((1, 1024, 16), dtype=torch_mod.float32, device="cuda")
    with bfm.Beamformer([600e6]) as b:
        with pytest.raises(ValueError):
            b.frame_u8(raw, tab.double(), tab)
        with pytest.raises(ValueError):
            b.frame_u8(raw, tab, tab[:, :512])
        out = b.frame_u8(raw, tab, tab + 7.0)
        assert out.dtype == torch_mod.uint8 and bool((out == 7).all())
