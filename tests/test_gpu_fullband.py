"""Full-band sky response through the GPU path (Fig. 3 and Sec. 3.3 aliasing; beam
widths of Sec. 3.1): one frame of all 1024 channels with a 26 deg point source,
and scans of a source across N-S beams at the bottom of the band.

Readings: the beam widths the paper quotes (about 0.5 deg at zenith, about 2.8 deg
at 10 deg elevation) are those of a single N-S beam at 400 MHz, the widest in the
band: 0.886 lambda / (N d cos theta) gives 0.49 and 2.81 deg."""
import math

import numpy as np
import pytest

import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

C0 = 299_792_458.0
D = 0.3048
TOL = {"fp32": 1e-5, "fp16": 2e-3, "fp32_mfma": 1e-5}
F_ALL = synth.chan_freq_hz(np.arange(1024))
S26 = math.sin(math.radians(26.0))
SIN_M = (np.arange(256) - 127.5) / 128


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
def fullband(torch_mod, bfm):
    raw = synth.point_source_frames(F_ALL, S26)
    print("fullband: 1024 channels x 1 frame, fp32", flush=True)
    with bfm.Beamformer(F_ALL, precision="fp32") as b:
        out = b.frame(torch_mod.from_numpy(raw).cuda())
        torch_mod.cuda.synchronize()
        return raw, out.cpu().numpy()[0], b.lut()


def _ns_af(kappa, k):
    """Closed-form power response of FFT bin k to a plane wave at bin position kappa
    (256 feeds, 512-point transform)."""
    n = np.arange(256)
    return np.abs(np.exp(2j * np.pi * np.outer(kappa - np.atleast_1d(k), n) / 512).sum(axis=1)) ** 2


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
def test_fullband_parity_sampled_channels(torch_mod, bfm, oracle_mod, fullband, precision):
    """Seeded channels across the band (below and inside the aliasing range), noiseless
    input: |P - P_ref| <= tol x max over the channel's outputs."""
    raw, out_fp32, _ = fullband
    idx = np.sort(np.concatenate([[0, 1023, 600], np.random.default_rng(71).choice(1024, 5,
                                                                               replace=False)]))
    if precision == "fp32":
        got = out_fp32[idx]
    else:
        with bfm.Beamformer(F_ALL[idx], precision=precision) as b:
            got = b.frame(torch_mod.from_numpy(np.ascontiguousarray(raw[:, idx])).cuda())
            got = got.cpu().numpy()[0]
    ref = oracle_mod.beamform(oracle_mod.Geometry(), F_ALL[idx], raw[:, idx])[0]
    for i, c in enumerate(idx):
        err = np.abs(got[i] - ref[i]).max() / ref[i].max()
        print("fullband %s channel %d (%.3f MHz): max err / max %.3e"
              % (precision, c, F_ALL[c] / 1e6, err))
        assert err <= TOL[precision]


def test_main_and_alias_beams_every_channel(fullband):
    """In every channel the strongest N-S beam holds the kept bin whose closed-form
    response to the source is largest (Eq. (1) clamping; within 3 % where two kept
    bins straddle the source), and every beam sharing that bin carries identical
    power.  The strongest beam pointing south of zenith (the alias of Sec. 3.3 once
    f > c / (d (1 + sin 26 deg)), about 684 MHz) has, relative to the main beam, the
    power the closed-form responses of the two kept bins predict."""
    _, out, lut = fullband
    ns = out[:, :, 8].reshape(1024, 4, 256).sum(axis=1).astype(np.float64)
    neg = np.nonzero(SIN_M < 0)[0]
    strong, strong_deg = [], []
    for c in range(1024):
        kappa = 512 * F_ALL[c] * D * S26 / C0
        m_main = int(np.argmax(ns[c]))
        k_main = lut[c][m_main]
        af_main = _ns_af(kappa, k_main)[0]
        assert af_main >= 0.97 * _ns_af(kappa, lut[c]).max(), c
        dup = set(np.nonzero(lut[c] == k_main)[0].tolist())
        same = set(np.nonzero(ns[c] == ns[c, m_main])[0].tolist())
        assert dup <= same, c
        # another bin may tie only where the source sits midway between two kept bins
        for m in same - dup:
            assert _ns_af(kappa, lut[c][m])[0] >= 0.97 * af_main, c
        m_alias = int(neg[np.argmax(ns[c, neg])])
        ratio = ns[c, m_alias] / ns[c, m_main]
        expect = _ns_af(kappa, lut[c][m_alias])[0] / af_main
        # 0.03 absolute: spatial harmonics of the quantised tone (about 1 % of the
        # main power) where the closed form predicts no alias
        assert abs(ratio - expect) <= 0.05 * expect + 0.03, (c, ratio, expect)
        if expect >= 0.5:
            strong.append(c)
            strong_deg.append(math.degrees(math.asin(SIN_M[m_alias])))
    f_edge = C0 / (D * (1 + S26))
    lo, hi = min(strong_deg), max(strong_deg)
    print("alias at >= half the main power: %d channels, %.3f .. %.3f MHz, %.2f .. %.2f deg"
          % (len(strong), F_ALL[strong[0]] / 1e6, F_ALL[strong[-1]] / 1e6, lo, hi))
    assert F_ALL[strong[0]] >= f_edge - 1e6 and F_ALL[strong[0]] < f_edge + 5e6
    assert strong[-1] == 1023
    # Sec. 3.3 prints about -88 .. -50 deg; the lowest pointing here is -84.93 deg
    assert abs(lo - (-88)) < 4 and abs(hi - (-50)) < 3


def _fwhm(th, p):
    h = p.max() / 2
    above = np.nonzero(p >= h)[0]
    i0, i1 = above[0], above[-1]
    left = np.interp(h, [p[i0 - 1], p[i0]], [th[i0 - 1], th[i0]])
    right = np.interp(h, [p[i1 + 1], p[i1]], [th[i1 + 1], th[i1]])
    return right - left


@pytest.mark.parametrize("m,span,paper_deg,paper_zenith_deg",
                         [(128, 0.6, 0.5, 0.0), (253, 3.0, 2.8, 80.0)])
def test_beam_width_at_band_bottom(torch_mod, bfm, m, span, paper_deg, paper_zenith_deg):
    """Scan a source across N-S beam m at 400 MHz (16 positions, one per channel slot)
    and measure the beam's FWHM from the GPU outputs."""
    f = 400e6
    k = int(bfm.compute_lut([f])[0][m])
    ks = k if k < 256 else k - 512
    centre = math.degrees(math.asin(ks * C0 / (512 * f * D)))
    th = centre + np.linspace(-span, span, 16)
    raw = synth.point_source_frames([f] * 16, np.sin(np.deg2rad(th)))
    print("beam width scan: beam %d (bin %d, %.3f deg), +-%.1f deg" % (m, k, centre, span),
          flush=True)
    with bfm.Beamformer([f] * 16, precision="fp32") as b:
        out = b.frame(torch_mod.from_numpy(raw).cuda()).cpu().numpy()[0]
    resp = out[:, m::256, 8].sum(axis=1).astype(np.float64)
    kappa = 512 * f * D * np.sin(np.deg2rad(th)) / C0
    af = np.array([_ns_af(kp, k)[0] for kp in kappa])
    assert np.abs(resp / resp.max() - af / af.max()).max() < 0.03
    w, w_af = _fwhm(th, resp), _fwhm(th, af)
    lam = C0 / f
    w_uniform = math.degrees(0.886 * lam / (256 * D)) / math.cos(math.radians(centre))
    print("FWHM beam %d: gpu %.4f deg, array factor %.4f, 0.886 lambda/(N d cos) %.4f"
          % (m, w, w_af, w_uniform))
    assert w == pytest.approx(w_af, rel=0.02)
    assert w == pytest.approx(w_uniform, rel=0.03)
    # scaled to the paper's elevation, the width is the paper's figure
    w_paper = w * math.cos(math.radians(centre)) / math.cos(math.radians(paper_zenith_deg))
    assert w_paper == pytest.approx(paper_deg, rel=0.1)


def _ew_af(f, u):
    """Closed-form power response of the 4 static E-W beams (R7 pointings, cylinders
    20 m apart) to a plane wave at E-W direction cosine u, per channel frequency f:
    [n_f][4]."""
    x = (np.arange(4) - 1.5) * 20.0
    sphi = np.sin(np.deg2rad((np.arange(4) - 1.5) * 0.4))
    ph = 2j * np.pi * np.asarray(f)[:, None, None] * x[None, None, :] \
        * (u - sphi)[None, :, None] / C0
    return np.abs(np.exp(ph).sum(axis=2)) ** 2


def _eq1_bins(f):
    """Eq. (1) for every channel and pointing, restated in FP64: [n_f][256]."""
    arg = 512 * np.asarray(f)[:, None] * D * SIN_M[None, :] / C0 + 0.5
    return np.mod(np.floor(arg).astype(np.int64), 512)


@pytest.fixture(scope="module", params=["fp32", "fp16"])
def summed_map(request, torch_mod, bfm):
    """Fig. 3's frequency-summed response: one noiseless frame of all 1024 channels
    with a source at 26 deg N-S, 0.2 deg E-W (on E-W beam 2), every output summed
    over the 16 sub-channels and the 1024 channels per beam."""
    precision = request.param
    raw = synth.point_source_frames(F_ALL, S26, phi_deg=0.2)
    print("summed map: 1024 channels x 1 frame, %s" % precision, flush=True)
    with bfm.Beamformer(F_ALL, precision=precision) as b:
        out = b.frame(torch_mod.from_numpy(raw).cuda())
        torch_mod.cuda.synchronize()
        out = out.cpu().numpy()[0].astype(np.float64)
    return precision, raw, out


def test_frequency_summed_map(summed_map, oracle_mod):
    """The summed map (Sec. 3.3, Fig. 3) against the closed-form array factors summed
    over the same channels: M[j][m] = sum_f AF_EW(j, f) AF_NS(k_m(f), f), independent
    of the oracle.  It peaks at the source's N-S pointing in its E-W beam; the alias
    south of zenith (from about 684 MHz up) is smeared over the pointings Sec. 3.3
    shows (about -88 .. -50 deg), much weaker than the main beam, with the summed
    alias-to-main ratio the closed form predicts; sampled channels match the oracle."""
    precision, raw, out = summed_map
    m_map = out.sum(axis=(0, 2)).reshape(4, 256)
    v = math.cos(math.radians(0.2)) * S26
    kappa = 512 * F_ALL * D * v / C0
    bins = _eq1_bins(F_ALL)
    n = np.arange(256)
    af_ns = np.abs(np.exp(2j * np.pi * (kappa[:, None, None] - bins[:, :, None]) * n / 512)
                   .sum(axis=2)) ** 2                                  # [f][m]
    af_ew = _ew_af(F_ALL, math.sin(math.radians(0.2)))                  # [f][j]
    pred = np.einsum("fj,fm->jm", af_ew, af_ns)
    j0, m0 = np.unravel_index(np.argmax(m_map), m_map.shape)
    jp, mp = np.unravel_index(np.argmax(pred), pred.shape)
    print("summed map %s: peak beam (j %d, m %d) at %.2f deg; closed form (j %d, m %d)"
          % (precision, j0, m0, math.degrees(math.asin(SIN_M[m0])), jp, mp))
    assert (j0, m0) == (jp, mp) == (2, int(np.argmin(np.abs(SIN_M - S26))))
    # whole map: shape of the closed form within the 4-bit tone's spatial harmonics
    mm, pp = m_map / m_map.max(), pred / pred.max()
    assert np.abs(mm - pp).max() <= 0.005
    south = SIN_M < 0
    row, row_p = mm[j0], pp[j0]
    ratio, ratio_p = row[south].max(), row_p[south].max()
    print("summed alias / main: gpu %.4f, closed form %.4f" % (ratio, ratio_p))
    assert ratio < 0.25                      # much weaker than the main beam
    assert abs(ratio - ratio_p) <= 0.05 * ratio_p + 0.001
    # where the alias power lies: pointings holding at least a tenth of the alias peak
    smear = np.degrees(np.arcsin(SIN_M[south & (row >= 0.1 * ratio)]))
    print("alias smear: %.2f .. %.2f deg over %d pointings" % (smear.min(), smear.max(), smear.size))
    assert smear.size >= 20
    assert smear.min() >= -88.5 and smear.max() <= -49.0
    assert smear.min() <= -80.0 and smear.max() >= -55.0
    # alias total power per channel starts at the predicted edge c / (d (1 + sin 26))
    ch_alias = out[:, j0 * 256:(j0 + 1) * 256][:, south].sum(axis=(1, 2))
    ch_main = out[:, j0 * 256 + m0].sum(axis=-1)
    first = int(np.argmax(ch_alias > 0.25 * ch_main))
    assert abs(F_ALL[first] - C0 / (D * (1 + v))) < 8e6
    idx = np.array([100, 683, 700, 1023])
    ref = oracle_mod.beamform(oracle_mod.Geometry(), F_ALL[idx], raw[:, idx])[0]
    err = np.abs(out[idx] - ref).max(axis=(1, 2)) / ref.max(axis=(1, 2))
    assert err.max() <= TOL[precision], err
