"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle by a route other than its own code: exhaustive
tables, exact rational evaluation, library transforms (numpy.fft) as special
cases, closed-form array factors, Parseval energy identities, exact Dirichlet
nulls, a point source whose beam geometry predicts, noise statistics from the
normal CDF, and an unstaged brute-force sum on a tiny array.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import norm

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
C0 = 299_792_458.0
D = 0.3048


def _geom(oracle_mod, **kw):
    return oracle_mod.Geometry(**kw)


# ---------------------------------------------------------------- P1 decode
def test_decode_exhaustive(oracle_mod):
    """All 256 byte values: decode inverts the generator's independent encoder."""
    re = np.repeat(np.arange(-8, 8), 16)
    im = np.tile(np.arange(-8, 8), 16)
    raw = synth.encode(re, im)
    assert sorted(raw.tolist()) == list(range(256))
    z = oracle_mod.decode(raw)
    np.testing.assert_array_equal(z.real, re)
    np.testing.assert_array_equal(z.imag, im)


def test_decode_fixed_values(oracle_mod):
    """Offset-binary with the real part in the high nibble."""
    z = oracle_mod.decode(np.array([0x88, 0x00, 0xF0, 0x0F, 0xFF, 0x97], dtype=np.uint8))
    np.testing.assert_array_equal(z, [0, -8 - 8j, 7 - 8j, -8 + 7j, 7 + 7j, 1 - 1j])


# ---------------------------------------------------------------- P2 LUT (Eq. 1)
def _lut_exact(f_hz_int: int, m: int, n_beam=256, nb=512):
    """Eq. (1) in exact rational arithmetic for the default sin-uniform pointings."""
    s = Fraction(2 * m - (n_beam - 1), n_beam)
    x = Fraction(nb) * Fraction(f_hz_int) * Fraction(3048, 10000) / Fraction(299792458) * s
    return math.floor(x + Fraction(1, 2)) % nb


def test_lut_matches_exact_rational_all_channels(oracle_mod):
    """FP64 evaluation never lands on the wrong side of a rounding boundary:
    every one of the 1024 channels x 256 pointings equals the exact value."""
    g = _geom(oracle_mod)
    bad = 0
    for c in range(0, 1024, 1):
        f_int = 400_000_000 + c * 390_625
        k = oracle_mod.lut(g, float(f_int))
        if c % 37 == 0 or c in (511, 512, 513, 1023):
            ref = [_lut_exact(f_int, m) for m in range(256)]
            bad += int(np.count_nonzero(k != np.array(ref)))
        else:
            # spot-check a stride of pointings elsewhere to keep the test fast
            ms = range(c % 7, 256, 7)
            ref = [_lut_exact(f_int, m) for m in ms]
            bad += int(np.count_nonzero(k[list(ms)] != np.array(ref)))
    assert bad == 0


def test_lut_half_bin_bound_and_aliasing(oracle_mod):
    """Sec. 3.1: the kept bin is the FFT beam nearest the desired pointing.
    Sec. 3.3: spatial aliasing (duplicate bins) appears only above c/(2d)."""
    g = _geom(oracle_mod)
    nb = 512
    f_alias = C0 / (2 * D)
    for c in range(0, 1024, 5):
        f = 400e6 + c * 390625.0
        k = oracle_mod.lut(g, f)
        scale = nb * f * D / C0          # bins per unit sin(theta)
        ks = np.where(k > nb // 2, k - nb, k)   # signed bin
        # unaliased pointings: |sin theta| small enough that the bin stays in range
        ok = np.abs(g.sin_theta_ns * scale) < nb / 2 - 1
        err = np.abs(ks[ok] / scale - g.sin_theta_ns[ok])
        assert np.all(err <= 0.5 / scale + 1e-12)
        n_unique = len(np.unique(k))
        if f < f_alias:
            assert n_unique == 256, (f, n_unique)
    # above the aliasing frequency the clamped set repeats bins
    assert len(np.unique(oracle_mod.lut(g, 600e6))) < 256
    assert len(np.unique(oracle_mod.lut(g, 750e6))) < 256


def test_paper_constants():
    """Table 1 / Sec. 3 rates follow from 384-sample frames and a 16-point DFT."""
    gold = json.load(open(os.path.join(GOLDEN, "table1_and_text.json")))
    frame = 384 * gold["input_time_resolution_s"]["value"]
    assert abs(frame / gold["output_time_resolution_s"]["approx_printed"] - 1) < 1e-3
    sub = gold["input_channel_width_hz"]["value"] / 16
    assert abs(sub / gold["output_channel_width_hz"]["approx_printed"] - 1) < 0.02
    assert 16 * 1024 == gold["output_channels_total"]["value"]
    assert 4 * 256 * 2 == gold["n_inputs"]["value"]
    assert gold["n_feed_ns"]["value"] * gold["padding_factor"]["value"] == \
        gold["fft_beams_before_clamp"]["value"]
    assert 4 * 256 == gold["output_beams"]["value"]
    f_alias = C0 / (2 * gold["feed_spacing_m"]["value"])
    assert abs(f_alias / gold["aliasing_onset_hz"]["approx_printed"] - 1) < 0.01


# ---------------------------------------------------------------- P3 N-S
def test_ns_equals_numpy_fft_zero_padded(oracle_mod):
    """The direct sums equal numpy's FFT of the line zero-padded to 512."""
    rng = np.random.default_rng(3)
    x = rng.integers(-8, 8, 256) + 1j * rng.integers(-8, 8, 256)
    k = rng.integers(0, 512, 300).astype(np.int32)
    y = oracle_mod.ns_beams(x, k, 512)
    ref = np.fft.fft(x, n=512)[k]
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_ns_parseval(oracle_mod):
    rng = np.random.default_rng(4)
    x = rng.normal(size=256) + 1j * rng.normal(size=256)
    y = oracle_mod.ns_beams(x, np.arange(512, dtype=np.int32), 512)
    assert abs(np.sum(np.abs(y) ** 2) / (512 * np.sum(np.abs(x) ** 2)) - 1) < 1e-12


def test_ns_tiny_brute_force(oracle_mod):
    """N = 4 feeds, P = 2: every bin written out term by term."""
    x = np.array([1 + 2j, -3 + 0.5j, 0.25 - 1j, 2 + 2j])
    w = [complex(math.cos(2 * math.pi * r / 8), -math.sin(2 * math.pi * r / 8)) for r in range(8)]
    for k in range(8):
        ref = x[0] * w[0] + x[1] * w[k % 8] + x[2] * w[(2 * k) % 8] + x[3] * w[(3 * k) % 8]
        y = oracle_mod.ns_beams(x, np.array([k], dtype=np.int32), 8)[0]
        assert abs(y - ref) < 1e-12


def test_ns_beam_centre_and_dirichlet_nulls(oracle_mod):
    """Sec. 3.1 beam-centre formula: a plane wave at sin(theta) = k0 c / (N P f d)
    gives |X_k0|^2 = 256^2 |A|^2, exact zeros at k0 +- 2r and the Dirichlet
    pattern |sin(pi*256*delta/512) / sin(pi*delta/512)|^2 elsewhere."""
    f = 600e6
    k0 = 77
    s = k0 * C0 / (512 * f * D)
    n = np.arange(256)
    A = 1.7 - 0.4j
    x = A * np.exp(2j * np.pi * f * n * D * s / C0)
    y = oracle_mod.ns_beams(x, np.arange(512, dtype=np.int32), 512)
    p = np.abs(y) ** 2
    assert abs(p[k0] / (256 ** 2 * abs(A) ** 2) - 1) < 1e-12
    delta = (np.arange(512) - k0)
    even = (delta % 2 == 0) & (delta != 0)
    assert np.all(p[even] < 1e-18 * p[k0])
    odd = delta % 2 == 1
    dir_ = np.abs(np.sin(np.pi * 256 * delta[odd] / 512) / np.sin(np.pi * delta[odd] / 512)) ** 2
    np.testing.assert_allclose(p[odd], dir_ * abs(A) ** 2, rtol=1e-9)


# ---------------------------------------------------------------- P4 E-W
def test_ew_array_factor_closed_form(oracle_mod):
    """Four cylinders 20 m apart: |b_j|^2 for a unit plane wave at u equals
    |sin(4 a / 2) / sin(a / 2)|^2 with a = 2 pi f D (u - sin phi_j) / c0."""
    g = _geom(oracle_mod)
    f = 650e6
    for u in (-0.01, -0.003, 0.0, 0.0021, 0.0105):
        y = np.exp(2j * np.pi * f * g.cyl_x_m * u / C0)
        b = oracle_mod.ew_beams(oracle_mod.ew_weights(g, f), y)
        a = 2 * np.pi * f * 20.0 * (u - g.sin_phi_ew) / C0
        with np.errstate(invalid="ignore", divide="ignore"):
            af = np.where(np.abs(np.sin(a / 2)) < 1e-15, 16.0,
                          (np.sin(2 * a) / np.sin(a / 2)) ** 2)
        np.testing.assert_allclose(np.abs(b) ** 2, af, rtol=1e-9, atol=1e-9)


def test_ew_scaled_unitary_energy(oracle_mod):
    """sin(phi_j) = j c0 / (4 f D) makes W a phased DFT-4: sum_j |b_j|^2 = 4 sum_c |y_c|^2."""
    f = 600e6
    g = _geom(oracle_mod, sin_phi_ew=np.arange(4) * C0 / (4 * f * 20.0))
    rng = np.random.default_rng(5)
    y = rng.normal(size=4) + 1j * rng.normal(size=4)
    b = oracle_mod.ew_beams(oracle_mod.ew_weights(g, f), y)
    assert abs(np.sum(np.abs(b) ** 2) / (4 * np.sum(np.abs(y) ** 2)) - 1) < 1e-12


# ---------------------------------------------------------------- P5 up-channelisation
def test_upchan_tone_and_parseval(oracle_mod):
    """A tone on sub-channel s lands in bin s only; Parseval holds; equals numpy.fft."""
    tau = np.arange(16)
    for s0 in (0, 3, 8, 15):
        b = (2 - 1j) * np.exp(2j * np.pi * s0 * tau / 16)
        u = oracle_mod.upchan(b)
        assert abs(u[s0] - 16 * (2 - 1j)) < 1e-12
        assert np.all(np.abs(np.delete(u, s0)) < 1e-12)
    rng = np.random.default_rng(6)
    b = rng.normal(size=16) + 1j * rng.normal(size=16)
    u = oracle_mod.upchan(b)
    np.testing.assert_allclose(u, np.fft.fft(b), atol=1e-12)
    assert abs(np.sum(np.abs(u) ** 2) / (16 * np.sum(np.abs(b) ** 2)) - 1) < 1e-12


# ---------------------------------------------------------------- whole pipeline
def _brute_force_unit(raw, f, geom_kw, k, sin_phi, cyl_x):
    """Unstaged sum: for each output, |sum over (tau, cyl, feed) of sample x phase|^2
    summed over blocks and pols, no intermediate arrays."""
    NF, NB, NC, NP, NM, NJ, L, T = (geom_kw[n] for n in
                                    ("n_feed", "nb", "n_cyl", "n_pol", "n_beam_ns",
                                     "n_beam_ew", "n_dft", "n_time"))
    out = np.zeros((NJ * NM, L))
    for j in range(NJ):
        for m in range(NM):
            for s in range(L):
                q = (s + L // 2) % L
                for blk in range(T // L):
                    for p in range(NP):
                        acc = 0j
                        for tau in range(L):
                            for c in range(NC):
                                for n in range(NF):
                                    byte = int(raw[blk * L + tau, (c * NF + n) * NP + p])
                                    xv = complex((byte >> 4) - 8, (byte & 15) - 8)
                                    ph = -(n * k[m] / NB + f * cyl_x[c] * sin_phi[j] / C0
                                           + s * tau / L)
                                    acc += xv * complex(math.cos(2 * math.pi * ph),
                                                        math.sin(2 * math.pi * ph))
                        out[j * NM + m, q] += abs(acc) ** 2
    return out


def test_pipeline_tiny_brute_force(oracle_mod):
    kw = dict(n_feed=4, pad=2, n_cyl=2, n_pol=2, n_beam_ns=3, n_beam_ew=2, n_dft=4, n_time=8)
    cyl_x = np.array([-10.0, 10.0])
    sin_theta = np.array([-0.3, 0.05, 0.6])
    sin_phi = np.array([-0.004, 0.007])
    g = oracle_mod.Geometry(**kw, cyl_x_m=cyl_x, sin_theta_ns=sin_theta, sin_phi_ew=sin_phi)
    f = 700e6
    raw = synth.uniform_bytes(11, (1, 1, 8, 16))
    out = oracle_mod.beamform(g, [f], raw)[0, 0]
    k = oracle_mod.lut(g, f)
    # independent Eq. (1) for these three pointings
    k_ref = [math.floor(8 * f * D / C0 * s + 0.5) % 8 for s in sin_theta]
    assert list(k) == k_ref
    ref = _brute_force_unit(raw[0, 0], f, dict(kw, nb=8), k_ref, sin_phi, cyl_x)
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-9)


def test_complex_beams_tiny_brute_force(oracle_mod):
    """The pre-detection beams (complex, before |.|^2) against the same unstaged sum:
    this pins the phases, which detection discards."""
    kw = dict(n_feed=4, pad=2, n_cyl=2, n_pol=2, n_beam_ns=3, n_beam_ew=2, n_dft=4, n_time=8)
    cyl_x = np.array([-10.0, 10.0])
    sin_theta = np.array([-0.3, 0.05, 0.6])
    sin_phi = np.array([-0.004, 0.007])
    g = oracle_mod.Geometry(**kw, cyl_x_m=cyl_x, sin_theta_ns=sin_theta, sin_phi_ew=sin_phi)
    f = 700e6
    raw = synth.uniform_bytes(13, (8, 16))
    got = oracle_mod.beams_unit(g, f, raw)                    # [blk][s][p][j][m]
    k = [math.floor(8 * f * D / C0 * st + 0.5) % 8 for st in sin_theta]
    ref = np.zeros_like(got)
    for blk in range(2):
        for s in range(4):
            for p in range(2):
                for j in range(2):
                    for m in range(3):
                        acc = 0j
                        for tau in range(4):
                            for c in range(2):
                                for n in range(4):
                                    byte = int(raw[blk * 4 + tau, (c * 4 + n) * 2 + p])
                                    xv = complex((byte >> 4) - 8, (byte & 15) - 8)
                                    ph = -(n * k[m] / 8 + f * cyl_x[c] * sin_phi[j] / C0 + s * tau / 4)
                                    acc += xv * complex(math.cos(2 * math.pi * ph),
                                                        math.sin(2 * math.pi * ph))
                        ref[blk, s, p, j, m] = acc
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-9)
    # detection of these beams is the pipeline's output
    pw = (np.abs(got) ** 2).sum(axis=(0, 2))                   # [s][j][m]
    out = oracle_mod.beamform_unit(g, f, raw)                  # [j*3+m][q]
    for s in range(4):
        assert np.allclose(out[:, (s + 2) % 4], pw[s].reshape(-1), rtol=1e-12)


def test_pipeline_energy_even_odd_bins(oracle_mod):
    """Run once keeping the 256 even bins and once the 256 odd bins, with the
    scaled-unitary E-W directions: the summed output equals 16 * 4 * 512 * sum|x|^2
    (Parseval through N-S, E-W and the time DFT)."""
    f = 600e6
    g = _geom(oracle_mod, sin_phi_ew=np.arange(4) * C0 / (4 * f * 20.0))
    raw = synth.uniform_bytes(12, (1, 1, 384, 2048))
    even = (2 * np.arange(256)).astype(np.int32)[None]
    odd = even + 1
    tot = (oracle_mod.beamform(g, [f], raw, lut_override=even).sum()
           + oracle_mod.beamform(g, [f], raw, lut_override=odd).sum())
    x = oracle_mod.decode(raw)
    assert abs(tot / (16 * 4 * 512 * np.sum(np.abs(x) ** 2)) - 1) < 1e-11


def test_noise_mean_statistics(oracle_mod):
    """Noise-only output mean = 16 * 24 * 2 * 1024 * E|x|^2, with E|x|^2 of
    N(0, 2.5^2) rounded and clipped to +-7 from the normal CDF; each output is
    a Gamma(48) sum (relative spread 1/sqrt(48))."""
    g = _geom(oracle_mod)
    raw = synth.noise_frames(21, 2, 2)
    out = oracle_mod.beamform(g, [450e6, 720e6], raw)
    k = np.arange(-7, 8)
    sig = 2.5
    p = norm.cdf((k + 0.5) / sig) - norm.cdf((k - 0.5) / sig)
    p[0] = norm.cdf(-6.5 / sig)
    p[-1] = 1 - norm.cdf(6.5 / sig)
    e_x2 = 2 * np.sum(p * k * k)
    expect = 16 * 24 * 2 * 1024 * e_x2
    n = out.size
    assert abs(out.mean() / expect - 1) < 6 / math.sqrt(48 * n)
    assert abs(out.std() / out.mean() - 1 / math.sqrt(48)) < 0.01


def _predicted_beam(oracle_mod, g, f, sin_theta, phi_deg):
    """Strongest beam predicted from FP64 closed-form array factors (no data)."""
    u = math.sin(math.radians(phi_deg))
    v = math.cos(math.radians(phi_deg)) * sin_theta
    k = oracle_mod.lut(g, f)
    kt = 512 * f * D * v / C0
    delta = kt - k
    ns = (np.sin(np.pi * 256 * delta / 512) / (256 * np.sin(np.pi * delta / 512))) ** 2
    a = 2 * np.pi * f * 20.0 * (u - g.sin_phi_ew) / C0
    ew = (np.sin(2 * a) / (4 * np.sin(a / 2))) ** 2
    resp = ew[:, None] * ns[None, :]
    return int(np.argmax(resp)), resp


def test_point_source_peaks_in_predicted_beam(oracle_mod):
    """Noisy 600 MHz frame with a source at theta = 20 deg, phi = 0.5 deg, tone at the
    channel centre: the strongest output is the beam the geometry predicts, at the
    centre sub-channel (q = 8, the DC bin after the centre shift)."""
    g = _geom(oracle_mod)
    c = synth.config0()
    out = oracle_mod.beamform(g, c["freqs"], c["raw"])[0, 0]
    beam, _ = _predicted_beam(oracle_mod, g, 600e6, math.sin(math.radians(20)), 0.5)
    b, q = np.unravel_index(np.argmax(out), out.shape)
    assert (b, q) == (beam, 8)
    assert beam == 3 * 256 + 171
    assert out[b, q] > 1000 * np.median(out)


def test_tracking_beam_follows_drifting_source(oracle_mod):
    """Sec. 3.1 (E-W beams static or tracking): a source drifting 0.3 deg E-W per frame
    stays at the peak of the beam whose direction follows it, while with static beams
    its power in that beam falls as the closed-form 4-cylinder array factor predicts
    and the peak moves to the next E-W beam."""
    f = 600e6
    raw, phi = synth.drifting_source(51, [f], 3)
    track = synth.tracking_pointings(phi)
    m = 171                                   # N-S beam of theta = 20 deg at 600 MHz
    x = (np.arange(4) - 1.5) * 20.0
    u_src = np.sin(np.deg2rad(phi))
    static = oracle_mod.beamform(_geom(oracle_mod), [f], raw)
    for fr in range(3):
        tr = oracle_mod.beamform(_geom(oracle_mod, sin_phi_ew=track[fr]), [f], raw[fr:fr + 1])
        b, q = np.unravel_index(np.argmax(tr[0, 0]), tr[0, 0].shape)
        assert (b, q) == (2 * 256 + m, 8)
        af = lambda s: abs(np.exp(2j * np.pi * f * x * (u_src[fr] - s) / C0).sum()) ** 2
        ratio = static[fr, 0, 2 * 256 + m, 8] / tr[0, 0, 2 * 256 + m, 8]
        expect = af(math.sin(math.radians(0.2))) / af(track[fr, 2])
        assert abs(ratio - expect) < 0.02 * max(expect, 0.05)
    # static beams: the peak E-W beam is the array factor's argmax (at 0.8 deg the
    # 1.43 deg grating-lobe spacing of 20 m cylinders at 600 MHz favours -0.6 deg)
    sphi = np.sin(np.deg2rad((np.arange(4) - 1.5) * 0.4))
    for fr in range(3):
        af = [abs(np.exp(2j * np.pi * f * x * (u_src[fr] - s) / C0).sum()) for s in sphi]
        j_pred = int(np.argmax(af))
        assert int(np.argmax(static[fr, 0, :, 8].reshape(4, 256)[:, m])) == j_pred
        assert j_pred == [2, 3, 0][fr]


def test_alias_lands_where_geometry_says(oracle_mod):
    """Sec. 3.3: above ~490 MHz a source also appears in an aliased beam; a 26 deg
    source at 760 MHz aliases to sin(theta) = sin(26) - c/(f d) (about -59 deg)."""
    g = _geom(oracle_mod)
    f = 760e6
    st = math.sin(math.radians(26.0))
    src = [synth.Source(sin_theta=st, phi_deg=0.0, amp=2.0)]
    raw = np.empty((1, 1, 384, 2048), dtype=np.uint8)
    synth.channel_frames(np.random.default_rng(0), f, 1, src, raw[:, 0], sigma=0.0)
    out = oracle_mod.beamform(g, [f], raw)[0, 0].sum(axis=1).reshape(4, 256).sum(axis=0)
    alias = st - C0 / (f * D)
    m_main = int(np.argmax(np.where(g.sin_theta_ns > 0, out, 0)))
    m_alias = int(np.argmax(np.where(g.sin_theta_ns < 0, out, 0)))
    assert abs(g.sin_theta_ns[m_main] - st) < 2 / 128
    assert abs(g.sin_theta_ns[m_alias] - alias) < 2 / 128
    gold = json.load(open(os.path.join(GOLDEN, "table1_and_text.json")))
    lo, hi = gold["alias_extent_deg_for_26deg_source"]["approx_printed"]
    # across the aliasing band the alias sweeps the range the paper reports
    f_edge = C0 / (D * (1 + st))
    ang = [math.degrees(math.asin(max(-1.0, st - C0 / (ff * D)))) for ff in (f_edge, 800e6)]
    assert abs(ang[0] - lo) < 3 and abs(ang[1] - hi) < 3


def test_dispersed_pulse_sweeps_down_in_subchannel(oracle_mod):
    """Sec. 3.2: dispersion delays lower frequencies, 4.148808 ms DM (f/GHz)^-2.  Inside one
    600 MHz channel a DM-500 pulse crosses the 16 sub-channels from the top (q = 15) to
    the bottom (q = 0) in about 7 ms; the oracle's sub-channel order must show that."""
    f = float(synth.chan_freq_hz(512))
    sky = synth.Config4Sky(rfi=(), pulse_sin_theta=0.3, pulse_phi_deg=0.0, pulse_amp=3.0)
    nu = (np.arange(16) - 8) * synth.SUBCHAN_HZ
    arr = synth.dispersion_delay_s(f + nu, 500) - synth.dispersion_delay_s(800e6, 500)
    frame_s = 384 * 2.56e-6
    # q = 0 .. 15 spans 15 sub-channel spacings: d/df of the delay law times 15 x 24.4 kHz
    slope = 2 * synth.DM_DELAY_S * 500 * (15 * synth.SUBCHAN_HZ / 1e9) / (f / 1e9) ** 3
    assert abs((arr[0] - arr[15]) / slope - 1) < 0.02
    f0 = int(arr[15] / frame_s)
    frames = np.arange(f0, f0 + 9)
    raw = synth.config4_frames(5, [512], frames, sky=sky)
    out = oracle_mod.beamform(oracle_mod.Geometry(), [f], raw)   # [frame][1][beam][q]
    per_q = out[:, 0].sum(axis=1)
    base = np.median(per_q)
    qs = [int(np.argmax(per_q[k])) for k in range(len(frames)) if per_q[k].max() > 1.5 * base]
    assert len(qs) >= 6
    assert all(a >= b for a, b in zip(qs, qs[1:]))        # moves down in frequency
    assert qs[0] >= 13 and qs[-1] <= 2
    # and it is seen in the beam of its direction
    k = len(frames) // 2
    beam = int(np.argmax(out[k, 0].sum(axis=1)))
    g = oracle_mod.Geometry()
    assert abs(g.sin_theta_ns[beam % 256] - 0.3) < 3 / 128


# ---------------------------------------------------------------- 8-bit output
def test_rescale_u8_definition(oracle_mod):
    """Sec. 3 and Table 1 put the output in 8-bit integers without a rule; the reading is
    code = clamp(rint(P scale + offset), 0, 255) decided in FP32.  Pinned by ties (round
    half to even), saturation at both ends, NaN, and an independent float32 evaluation
    on seeded values (product exact in float64, one rounding to float32)."""
    P = np.array([2.5, 3.5, -0.5, 0.5, 1.5, 254.5, 255.5, 1e30, -1e30, np.nan, 0.49999997])
    assert oracle_mod.rescale_u8(P, 1.0, 0.0).tolist() == [2, 4, 0, 0, 2, 254, 255, 255, 0, 0, 0]
    assert oracle_mod.rescale_u8([10.0], 0.0, 7.0).tolist() == [7]
    rng = np.random.default_rng(81)
    P = rng.uniform(0, 4e7, 20000)
    sc = rng.uniform(2e-6, 1e-5, P.size).astype(np.float32)
    of = rng.uniform(-40, 40, P.size).astype(np.float32)
    t = (np.float32(P).astype(np.float64) * sc.astype(np.float64) + of.astype(np.float64))
    t32 = t.astype(np.float32)
    ref = np.clip(np.rint(t32), 0, 255).astype(np.uint8)
    got = oracle_mod.rescale_u8(P, sc, of)
    assert 0 < (ref == 0).sum() and 0 < (ref == 255).sum()
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------- 128-point up-channelisation
def test_group_bins_brute_force(oracle_mod):
    """Coarse sub-channel q sums the 8 centre-shifted fine bins 8q - 4 .. 8q + 3 (mod 128)."""
    fine = np.random.default_rng(5).uniform(0, 1, (3, 7, 128))
    ref = np.roll(fine, 4, axis=-1).reshape(3, 7, 16, 8).sum(-1)
    assert np.allclose(oracle_mod.group_bins(fine, 8), ref, rtol=1e-15, atol=0)
    one = np.zeros(128)
    for qf in range(128):
        one[:] = 0
        one[qf] = 1
        assert int(np.argmax(oracle_mod.group_bins(one, 8))) == ((qf + 4) // 8) % 16


def test_upchan128_dc_tone_and_parseval(oracle_mod):
    """Sec. 3 and Sec. 3.2: 128-point DFTs of 128-sample blocks, integrated to 16 sub-
    channels.  A tone at the channel centre (constant integer samples, so exact) puts
    everything in sub-channel 8 with 3 x 128^2 / (24 x 16^2) = 8 times the 16-point
    power; for any input the total over sub-channels is 8 times the 16-point total
    (Parseval: L sum |x|^2 per block)."""
    g = _geom(oracle_mod)
    raw = np.empty((1, 1, 384, 2048), np.uint8)
    synth.channel_frames(None, 600e6, 1, [synth.Source(0.3, 0.2, 3.0)], raw[:, 0], sigma=0.0)
    o16 = oracle_mod.beamform(g, [600e6], raw)[0, 0]
    o128 = oracle_mod.beamform_upchan128(g, [600e6], raw)[0, 0]
    assert np.allclose(o128[:, 8], 8 * o16[:, 8], rtol=1e-12, atol=0)
    assert np.abs(np.delete(o128, 8, axis=1)).max() < 1e-9 * o128.max()
    rnd = synth.uniform_bytes(6, (1, 1, 384, 2048))
    t16 = oracle_mod.beamform(g, [450e6], rnd)[0, 0].sum(axis=1)
    t128 = oracle_mod.beamform_upchan128(g, [450e6], rnd)[0, 0].sum(axis=1)
    assert np.allclose(t128, 8 * t16, rtol=1e-12, atol=0)


# Tones on exact fine-channel frequencies: fine channel spacing 390.625 kHz / 128.
FINE_HZ = synth.CHAN_BW_HZ / 128
# (sub-channel whose centre the tone is placed near, offset in fine channels)
TONE_CASES = [(3, -5), (3, -4), (3, -1), (3, 0), (3, 3), (3, 4), (11, 8), (11, 11),
              (11, 12), (0, -4), (15, 3)]


def tone_frames(cases, f_hz, amp=6.0):
    """One noiseless frame per case: a point source whose tone sits `off` fine
    channels from the centre of sub-channel q (offset (q - 8) x 24.4 kHz from the
    channel centre).  A tone on a fine-channel frequency completes a whole number
    of cycles per 128-sample block, so it falls in one fine channel."""
    raw = np.empty((1, len(cases), 384, 2048), np.uint8)
    for i, (q, off) in enumerate(cases):
        nu = (q - 8) * synth.SUBCHAN_HZ + off * FINE_HZ
        src = [synth.Source(sin_theta=0.3, phi_deg=0.2, amp=amp, tone_hz=nu, phase=0.4)]
        synth.channel_frames(None, f_hz, 1, src, raw[:, i], sigma=0.0)
    return raw


def expected_subchannel(nu_hz):
    """The sub-channel a tone at offset nu from the channel centre belongs to in the
    128-point form, from frequencies alone: each sub-channel collects the 8 fine
    channels nearest its centre; 8 is even, so the group's own centre sits half a
    fine channel (1.5 kHz) below the sub-channel's nominal centre (q - 8) x 24.4 kHz.
    The tone therefore goes to the sub-channel whose group centre is nearest."""
    centres = (np.arange(16) - 8) * synth.SUBCHAN_HZ - 0.5 * FINE_HZ
    d = (nu_hz - centres + synth.CHAN_BW_HZ / 2) % synth.CHAN_BW_HZ - synth.CHAN_BW_HZ / 2
    return int(np.argmin(np.abs(d)))


def test_upchan128_tone_grouping(oracle_mod):
    """Sec. 3 and Sec. 3.2 (fine channels of 3 kHz summed to 24 kHz): tones at fine-
    channel offsets -5 .. +12 from several sub-channel centres land, with more than
    99 % of their power, in the sub-channel whose 8-fine-channel group holds their
    frequency.  Offsets -4 .. +3 stay in the sub-channel they were placed near, +4,
    +8 and +11 move one up, +12 two, -5 one down, so a grouping shifted or mirrored
    by even one fine channel fails."""
    f = 600e6
    raw = tone_frames(TONE_CASES, f)
    out = oracle_mod.beamform_upchan128(_geom(oracle_mod), [f] * len(TONE_CASES), raw)
    tot = out[0].sum(axis=1)  # [case][q], all beams
    for i, (q, off) in enumerate(TONE_CASES):
        nu = (q - 8) * synth.SUBCHAN_HZ + off * FINE_HZ
        want = expected_subchannel(nu)
        assert want == (q + (off + 4) // 8) % 16  # -4 .. +3 keep q, +4 .. +11 go up one
        assert int(np.argmax(tot[i])) == want, (q, off, tot[i])
        assert tot[i, want] >= 0.99 * tot[i].sum(), (q, off)


def test_frequency_summed_map_against_closed_form(oracle_mod):
    """Sec. 3.3 / Fig. 3: the oracle's beams summed over channels (every 32nd channel of
    the band, noiseless 4-bit frames of a source at 26 deg N-S, 0.2 deg E-W) have the
    shape of the closed-form N-S x E-W array factors summed over the same channels:
    peak in the source's pointing and E-W beam, alias south of zenith at the predicted
    fraction of the main beam.  A dropped E-W weight, a mis-signed N-S phase or a wrong
    bin would move or reshape the map."""
    f = synth.chan_freq_hz(np.arange(8, 1024, 32))
    s26 = math.sin(math.radians(26.0))
    raw = synth.point_source_frames(f, s26, phi_deg=0.2)
    out = oracle_mod.beamform(oracle_mod.Geometry(), f, raw)[0]
    m_map = out.sum(axis=(0, 2)).reshape(4, 256)
    sin_m = (np.arange(256) - 127.5) / 128
    v = math.cos(math.radians(0.2)) * s26
    kappa = 512 * f * D * v / C0
    bins = np.mod(np.floor(512 * f[:, None] * D * sin_m[None, :] / C0 + 0.5).astype(np.int64), 512)
    n = np.arange(256)
    af_ns = np.abs(np.exp(2j * np.pi * (kappa[:, None, None] - bins[:, :, None]) * n / 512)
                   .sum(axis=2)) ** 2
    x = (np.arange(4) - 1.5) * 20.0
    sphi = np.sin(np.deg2rad((np.arange(4) - 1.5) * 0.4))
    u = math.sin(math.radians(0.2))
    af_ew = np.abs(np.exp(2j * np.pi * f[:, None, None] * x[None, None, :] * (u - sphi)[None, :, None]
                          / C0).sum(axis=2)) ** 2
    pred = np.einsum("fj,fm->jm", af_ew, af_ns)
    assert np.unravel_index(np.argmax(m_map), m_map.shape) == (2, 184)
    assert np.abs(m_map / m_map.max() - pred / pred.max()).max() <= 0.005
    south = sin_m < 0
    r, rp = m_map[2][south].max() / m_map.max(), pred[2][south].max() / pred.max()
    assert 0.005 < rp < 0.1 and abs(r - rp) <= 0.05 * rp
