"""Seeded synthetic baseband for the hybrid beamformer.

This module only simulates what the F-engine would deliver: Gaussian noise
plus monochromatic point sources seen by the CHIME array, quantised to 4+4-bit
offset-binary complex samples.  It holds no beamforming arithmetic and is
shared by the oracle tests and the GPU tests/benchmark as their common input.

Array model (paper Sec. 1): four cylinders, each with 256 dual-polarisation
feeds at 0.3048 m N-S spacing; cylinders are 20 m wide and sit side by side,
so cylinder c is at x_c = (c - 1.5) * 20 m (east positive) and feed n at
y_n = n * 0.3048 m (north positive).  A source in direction (u, v) =
(sin phi, cos phi * sin theta) -- phi the E-W offset, theta the N-S zenith
angle -- reaches input (c, n, p) with phase exp(+2 pi i f (x_c u + y_n v)/c0).

Byte layout: ``raw[frame][chan][t][i]`` with t < 384 samples of 2.56 us and
i = (cyl * 256 + feed) * 2 + pol; byte = ((re + 8) << 4) | (im + 8).
Quantisation: sigma applies per real component, values are rounded half to
even and clipped to [-7, 7]; sources are added before rounding.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

C0 = 299_792_458.0
FEED_SPACING_M = 0.3048
CYL_SPACING_M = 20.0
N_CYL, N_FEED, N_POL = 4, 256, 2
N_INPUTS = N_CYL * N_FEED * N_POL
N_TIME = 384                 # samples per 0.983 ms frame
SAMPLE_DT = 2.56e-6          # s
CHAN_BW_HZ = 390_625.0
F_BOTTOM_HZ = 400e6
SUBCHAN_HZ = CHAN_BW_HZ / 16.0
SIGMA = 2.5


def chan_freq_hz(c_idx) -> np.ndarray:
    """Centre frequency of F-engine channel c_idx (1024 channels, 400-800 MHz)."""
    return F_BOTTOM_HZ + np.asarray(c_idx, dtype=np.float64) * CHAN_BW_HZ


def encode(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Integers in [-8, 7] -> offset-binary 4+4-bit bytes (high nibble real)."""
    return (((re.astype(np.int16) + 8) << 4) | (im.astype(np.int16) + 8)).astype(np.uint8)


def input_positions():
    """(x, y) in metres of each of the 2048 inputs, in input order."""
    i = np.arange(N_INPUTS)
    cyl = i // (N_FEED * N_POL)
    feed = (i // N_POL) % N_FEED
    x = (cyl - (N_CYL - 1) / 2.0) * CYL_SPACING_M
    y = feed * FEED_SPACING_M
    return x, y


@dataclass
class Source:
    """Monochromatic point source.  tone_hz is the offset from the channel centre."""
    sin_theta: float         # N-S zenith angle sine
    phi_deg: float           # E-W offset
    amp: float               # amplitude per real+imag sample
    tone_hz: float = 0.0
    phase: float = 0.0


def _spatial(freq_hz: float, sources) -> np.ndarray:
    x, y = input_positions()
    rows = []
    for s in sources:
        phi = np.deg2rad(s.phi_deg)
        u = np.sin(phi)
        v = np.cos(phi) * s.sin_theta
        rows.append(np.exp(2j * np.pi * freq_hz * (x * u + y * v) / C0))
    return np.asarray(rows, dtype=np.complex128).reshape(len(sources), N_INPUTS)


def _temporal(t_abs: np.ndarray, sources) -> np.ndarray:
    cols = [s.amp * np.exp(1j * (2 * np.pi * s.tone_hz * t_abs * SAMPLE_DT + s.phase))
            for s in sources]
    return np.asarray(cols, dtype=np.complex128).reshape(len(sources), t_abs.size).T


def channel_frames(rng: np.random.Generator, freq_hz: float, n_frames: int, sources,
                   out: np.ndarray, sigma: float = SIGMA, frame0: int = 0) -> None:
    """Fill out[f][t][i] (u8) for frames frame0 .. frame0+n_frames-1 of one channel.

    Draw order per frame: real noise [384][2048], then imaginary noise (nothing is
    drawn when sigma = 0).
    """
    spat = _spatial(freq_hz, sources) if sources else None
    for f in range(n_frames):
        if sigma == 0.0:      # noiseless: nothing drawn (the values would be zeroed)
            re = np.zeros((N_TIME, N_INPUTS), dtype=np.float32)
            im = np.zeros((N_TIME, N_INPUTS), dtype=np.float32)
        else:
            re = rng.standard_normal((N_TIME, N_INPUTS), dtype=np.float32)
            im = rng.standard_normal((N_TIME, N_INPUTS), dtype=np.float32)
            re *= sigma
            im *= sigma
        if spat is not None:
            t_abs = (frame0 + f) * N_TIME + np.arange(N_TIME, dtype=np.float64)
            sig = _temporal(t_abs, sources) @ spat
            re += sig.real.astype(np.float32)
            im += sig.imag.astype(np.float32)
        np.rint(re, out=re)
        np.rint(im, out=im)
        np.clip(re, -7, 7, out=re)
        np.clip(im, -7, 7, out=im)
        out[f] = encode(re, im)


def config0():
    """One channel at 600 MHz, one frame, one source at theta=20 deg, phi=0.5 deg, A=3."""
    c_idx = np.array([512])
    freqs = chan_freq_hz(c_idx)
    src = [Source(sin_theta=float(np.sin(np.deg2rad(20.0))), phi_deg=0.5, amp=3.0)]
    rng = np.random.Generator(np.random.PCG64(1000))
    raw = np.empty((1, 1, N_TIME, N_INPUTS), dtype=np.uint8)
    channel_frames(rng, float(freqs[0]), 1, src, raw[:, 0])
    return {"name": "config0", "c_idx": c_idx, "freqs": freqs, "raw": raw,
            "sources": {0: src}}


def random_sources(rng: np.random.Generator, n: int, amp: float):
    """n sources inside the primary beam: sin(theta) ~ U[-sin 60, sin 60] (the ~120 deg
    N-S field of view), phi ~ U[-0.65, 0.65] deg (half the narrowest 1.3 deg E-W field),
    tone on a seeded 24.4 kHz sub-channel centre, random phase."""
    s60 = np.sin(np.deg2rad(60.0))
    out = []
    for _ in range(n):
        st = rng.uniform(-s60, s60)
        ph = rng.uniform(-0.65, 0.65)
        q = int(rng.integers(0, 16))
        pha = rng.uniform(0.0, 2 * np.pi)
        out.append(Source(sin_theta=float(st), phi_deg=float(ph), amp=amp,
                          tone_hz=(q - 8) * SUBCHAN_HZ, phase=float(pha)))
    return out


def config1(n_frames: int = 128, n_sources: int = 8, seed: int = 1001,
            c_idx=(128, 384, 640, 896)):
    """One node's share: 4 channels over 400-800 MHz, n_frames frames each, noise plus
    n_sources point sources of amplitude 1.5 (same sources in every channel)."""
    c_idx = np.asarray(c_idx)
    freqs = chan_freq_hz(c_idx)
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(1 + len(c_idx))
    srcs = random_sources(np.random.Generator(np.random.PCG64(kids[0])), n_sources, 1.5)
    raw = np.empty((n_frames, len(c_idx), N_TIME, N_INPUTS), dtype=np.uint8)
    for ci in range(len(c_idx)):
        rng = np.random.Generator(np.random.PCG64(kids[1 + ci]))
        buf = np.empty((n_frames, N_TIME, N_INPUTS), dtype=np.uint8)
        channel_frames(rng, float(freqs[ci]), n_frames, srcs, buf)
        raw[:, ci] = buf
    return {"name": "config1", "c_idx": c_idx, "freqs": freqs, "raw": raw,
            "sources": srcs}


def noise_frames(seed: int, n_frames: int, n_chan: int, sigma: float = SIGMA) -> np.ndarray:
    """Noise-only bytes [n_frames][n_chan][384][2048] (statistics tests, ragged shapes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    raw = np.empty((n_frames, n_chan, N_TIME, N_INPUTS), dtype=np.uint8)
    for c in range(n_chan):
        buf = np.empty((n_frames, N_TIME, N_INPUTS), dtype=np.uint8)
        channel_frames(rng, 600e6, n_frames, [], buf, sigma=sigma)
        raw[:, c] = buf
    return raw


def drifting_source(seed: int, freqs, n_frames: int, phi0_deg: float = 0.2,
                    rate_deg: float = 0.3, sin_theta: float = float(np.sin(np.deg2rad(20.0))),
                    amp: float = 3.0):
    """Noise plus one point source that moves E-W by rate_deg per frame (tone at
    the channel centre).  Returns raw u8 [n_frames][n_chan][384][2048] and the
    source's E-W offset in degrees per frame.  One seeded stream per channel."""
    freqs = np.atleast_1d(np.asarray(freqs, dtype=np.float64))
    raw = np.empty((n_frames, len(freqs), N_TIME, N_INPUTS), np.uint8)
    phi = phi0_deg + rate_deg * np.arange(n_frames)
    kids = np.random.SeedSequence(seed).spawn(len(freqs))
    for ci, f in enumerate(freqs):
        rng = np.random.default_rng(kids[ci])
        for fr in range(n_frames):
            channel_frames(rng, float(f), 1, [Source(sin_theta, float(phi[fr]), amp)],
                           raw[fr:fr + 1, ci], frame0=fr)
    return raw, phi


def point_source_frames(freqs, sin_theta, phi_deg: float = 0.0, amp: float = 6.0) -> np.ndarray:
    """One noiseless frame per channel slot: slot i at freqs[i] sees one point
    source at sin_theta[i] (a scalar applies to every slot), E-W offset phi_deg,
    tone at the channel centre.  Returns u8 [1][n][384][2048]."""
    freqs = np.atleast_1d(np.asarray(freqs, dtype=np.float64))
    st = np.broadcast_to(np.asarray(sin_theta, dtype=np.float64), freqs.shape)
    raw = np.empty((1, len(freqs), N_TIME, N_INPUTS), np.uint8)
    for i, f in enumerate(freqs):
        channel_frames(None, float(f), 1, [Source(float(st[i]), phi_deg, amp)], raw[:, i],
                       sigma=0.0)
    return raw


def tracking_pointings(phi_src_deg, lead_beam: int = 2, spacing_deg: float = 0.4) -> np.ndarray:
    """E-W directions sin(phi_j) per frame for four beams spaced spacing_deg
    apart whose beam lead_beam sits on the source offset phi_src_deg[frame]."""
    phi_src = np.atleast_1d(np.asarray(phi_src_deg, dtype=np.float64))
    j = np.arange(4)
    deg = (j[None, :] - lead_beam) * spacing_deg + phi_src[:, None]
    return np.sin(np.deg2rad(deg))


def uniform_bytes(seed: int, shape) -> np.ndarray:
    """Every byte value equally likely, -8 included (exercises the full decode range)."""
    return np.random.Generator(np.random.PCG64(seed)).integers(0, 256, size=shape,
                                                              dtype=np.uint8)


JOIN, LEAVE = 1, 2


def churn_events(seed: int, n_frames: int, n_ids: int = 1024, initial: int = 64,
                 rate_join=0.02, rate_leave=0.02, lo: int = 16, hi: int = 128):
    """Seeded channel churn for the serving loop: frame 0 joins `initial` channel ids drawn
    from [0, n_ids); then per frame Poisson(rate_join) joins and Poisson(rate_leave) leaves,
    ids drawn uniformly from the inactive / active sets.  Events that would take the active
    count outside [lo, hi] are counted in `clamped` and not emitted.  Each rate is a number
    or a per-frame sequence of length n_frames.
    Returns (events [(frame, op, id, freq_hz)], clamped)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rj = np.broadcast_to(np.asarray(rate_join, dtype=np.float64), (n_frames,))
    rl = np.broadcast_to(np.asarray(rate_leave, dtype=np.float64), (n_frames,))
    active = set(int(c) for c in rng.choice(n_ids, size=initial, replace=False))
    events = [(0, JOIN, c, float(chan_freq_hz(c))) for c in sorted(active)]
    clamped = 0
    for f in range(1, n_frames):
        nj = int(rng.poisson(rj[f]))
        nl = int(rng.poisson(rl[f]))
        for _ in range(nl):
            if len(active) <= lo:
                clamped += 1
                continue
            c = int(rng.choice(sorted(active)))
            active.remove(c)
            events.append((f, LEAVE, c, 0.0))
        for _ in range(nj):
            if len(active) >= hi:
                clamped += 1
                continue
            free = sorted(set(range(n_ids)) - active)
            c = int(rng.choice(free))
            active.add(c)
            events.append((f, JOIN, c, float(chan_freq_hz(c))))
    return events, clamped


def churn_rates_to_clamps(n_frames: int, fast: float = 0.05, slow: float = 0.01):
    """Per-frame (join, leave) Poisson rates that drive the active count up, then
    down, then up again (net +-0.04 channels per frame over quarters, a half and a
    quarter of the run), so that a serving run from 120 channels reaches both the
    128-channel and the 16-channel clamp."""
    f = np.arange(n_frames)
    down = (f >= n_frames // 4) & (f < 3 * n_frames // 4)
    return np.where(down, slow, fast), np.where(down, fast, slow)


def frame_pool(seed: int, n_distinct: int, sigma: float = SIGMA, freq_hz: float = 600e6,
               n_sources: int = 2) -> np.ndarray:
    """n_distinct seeded frames [n][384][2048] (noise plus a few point sources) used to fill
    serving-loop input rings."""
    ss = np.random.SeedSequence(seed)
    a, b = ss.spawn(2)
    srcs = random_sources(np.random.Generator(np.random.PCG64(a)), n_sources, 1.5)
    out = np.empty((n_distinct, N_TIME, N_INPUTS), dtype=np.uint8)
    channel_frames(np.random.Generator(np.random.PCG64(b)), freq_hz, n_distinct, srcs, out,
                   sigma=sigma)
    return out


# ---------------------------------------------------------------- config 4 sky
DM_DELAY_S = 4.148808e-3   # cold-plasma dispersion delay constant, s GHz^2 / (pc cm^-3)


def dispersion_delay_s(f_hz, dm: float) -> np.ndarray:
    """Delay relative to infinite frequency: 4.148808 ms * DM * (f / GHz)^-2."""
    return DM_DELAY_S * dm * (np.asarray(f_hz, dtype=np.float64) / 1e9) ** -2


def sweep_c_idx(n_chan: int) -> np.ndarray:
    """n_chan channels spread over the band: c_idx_i = floor((i + 1/2) * 1024 / n_chan)."""
    return np.floor((np.arange(n_chan) + 0.5) * 1024 / n_chan).astype(np.int64)


@dataclass
class Config4Sky:
    dm: float = 500.0
    width_s: float = 1e-3
    pulse_amp: float = 2.0          # per sub-channel component inside the pulse
    pulse_sin_theta: float = 0.25
    pulse_phi_deg: float = 0.2
    t_arrive_800_s: float = 0.0     # arrival time at 800 MHz
    rfi: tuple = ()                 # ((c_idx, sub-channel q, amplitude), ...)


def config4_sky(seed: int, c_idx) -> Config4Sky:
    """Seeded config-4 sky: the DM-500 1 ms pulse in one direction and 5 RFI tones at
    seeded (channel, sub-channel) of the given channel set, amplitude 2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c_idx = np.asarray(c_idx)
    rfi = tuple((int(c_idx[rng.integers(0, len(c_idx))]), int(rng.integers(0, 16)), 2.0)
                for _ in range(5))
    return Config4Sky(pulse_sin_theta=float(rng.uniform(-0.5, 0.5)),
                      pulse_phi_deg=float(rng.uniform(-0.5, 0.5)), rfi=rfi)


def config4_frames(seed: int, c_idx, frames, sky: Config4Sky | None = None,
                   sigma: float = SIGMA) -> np.ndarray:
    """Bytes [len(frames)][len(c_idx)][384][2048]: noise + RFI tones (identical phase on
    every input) + the dispersed pulse.  The pulse is built per 24.4 kHz sub-channel:
    sub-channel q of channel f arrives at the cold-plasma delay of f + (q - 8) * 24.4 kHz
    (relative to 800 MHz) and, inside its 1 ms width, carries a complex Gaussian amplitude
    per 16-sample block placed on that sub-channel's frequency (an inverse 16-point DFT
    of the block's sub-channel amplitudes)."""
    c_idx = np.asarray(c_idx)
    frames = np.asarray(frames)
    sky = sky or config4_sky(seed, c_idx)
    x, y = input_positions()
    out = np.empty((len(frames), len(c_idx), N_TIME, N_INPUTS), dtype=np.uint8)
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(len(c_idx))
    tau = np.arange(16)
    q = np.arange(16)
    nu = (q - 8) * SUBCHAN_HZ
    for ci, c in enumerate(c_idx):
        f = float(chan_freq_hz(c))
        rng = np.random.Generator(np.random.PCG64(kids[ci]))
        u = np.sin(np.deg2rad(sky.pulse_phi_deg))
        v = np.cos(np.deg2rad(sky.pulse_phi_deg)) * sky.pulse_sin_theta
        spat = np.exp(2j * np.pi * f * (x * u + y * v) / C0)
        t_arr = sky.t_arrive_800_s + dispersion_delay_s(f + nu, sky.dm) - dispersion_delay_s(800e6, sky.dm)
        tones = [(qq, a) for (cc, qq, a) in sky.rfi if cc == c]
        for k, fr in enumerate(frames):
            re = rng.standard_normal((N_TIME, N_INPUTS), dtype=np.float32) * sigma
            im = rng.standard_normal((N_TIME, N_INPUTS), dtype=np.float32) * sigma
            t_blk = (fr * N_TIME + 16 * np.arange(N_TIME // 16) + 8) * SAMPLE_DT   # block centres
            inside = np.abs(t_blk[:, None] - t_arr[None, :]) <= sky.width_s / 2    # [blk][q]
            if inside.any():
                amp = (rng.standard_normal(inside.shape) + 1j * rng.standard_normal(inside.shape))
                amp *= sky.pulse_amp / np.sqrt(2) * inside
                # time samples of each block: sum_q amp[b, q] e^{+2 pi i nu_q t}
                tt = (fr * N_TIME + np.arange(N_TIME)) * SAMPLE_DT
                ph = np.exp(2j * np.pi * np.outer(tt, nu))                           # [t][q]
                sig_t = (ph.reshape(N_TIME // 16, 16, 16) * amp[:, None, :]).sum(-1).reshape(-1)
                sig = np.outer(sig_t, spat)
                re += sig.real.astype(np.float32)
                im += sig.imag.astype(np.float32)
            for qq, a in tones:
                tt = (fr * N_TIME + np.arange(N_TIME)) * SAMPLE_DT
                s = a * np.exp(2j * np.pi * (qq - 8) * SUBCHAN_HZ * tt + 0.7j)
                re += s.real.astype(np.float32)[:, None]
                im += s.imag.astype(np.float32)[:, None]
            np.rint(re, out=re)
            np.rint(im, out=im)
            np.clip(re, -7, 7, out=re)
            np.clip(im, -7, 7, out=im)
            out[k, ci] = encode(re, im)
    _ = tau
    return out
