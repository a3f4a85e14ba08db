"""GPU tests of the serving loop (beamform_stream): per-frame outputs equal the
batch path bitwise and the oracle within tolerance, across channel churn;
chunked ingest (partial integrations kept in HBM) equals whole-frame ingest
bitwise; hipGraph replay equals plain launches bitwise; host-paced and device-gated
real time (the gate holds every queued launch until its chunk's arrival) and
admission."""
import numpy as np
import pytest

import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = {"fp32": 1e-5, "fp16": 2e-3, "fp32_mfma": 1e-5}
J, L = 1, 2


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
def pool():
    return synth.frame_pool(77, 7)


def _ring(torch_mod, pool, depth, slots):
    idx = np.array([(3 * k + s) % len(pool) for k in range(depth) for s in range(slots)])
    dev = torch_mod.from_numpy(pool).cuda()
    return dev[torch_mod.from_numpy(idx).cuda()].reshape(depth, slots, 384, 2048).contiguous()


def _f(c):
    return float(synth.chan_freq_hz(c))


EVENTS = [(0, J, 100, _f(100)), (0, J, 700, _f(700)), (0, J, 300, _f(300)), (0, J, 901, _f(901)),
          (3, L, 700, 0.0), (3, J, 512, _f(512)), (3, J, 44, _f(44)),
          (6, L, 100, 0.0), (6, L, 901, 0.0), (6, J, 1000, _f(1000)),
          (8, L, 44, 0.0), (8, J, 45, _f(45))]


def _stream(torch_mod, bfm, ring, precision, n_frames=10, events=EVENTS, **kw):
    depth, slots = ring.shape[0], ring.shape[1]
    out = torch_mod.full((depth, slots, 1024, 16), -1.0, dtype=torch_mod.float32, device="cuda")
    print("stream: precision %s ring %s frames %d %s" % (precision, tuple(ring.shape), n_frames, kw),
          flush=True)
    with bfm.Beamformer([600e6], precision=precision) as b:
        st, log = b.stream(ring, out, events, n_frames, **kw)
    torch_mod.cuda.synchronize()
    return st, log, out.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
def test_stream_outputs_match_batch_and_oracle(torch_mod, bfm, oracle_mod, pool, precision):
    ring = _ring(torch_mod, pool, 4, 6)
    st, log, out = _stream(torch_mod, bfm, ring, precision, use_graph=True)
    assert st["frames"] == 10 and st["joins"] == 8 and st["leaves"] == 4
    assert st["channel_frames"] == int((log >= 0).sum())
    ring_np = ring.cpu().numpy()
    checked = 0
    for i in range(6, 10):                       # the ring keeps the last 4 frames
        for s in np.nonzero(log[i] >= 0)[0]:
            cid = int(log[i][s])
            raw = ring_np[i % 4, s][None, None]
            with bfm.Beamformer([_f(cid)], precision=precision) as b:
                ref = b.frame(torch_mod.from_numpy(raw).cuda()).cpu().numpy()[0, 0]
            np.testing.assert_array_equal(out[i % 4, s], ref)
            checked += 1
            if checked <= 3:
                o = oracle_mod.beamform(oracle_mod.Geometry(), [_f(cid)], raw)[0, 0]
                assert np.max(np.abs(out[i % 4, s] - o) / o) <= TOL[precision]
    assert checked >= 10


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
def test_stream_full_size_512_channels(torch_mod, bfm, oracle_mod, precision):
    """The max-load sweep's launch configuration at full size: 512 channels over
    400-800 MHz, all joined at frame 0, hipGraph replay, whole frames, config-4 frames
    tiled over a 2-deep ring.  Every output of the last two frames equals the batch
    path on the same bytes (bit for bit), and sampled channel-frames match the oracle."""
    n = 512
    c_idx = synth.sweep_c_idx(n)
    freqs = synth.chan_freq_hz(c_idx)
    pool16 = torch_mod.from_numpy(
        synth.config4_frames(1004, synth.sweep_c_idx(16), [0]).reshape(16, 384, 2048)).cuda()
    depth = 2
    idx = torch_mod.tensor([(7 * k + s) % 16 for k in range(depth) for s in range(n)], device="cuda")
    ring = pool16[idx].reshape(depth, n, 384, 2048).contiguous()
    events = [(0, J, int(c), float(f)) for c, f in zip(c_idx, freqs)]
    st, log, out = _stream(torch_mod, bfm, ring, precision, n_frames=4, events=events,
                           use_graph=True)
    assert st["frames"] == 4 and st["channel_frames"] == 4 * n
    assert (log[-1] == c_idx).all()
    with bfm.Beamformer(freqs, precision=precision) as b:
        for i in (2, 3):
            ref = b.frame(ring[i % depth][None]).cpu().numpy()[0]
            np.testing.assert_array_equal(out[i % depth], ref)
    for s_ in (0, 170, 341, 511):
        raw = ring[3 % depth, s_].cpu().numpy()[None, None]
        o = oracle_mod.beamform(oracle_mod.Geometry(), [freqs[s_]], raw)[0, 0]
        assert np.max(np.abs(out[3 % depth, s_] - o) / o) <= TOL[precision], s_
    del ring, pool16


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
@pytest.mark.parametrize("chunk", [128, 16])
def test_chunked_partial_sums_equal_whole_frames(torch_mod, bfm, pool, precision, chunk):
    ring = _ring(torch_mod, pool, 3, 5)
    _, log_a, a = _stream(torch_mod, bfm, ring, precision, n_frames=7, chunk=0)
    st, log_b, b = _stream(torch_mod, bfm, ring, precision, n_frames=7, chunk=chunk)
    np.testing.assert_array_equal(log_a, log_b)
    assert st["launches"] == 7 * (384 // chunk)
    live = log_a[-1] >= 0
    np.testing.assert_array_equal(a[:, live], b[:, live])


def test_graph_replay_equals_plain_launches(torch_mod, bfm, pool):
    ring = _ring(torch_mod, pool, 4, 6)
    _, _, a = _stream(torch_mod, bfm, ring, "fp32", use_graph=True)
    _, _, b = _stream(torch_mod, bfm, ring, "fp32", use_graph=False)
    np.testing.assert_array_equal(a, b)


def test_paced_latency(torch_mod, bfm, pool):
    ring = _ring(torch_mod, pool, 4, 8)
    ev = [(0, J, c, _f(c)) for c in (10, 200, 400, 600, 800, 1000)]
    st, _, _ = _stream(torch_mod, bfm, ring, "fp32", n_frames=300, events=ev, pacing=True)
    print(st)
    budget = 384 * 2.56e-3
    assert st["frames"] == 300 and st["channel_frames"] == 1800
    assert 0 < st["latency_p50_ms"] < budget
    assert st["late_frames"] <= 30
    # paced: wall time is at least the stream's own duration
    assert st["wall_s"] >= 300 * budget * 1e-3
    assert st["service_mean_ms"] > 0


@pytest.mark.parametrize("chunk,use_graph", [(0, True), (128, True), (0, False)])
def test_gated_pacing_equals_unpaced(torch_mod, bfm, pool, chunk, use_graph):
    ring = _ring(torch_mod, pool, 4, 6)
    _, log_a, a = _stream(torch_mod, bfm, ring, "fp16", chunk=chunk)
    st, log_b, b = _stream(torch_mod, bfm, ring, "fp16", chunk=chunk, pacing="gated",
                           use_graph=use_graph)
    np.testing.assert_array_equal(log_a, log_b)
    np.testing.assert_array_equal(a, b)
    assert st["launches"] == 10 * (384 // (chunk or 384))
    # held to the arrival clock: the run lasts at least the stream's own duration
    assert st["wall_s"] >= 10 * 384 * 2.56e-6


@pytest.mark.parametrize("chunk", [0, 128])
def test_gated_launches_queue_ahead_and_wait_for_data(torch_mod, bfm, pool, chunk):
    """Device-gated pacing: the host queues launches ahead of their data (issue log
    negative), yet no frame completes before its last chunk has arrived (latency
    > 0 for every frame: the gate holds each launch until its arrival time on the
    device clock), a gate opens close to that time (median latency within 0.15 ms
    of the device time), and the frames keep up."""
    ring = _ring(torch_mod, pool, 4, 8)
    ev = [(0, J, c, _f(c)) for c in (10, 200, 400, 600, 800, 1000)]
    n, warm = 300, 20
    lat, svc, iss = np.zeros(n), np.zeros(n), np.zeros(n)
    st, _, _ = _stream(torch_mod, bfm, ring, "fp32", n_frames=n, events=ev, chunk=chunk,
                       pacing="gated", warmup_frames=warm, latency_log=lat, service_log=svc,
                       issue_log=iss)
    print(st)
    budget = 384 * 2.56e-3
    assert st["frames"] == n and st["channel_frames"] == 6 * n
    assert lat.min() > 0.0
    assert np.median(iss[warm:]) < -budget
    assert 0 < st["latency_p50_ms"] < st["service_mean_ms"] + 0.15
    assert st["late_frames"] <= 3
    assert np.all(svc[warm:] > 0)
    assert st["wall_s"] >= n * budget * 1e-3


def test_gated_wait_timeout_is_an_error(torch_mod, bfm):
    """A gate that would wait longer than its bound (9.8 ms frames queued ahead of
    their data, 1 ms bound) fails the loop with BF_E_DEVICE; every gate still
    returns (bounded wait), and the plan serves again afterwards."""
    ring = torch_mod.zeros((2, 1, 3840, 2048), dtype=torch_mod.uint8, device="cuda")
    out = torch_mod.zeros((2, 1, 1024, 16), dtype=torch_mod.float32, device="cuda")
    with bfm.Beamformer([600e6], n_time=3840) as b:
        with pytest.raises(bfm.BeamformError, match="gate"):
            b.stream(ring, out, [(0, J, 5, _f(5))], 3, pacing="gated", gate_timeout_ms=1)
        st, _ = b.stream(ring, out, [(0, J, 5, _f(5))], 2, pacing="gated")
    torch_mod.cuda.synchronize()
    assert st["frames"] == 2 and st["channel_frames"] == 2


def test_admission_under_memory_cap(torch_mod, bfm, pool):
    ring = _ring(torch_mod, pool, 2, 6)
    ev = [(0, J, c, _f(c)) for c in (1, 2, 3, 4, 5)] + [(2, L, 2, 0.0), (2, J, 6, _f(6))]
    with bfm.Beamformer([600e6]) as b:
        out = torch_mod.zeros((2, 6, 1024, 16), dtype=torch_mod.float32, device="cuda")
        st0, _ = b.stream(ring, out, [], 0)
        psb = st0["per_slot_bytes"]
        st, log = b.stream(ring, out, ev, 4, mem_cap_bytes=3 * psb)
    dry, dry_log = bfm.stream_schedule(ev, 4, 6, psb, 3 * psb)
    assert st["slot_capacity"] == 3 and st["rejected_joins"] == 2
    np.testing.assert_array_equal(log, dry_log)
    assert dry["rejected_joins"] == st["rejected_joins"]


def test_stream_argument_errors(torch_mod, bfm, pool):
    ring = _ring(torch_mod, pool, 2, 2)
    out = torch_mod.zeros((2, 2, 1024, 16), dtype=torch_mod.float32, device="cuda")
    with bfm.Beamformer([600e6]) as b:
        with pytest.raises(bfm.BeamformError):
            b.stream(ring, out, [], 3, chunk=100)
        with pytest.raises(bfm.BeamformError):
            b.stream(ring, out, [(2, J, 1, 5e8), (1, J, 2, 5e8)], 3)
        with pytest.raises(ValueError):
            b.stream(ring, out[:1], [], 3)
        with pytest.raises(bfm.BeamformError):
            b.stream(ring, out, [], 3, warmup_frames=4)
        with pytest.raises(bfm.BeamformError):
            b.stream(ring, out, [], 3, warmup_frames=-1)
        st, _ = b.stream(ring, out, [], 0)
        assert st["frames"] == 0
        # statistics after a warm-up: every frame still runs, the figures cover the rest
        st, _ = b.stream(ring, out, [(0, J, 1, 5e8)], 5, warmup_frames=5)
        assert st["frames"] == 5 and st["channel_frames"] == 5 and st["late_frames"] == 0
        assert st["latency_p99_ms"] == 0.0


@pytest.mark.parametrize("precision", ["fp32", "fp16", "fp32_mfma"])
@pytest.mark.parametrize("chunk", [0, 128])
@pytest.mark.parametrize("pacing", ["none", "gated"])
def test_lossy_ingest_zeroes_and_flags_missing_frames(torch_mod, bfm, pool, precision, chunk, pacing):
    """Channel-frames the ingest did not deliver (ingest_ok = 0: an empty or late
    ring entry) are skipped: their output entry is exactly zero and flagged 0 in
    out_valid, and they are counted; every delivered one is flagged 1 and equals
    the batch path bit for bit, also right after a loss with chunked ingest (the
    partial sums restart at each frame's first chunk)."""
    ring = _ring(torch_mod, pool, 4, 6)
    rng = np.random.default_rng(11)
    ok = (rng.random((10, 6)) > 0.3).astype(np.uint8)
    depth, slots = 4, 6
    valid = torch_mod.full((depth, slots), 255, dtype=torch_mod.uint8, device="cuda")
    st, log, out = _stream(torch_mod, bfm, ring, precision, chunk=chunk, ingest_ok=ok,
                           out_valid=valid, pacing=pacing)
    valid = valid.cpu().numpy()
    assert st["missing_frames"] == int(((log >= 0) & (ok == 0)).sum()) > 0
    ring_np = ring.cpu().numpy()
    n_missing = n_ok = 0
    for i in range(6, 10):                       # the ring keeps the last 4 frames
        for s in range(slots):
            if log[i][s] < 0:
                continue
            if not ok[i][s]:
                assert valid[i % 4, s] == 0
                assert not out[i % 4, s].any()
                n_missing += 1
                continue
            assert valid[i % 4, s] == 1
            with bfm.Beamformer([_f(int(log[i][s]))], precision=precision) as b:
                ref = b.frame(torch_mod.from_numpy(ring_np[i % 4, s][None, None]).cuda())
            np.testing.assert_array_equal(out[i % 4, s], ref.cpu().numpy()[0, 0])
            n_ok += 1
    assert n_missing >= 2 and n_ok >= 6
