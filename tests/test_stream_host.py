"""Host logic of the serving loop, no GPU: the scheduler's slot assignment,
admission by memory, event handling and logs (through the library's own
dry-run entry point), and the seeded churn generator."""
import numpy as np
import pytest

import paper_1702_04728_amd as bf
import synth

J, L = bf.STREAM_JOIN, bf.STREAM_LEAVE
PSB = 1000  # per-slot bytes used in these dry runs


def _model(events, n_frames, max_slots, capacity):
    """Independent replay: lowest free slot on join, admission by capacity."""
    slots = [-1] * max_slots
    log = np.full((n_frames, max_slots), -1, np.int32)
    rej = ign = 0
    ev = sorted(events, key=lambda e: e[0])
    k = 0
    for f in range(n_frames):
        while k < len(ev) and ev[k][0] <= f:
            _, op, cid, freq = ev[k]
            k += 1
            if op == J:
                if cid in slots or freq <= 0:
                    ign += 1
                elif sum(s >= 0 for s in slots) >= capacity:
                    rej += 1
                else:
                    slots[slots.index(-1)] = cid
            elif op == L:
                if cid in slots:
                    slots[slots.index(cid)] = -1
                else:
                    ign += 1
            else:
                ign += 1
        log[f] = slots
    return log, rej, ign + (len(ev) - k)


def test_slots_lowest_free_and_reuse():
    ev = [(0, J, 10, 450e6), (0, J, 11, 460e6), (0, J, 12, 470e6),
          (2, L, 11, 0.0), (3, J, 13, 480e6), (5, L, 10, 0.0), (5, J, 14, 490e6)]
    st, log = bf.stream_schedule(ev, 7, 4, PSB, 4 * PSB)
    assert log[0].tolist() == [10, 11, 12, -1]
    assert log[2].tolist() == [10, -1, 12, -1]
    assert log[3].tolist() == [10, 13, 12, -1]
    assert log[5].tolist() == [14, 13, 12, -1]   # leave then join in one frame reuses slot 0
    assert (st["joins"], st["leaves"], st["rejected_joins"], st["ignored_events"]) == (5, 2, 0, 0)
    assert st["channel_frames"] == int((log >= 0).sum())
    assert (st["max_active"], st["min_active"]) == (3, 2)


def test_admission_by_memory_cap():
    ev = [(0, J, c, 400e6 + c * 390625.0) for c in range(6)] + [(1, L, 2, 0.0), (1, J, 9, 500e6)]
    # room for exactly 4 channels
    st, log = bf.stream_schedule(ev, 3, 8, PSB, 4 * PSB + PSB - 1)
    assert st["slot_capacity"] == 4
    assert st["rejected_joins"] == 2
    assert log[0].tolist() == [0, 1, 2, 3, -1, -1, -1, -1]
    assert log[1].tolist() == [0, 1, 9, 3, -1, -1, -1, -1]
    assert st["per_slot_bytes"] == PSB
    # cap below one slot: every join rejected
    st, log = bf.stream_schedule(ev, 3, 8, PSB, PSB - 1)
    assert st["rejected_joins"] == 7 and (log < 0).all()


def test_ignored_events():
    ev = [(0, J, 1, 450e6), (0, J, 1, 450e6), (1, L, 7, 0.0), (1, 3, 2, 450e6),
          (2, J, 5, -1.0), (9, J, 6, 500e6)]
    st, log = bf.stream_schedule(ev, 4, 2, PSB, 10 * PSB)
    assert st["joins"] == 1
    assert st["ignored_events"] == 5   # duplicate, unknown leave, bad op, bad freq, after end


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_churn_schedule_matches_model(seed):
    ev, clamped = synth.churn_events(seed, 600, rate_join=0.3, rate_leave=0.3, initial=20,
                                     lo=16, hi=32)
    for cap_slots in (40, 25):
        st, log = bf.stream_schedule(ev, 600, 40, PSB, cap_slots * PSB)
        ref_log, rej, ign = _model(ev, 600, 40, cap_slots)
        np.testing.assert_array_equal(log, ref_log)
        assert st["rejected_joins"] == rej and st["ignored_events"] == ign


def test_churn_generator_properties():
    ev, clamped = synth.churn_events(1003, 10000)
    ev2, clamped2 = synth.churn_events(1003, 10000)
    assert ev == ev2 and clamped == clamped2          # seeded
    assert sum(1 for e in ev if e[0] == 0) == 64       # initial joins
    active, lo, hi = set(), 10 ** 9, 0
    frames = [e[0] for e in ev]
    assert frames == sorted(frames)
    k = 0
    for f in range(10000):
        while k < len(ev) and ev[k][0] == f:
            _, op, cid, freq = ev[k]
            if op == J:
                assert cid not in active and freq == synth.chan_freq_hz(cid)
                active.add(cid)
            else:
                assert cid in active
                active.remove(cid)
            k += 1
        lo, hi = min(lo, len(active)), max(hi, len(active))
    assert 16 <= lo and hi <= 128
    # about 0.02 joins and leaves per frame
    n_join = sum(1 for e in ev if e[1] == J) - 64
    assert 120 < n_join < 300


def test_schedule_rejects_bad_descriptors():
    with pytest.raises(bf.BeamformError):
        bf.stream_schedule([(3, J, 1, 450e6), (1, J, 2, 450e6)], 5, 4, PSB, 4 * PSB)
    with pytest.raises(bf.BeamformError):
        bf.stream_schedule([], 5, bf.STREAM_MAX_SLOTS + 1, PSB, PSB)
    with pytest.raises(bf.BeamformError):
        bf.stream_schedule([], 5, 4, PSB, 4 * PSB, depth=0)
    # warm-up frames left out of the statistics: 0 .. n_frames
    for bad in (-1, 6):
        with pytest.raises(bf.BeamformError):
            bf.stream_schedule([], 5, 4, PSB, 4 * PSB, warmup_frames=bad)
    for ok in (0, 5):
        bf.stream_schedule([], 5, 4, PSB, 4 * PSB, warmup_frames=ok)
    # pacing: none, host-paced, device-gated; a gated wait's bound is >= 0 (0: default)
    for ok in ("none", "host", "gated", 0, 1, 2):
        bf.stream_schedule([], 5, 4, PSB, 4 * PSB, pacing=ok)
    for bad in (3, -1):
        with pytest.raises(bf.BeamformError):
            bf.stream_schedule([], 5, 4, PSB, 4 * PSB, pacing=bad)
    with pytest.raises(ValueError):
        bf.stream_schedule([], 5, 4, PSB, 4 * PSB, pacing="fast")
    with pytest.raises(bf.BeamformError):
        bf.stream_schedule([], 5, 4, PSB, 4 * PSB, pacing="gated", gate_timeout_ms=-1)


def test_join_with_unformable_bin_table_is_ignored():
    """A JOIN whose Eq. (1) bins cannot be formed (frequency so large that the
    argument leaves the exact integer floor, or not finite) is ignored, as a bad
    frequency is, instead of admitting a slot with a stale bin table."""
    ev = [(0, J, 1, 600e6), (0, J, 2, 1e30), (0, J, 3, float("inf")), (0, J, 4, float("nan")),
          (1, J, 5, 700e6)]
    st, log = bf.stream_schedule(ev, 3, 8, PSB, 8 * PSB)
    assert log[0].tolist()[:2] == [1, -1]
    assert log[2].tolist()[:3] == [1, 5, -1]
    assert (st["joins"], st["ignored_events"]) == (2, 3)


def test_missing_frames_counted_for_active_slots_only():
    """Lossy ingest: a zero in ingest_ok marks a channel-frame that did not arrive.
    The dry run counts exactly the zeros that fall on active slots (an empty slot
    has no frame to lose), every frame and warm-up included."""
    rng = np.random.default_rng(5)
    ev, _ = synth.churn_events(9, 40, n_ids=64, initial=5, rate_join=0.3, rate_leave=0.3,
                               lo=2, hi=7)
    ok = (rng.random((40, 8)) > 0.25).astype(np.uint8)
    st, log = bf.stream_schedule(ev, 40, 8, PSB, 8 * PSB, warmup_frames=5, ingest_ok=ok)
    expect = int(((log >= 0) & (ok == 0)).sum())
    assert expect > 10
    assert st["missing_frames"] == expect
    st0, log0 = bf.stream_schedule(ev, 40, 8, PSB, 8 * PSB)
    assert st0["missing_frames"] == 0
    np.testing.assert_array_equal(log, log0)   # losses never change the schedule
    with pytest.raises(ValueError):
        bf.stream_schedule(ev, 40, 8, PSB, 8 * PSB, ingest_ok=ok[:, :4])
