// Ingest gate of the serving loop's device-gated mode (beamform_stream with
// BF_STREAM_PACE_GATED): the host queues each launch ahead of its data, and a
// one-wave kernel in front of it holds the stream until that chunk's arrival
// time on the device's constant-rate wall clock (the emulated receiver writes
// into HBM at line rate, as a NIC would, whatever the host threads do).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bf {

// Launch state words one lane of the gate copies, at most (64 lanes cover a
// StreamState of BF_STREAM_MAX_SLOTS slots plus its header).
constexpr int kGateStateWordsPerLane = 17;

// Enqueue on `stream` a wait until the device wall clock (wall_clock64())
// reaches arrival_tick.  Before waiting, the kernel copies state_words 32-bit
// words of the launch's state from state_src (pinned host memory, read with
// system-scope loads) to state_dst (device memory, at most
// 64 x kGateStateWordsPerLane words), so that the launch needs no copy of its own.  The wait is bounded: after
// max_ticks the kernel sets *timed_out = 1 and returns.
hipError_t launch_ingest_gate(uint64_t arrival_tick, uint64_t max_ticks, int32_t* timed_out,
                              const uint32_t* state_src, uint32_t* state_dst, uint32_t state_words,
                              hipStream_t stream);

// Enqueue on `stream` one read of the device wall clock into *out (device or
// pinned host memory; a system-scope store, visible to the host once the
// kernel has completed).
hipError_t launch_wall_clock_probe(uint64_t* out, hipStream_t stream);

}  // namespace bf
