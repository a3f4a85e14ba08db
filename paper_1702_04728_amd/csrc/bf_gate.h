// Ingest gate of the serving loop's device-gated mode (beamform_stream with
// BF_STREAM_PACE_GATED): the host queues each launch ahead of its data, and a
// one-wave kernel in front of it holds the stream until the receiver has
// published that chunk's arrival.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bf {

// Words of the gate, in coherent pinned host memory written by the receiver:
//   gate[0]  chunks that have arrived (a count, modulo 2^32)
//   gate[1]  nonzero: every gate passes at once (set when the loop ends or
//            fails, so that nothing queued can wait on a receiver that stopped)
constexpr int kGateWords = 2;

// Enqueue on `stream` a wait until (int32_t)(gate[0] - target) >= 0 or
// gate[1] != 0.  The wait is bounded: after max_ticks of the device's
// constant-rate wall clock the kernel sets *timed_out = 1 and returns.
hipError_t launch_ingest_gate(const uint32_t* gate, uint32_t target, uint64_t max_ticks,
                              int32_t* timed_out, hipStream_t stream);

}  // namespace bf
