// The plan behind the opaque bf_plan handle (host code only).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "bf_internal.h"

struct bf_plan {
    bf_config cfg{};                 // host-array pointers cleared; copies below
    std::vector<double> cyl_x, sin_theta, sin_phi, freqs;
    std::vector<int32_t> lut;        // [n_chan][256]
    int32_t n_chan = 0;
    int device = 0;
    int32_t* d_lut = nullptr;
    float2* d_ew = nullptr;
    float2* d_tw = nullptr;
    void* d_mf = nullptr;
    int32_t sym_ew = 0;              // geometry symmetric about the array centre
    int32_t cyl_sym = 0;             // cylinder positions symmetric about the centre
    // Tracking E-W weights, double-buffered so that the host fills one table
    // while the previous call's kernel reads the other: device [cap][4][4],
    // pinned host staging of the same size, and the event recorded after the
    // kernel that last read it.
    struct EwTrack {
        float2* d = nullptr;
        float2* h = nullptr;
        size_t cap = 0;              // rows (channel-frames)
        hipEvent_t done = nullptr;
    } ew_track[2];
    int ew_track_next = 0;
    // 128-point up-channelisation: the w128^(k m) table
    float2* d_tw128 = nullptr;
    // Allocation-free tracking: this device's fixed weight table (library-wide,
    // not owned by the plan) and the event that tells when its upload has read
    // the host staging table.
    float2* d_scratch = nullptr;
    hipEvent_t noalloc_upload = nullptr;
    std::string err;
};
