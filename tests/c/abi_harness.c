/*
 * Plain C caller of the library's host-only entry points (beamform.h): default
 * configuration, the Eq. (1) bin table (Sec. 3.1), status strings and the
 * serving loop's scheduler dry run.  No device call.  Built and run by
 * tests/test_c_abi_and_sanitizers.py, once against libbeamform.so and once
 * with the host code under AddressSanitizer and UndefinedBehaviorSanitizer.
 * Exit status 0 and a last line "abi harness ok" on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "beamform.h"

static int failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

/* Eq. (1) written out here: floor(N P f d sin(theta) / c + 1/2) mod N P. */
static int eq1(double f, double sin_theta)
{
    double t = 256.0 * 2.0 * f * (0.3048 / 299792458.0) * sin_theta + 0.5;
    long long k = (long long)floor(t) % 512;
    return (int)(k < 0 ? k + 512 : k);
}

int main(void)
{
    bf_config cfg;
    CHECK(beamform_default_config(NULL) == BF_E_INVAL);
    CHECK(beamform_default_config(&cfg) == BF_OK);
    CHECK(cfg.n_cyl == 4 && cfg.n_feed == 256 && cfg.n_pol == 2 && cfg.pad == 2);
    CHECK(cfg.n_beam_ns == 256 && cfg.n_beam_ew == 4 && cfg.n_upchan == 16 && cfg.n_time == 384);
    CHECK(cfg.feed_spacing_m == 0.3048 && cfg.c0 == 299792458.0 && cfg.precision == BF_FP32_FFT);
    CHECK(cfg.cyl_x_m == NULL && cfg.sin_theta_ns == NULL && cfg.lut_override == NULL);

    /* bin table of five channels across 400-800 MHz against Eq. (1) */
    double freqs[5] = {400e6, 491.796875e6, 600e6, 683.59375e6, 799.609375e6};
    int32_t *lut = (int32_t *)malloc(sizeof(int32_t) * 5 * 256);
    CHECK(lut != NULL);
    CHECK(beamform_compute_lut(&cfg, freqs, 5, lut) == BF_OK);
    for (int c = 0; c < 5; ++c)
        for (int m = 0; m < 256; ++m)
            CHECK(lut[c * 256 + m] == eq1(freqs[c], (m - 127.5) / 128.0));
    /* errors: bad arguments, a bad frequency, an argument beyond an exact floor */
    CHECK(beamform_compute_lut(NULL, freqs, 5, lut) == BF_E_INVAL);
    CHECK(beamform_compute_lut(&cfg, freqs, 0, lut) == BF_E_INVAL);
    double bad[1] = {-1.0};
    CHECK(beamform_compute_lut(&cfg, bad, 1, lut) == BF_E_INVAL);
    CHECK(strlen(beamform_last_error(NULL)) > 0);
    double huge[1] = {1e30};
    CHECK(beamform_compute_lut(&cfg, huge, 1, lut) == BF_E_INVAL);
    free(lut);

    CHECK(strcmp(beamform_strerror(BF_OK), "ok") == 0);
    const int codes[] = {BF_E_INVAL, BF_E_NOMEM, BF_E_DEVICE, BF_E_STATE, BF_E_UNSUPPORTED, -99};
    for (size_t i = 0; i < sizeof(codes) / sizeof(codes[0]); ++i)
        CHECK(beamform_strerror(codes[i]) != NULL && strlen(beamform_strerror(codes[i])) > 0);

    /* an unsupported geometry is refused before any device call */
    bf_config bad_cfg = cfg;
    bad_cfg.n_cyl = 3;
    bf_plan *plan = NULL;
    CHECK(beamform_init(&bad_cfg, freqs, 1, NULL, &plan) == BF_E_UNSUPPORTED && plan == NULL);
    CHECK(beamform_destroy(NULL) == BF_OK);

    /* scheduler dry run: 6 frames, 3 slots, room for 2 channels; a rejected join,
     * an ignored leave, an unformable frequency, and lost frames */
    bf_stream_event ev[] = {
        {0, BF_STREAM_JOIN, 10, 0, 450e6}, {0, BF_STREAM_JOIN, 11, 0, 460e6},
        {0, BF_STREAM_JOIN, 12, 0, 470e6}, {1, BF_STREAM_LEAVE, 99, 0, 0.0},
        {2, BF_STREAM_LEAVE, 10, 0, 0.0},  {2, BF_STREAM_JOIN, 13, 0, 1e30},
        {3, BF_STREAM_JOIN, 14, 0, 700e6}};
    int32_t slot_log[6 * 3];
    uint8_t ok[6 * 3];
    for (int i = 0; i < 18; ++i) ok[i] = (uint8_t)((i % 5) != 1);  /* 0 at 1, 6, 11, 16 */
    bf_stream_desc d;
    memset(&d, 0, sizeof(d));
    d.depth = 2;
    d.max_slots = 3;
    d.n_frames = 6;
    d.events = ev;
    d.n_events = (int32_t)(sizeof(ev) / sizeof(ev[0]));
    d.slot_log = slot_log;
    d.ingest_ok = ok;
    bf_stream_stats st;
    CHECK(beamform_stream_schedule(&d, 1000, 2999, &st) == BF_OK);
    CHECK(st.slot_capacity == 2);
    CHECK(st.joins == 3 && st.leaves == 1 && st.rejected_joins == 1 && st.ignored_events == 2);
    CHECK(slot_log[0] == 10 && slot_log[1] == 11 && slot_log[2] == -1);
    CHECK(slot_log[2 * 3 + 0] == -1 && slot_log[2 * 3 + 1] == 11);
    CHECK(slot_log[3 * 3 + 0] == 14 && slot_log[3 * 3 + 1] == 11);
    int64_t cf = 0, miss = 0;
    for (int i = 0; i < 6; ++i)
        for (int s = 0; s < 3; ++s)
            if (slot_log[i * 3 + s] >= 0) {
                ++cf;
                miss += ok[i * 3 + s] == 0;
            }
    CHECK(st.channel_frames == cf && st.missing_frames == miss && miss > 0);
    d.pacing = BF_STREAM_PACE_GATED;
    d.gate_timeout_ms = 5;
    CHECK(beamform_stream_schedule(&d, 1000, 2999, &st) == BF_OK);
    d.gate_timeout_ms = -1;
    CHECK(beamform_stream_schedule(&d, 1000, 2999, &st) == BF_E_INVAL);
    d.gate_timeout_ms = 0;
    d.pacing = 3;
    CHECK(beamform_stream_schedule(&d, 1000, 2999, &st) == BF_E_INVAL);
    d.pacing = BF_STREAM_PACE_HOST;
    d.depth = 0;
    CHECK(beamform_stream_schedule(&d, 1000, 2999, &st) == BF_E_INVAL);
    /* struct sizes, for the ctypes binding's mirror of these structs */
    printf("sizes config %zu stream_event %zu stream_desc %zu stream_stats %zu\n", sizeof(bf_config),
           sizeof(bf_stream_event), sizeof(bf_stream_desc), sizeof(bf_stream_stats));

    if (failures) {
        fprintf(stderr, "abi harness: %d failures\n", failures);
        return 1;
    }
    printf("abi harness ok\n");
    return 0;
}
