/*
 * FP64 reference oracle for the CHIME/FRB hybrid FFT beamformer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU definition that the GPU library is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the product path never calls it.  It shares no code, header, table or
 * constant with the HIP library.
 *
 * Paper: Ng et al., "CHIME FRB: An application of FFT beamforming for a radio
 * telescope" (arXiv:1702.04728).  What is computed, per frequency channel and
 * per 0.983 ms frame:
 *
 *   decode   Sec. 2 and Table 1: 2048 inputs (4 cylinders x 256 N-S feeds x 2
 *            polarisations), each sample a 4-bit real + 4-bit imaginary pair
 *            at a 2.56 us cadence.
 *   N-S      Sec. 3.1: a zero-padded spatial FFT (N = 256 feeds, padding P = 2,
 *            so N*P = 512 bins), subsampled to the bin nearest each of 256
 *            desired pointings.  Eq. (1) gives that bin; Eq. (2) is the same
 *            formula moved to another frequency, so it is evaluated per
 *            channel directly.  Bin k of a zero-padded FFT is, by definition,
 *            sum_n x_n exp(-2 pi i n k / (N P)); the oracle evaluates each kept
 *            beam as exactly that direct O(N^2) sum.
 *   E-W      Sec. 3 (first kernel) and Sec. 3.1 (static E-W beams): four beams
 *            by exact phasing across the four cylinders.
 *   upchan   Sec. 3 (third kernel) and Sec. 3.2: a DFT along time of each
 *            beam; here a naive L-point DFT over consecutive, non-overlapping
 *            blocks of L samples (L = 16 gives 390.625 kHz / 16 = 24.4 kHz).
 *   detect   Sec. 3: Stokes I, i.e. |X|^2 + |Y|^2 (square the real and
 *            imaginary parts and sum the two polarisations), integrated over
 *            all blocks of the frame (24 blocks of 16 = 384 samples = 0.983 ms,
 *            Table 1).
 *   8-bit    Sec. 3 and Table 1: the integrated beams are rescaled to 8-bit
 *            integers (rule not given: an affine rescale per output, decided
 *            in FP32 like the library, since floating point decides an
 *            integer there).
 *
 * Conventions the paper leaves open (nibble order, input order, signs,
 * rounding of Eq. (1), sub-channel order) are fixed by the library's
 * documented readings and are restated where they are used below:
 *   - byte = ((re + 8) << 4) | (im + 8): high nibble real, offset 8;
 *   - input index i = (cyl * n_feed + feed) * n_pol + pol;
 *   - forward transforms use exp(-2 pi i ...);
 *   - Eq. (1) index rounded as floor(x + 0.5), then reduced mod N*P;
 *   - E-W weight W[j][c] = exp(-2 pi i f x_c sin(phi_j) / c0);
 *   - output sub-channel q holds DFT bin s = (q + L/2) mod L (centre-shifted),
 *     beam index = j * n_beam_ns + m.
 * All arithmetic is FP64 except the 8-bit code decision.  Sizes are
 * parameters so that tiny cases can be brute-forced in tests.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n_feed;     /* N, feeds per cylinder line (256) */
    int32_t pad;        /* P, zero-padding factor (2) */
    int32_t n_cyl;      /* cylinders (4) */
    int32_t n_pol;      /* polarisations (2) */
    int32_t n_beam_ns;  /* kept N-S beams (256) */
    int32_t n_beam_ew;  /* E-W beams (4) */
    int32_t n_dft;      /* L, up-channelisation length (16) */
    int32_t n_time;     /* samples per frame (384) */
    double feed_spacing_m; /* d (0.3048 m) */
    double c0;             /* speed of light (m/s) */
    const double *cyl_x_m;      /* [n_cyl] cylinder E-W positions */
    const double *sin_theta_ns; /* [n_beam_ns] desired N-S pointings */
    const double *sin_phi_ew;   /* [n_beam_ew] E-W beam directions */
} orc_geom;

static const double ORC_TWO_PI = 6.283185307179586476925286766559;

/* exp(-2 pi i r / n) for r = 0..n-1, from cos/sin of the reduced angle. */
static void orc_roots(int32_t n, double *tab)
{
    for (int32_t r = 0; r < n; ++r) {
        double a = ORC_TWO_PI * (double)r / (double)n;
        tab[2 * r] = cos(a);
        tab[2 * r + 1] = -sin(a);
    }
}

/* Decode 4+4-bit samples (Sec. 2, Table 1): out[2i] = re, out[2i+1] = im. */
void orc_decode(const uint8_t *in, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        out[2 * i] = (double)((int)(in[i] >> 4) - 8);
        out[2 * i + 1] = (double)((int)(in[i] & 15) - 8);
    }
}

/*
 * Eq. (1): reference beam index t_m = N P f d sin(theta_m) / c + 0.5, taken
 * as floor() and reduced mod N*P so that southern (negative) pointings and
 * aliased ones land on the FFT bin that holds them.
 */
void orc_lut(const orc_geom *g, double f_hz, int32_t *k_out)
{
    const int32_t nb = g->n_feed * g->pad;
    for (int32_t m = 0; m < g->n_beam_ns; ++m) {
        double t = (double)g->n_feed * (double)g->pad * f_hz
                   * (g->feed_spacing_m / g->c0) * g->sin_theta_ns[m] + 0.5;
        int64_t k = (int64_t)floor(t);
        int64_t r = k % nb;
        if (r < 0) r += nb;
        k_out[m] = (int32_t)r;
    }
}

/*
 * N-S beams of one line (Sec. 3.1): y_m = sum_{n < n_feed} x_n w^(n k_m),
 * w = exp(-2 pi i / n_bins), i.e. bin k_m of the n_bins-point DFT of the line
 * zero-padded from n_feed to n_bins samples.  `roots` holds w^r.
 */
static void orc_ns_beams_tab(int32_t n_feed, int32_t n_bins, const double *roots,
                             const double *x, int32_t n_k, const int32_t *k,
                             double *y)
{
    for (int32_t m = 0; m < n_k; ++m) {
        /* r = (n * k_m) mod n_bins, stepped by k_m (0 <= k_m < n_bins) */
        const int32_t km = k[m];
        int32_t r = 0;
        double re = 0.0, im = 0.0;
        for (int32_t n = 0; n < n_feed; ++n) {
            double wr = roots[2 * r], wi = roots[2 * r + 1];
            double xr = x[2 * n], xi = x[2 * n + 1];
            re += xr * wr - xi * wi;
            im += xr * wi + xi * wr;
            r += km;
            if (r >= n_bins) r -= n_bins;
        }
        y[2 * m] = re;
        y[2 * m + 1] = im;
    }
}

void orc_ns_beams(int32_t n_feed, int32_t n_bins, const double *x, int32_t n_k,
                  const int32_t *k, double *y)
{
    for (int32_t m = 0; m < n_k; ++m)
        if (k[m] < 0 || k[m] >= n_bins) return;
    double *roots = (double *)malloc(sizeof(double) * 2 * (size_t)n_bins);
    orc_roots(n_bins, roots);
    orc_ns_beams_tab(n_feed, n_bins, roots, x, n_k, k, y);
    free(roots);
}

/* E-W exact-phasing weights (Sec. 3.1): W[j][c] = exp(-2 pi i f x_c sin(phi_j) / c0). */
void orc_ew_weights(const orc_geom *g, double f_hz, double *w)
{
    for (int32_t j = 0; j < g->n_beam_ew; ++j)
        for (int32_t c = 0; c < g->n_cyl; ++c) {
            double a = ORC_TWO_PI * f_hz * g->cyl_x_m[c] * g->sin_phi_ew[j] / g->c0;
            w[2 * (j * g->n_cyl + c)] = cos(a);
            w[2 * (j * g->n_cyl + c) + 1] = -sin(a);
        }
}

/* E-W beams for one (sample, pol, N-S beam): b_j = sum_c W[j][c] y_c. */
void orc_ew_beams(int32_t n_cyl, int32_t n_ew, const double *w, const double *y,
                  double *b)
{
    for (int32_t j = 0; j < n_ew; ++j) {
        double re = 0.0, im = 0.0;
        for (int32_t c = 0; c < n_cyl; ++c) {
            double wr = w[2 * (j * n_cyl + c)], wi = w[2 * (j * n_cyl + c) + 1];
            re += wr * y[2 * c] - wi * y[2 * c + 1];
            im += wr * y[2 * c + 1] + wi * y[2 * c];
        }
        b[2 * j] = re;
        b[2 * j + 1] = im;
    }
}

/* Naive L-point DFT along time (Sec. 3.2): u_s = sum_tau b_tau exp(-2 pi i s tau / L). */
static void orc_upchan_tab(int32_t L, const double *roots, const double *b, double *u)
{
    for (int32_t s = 0; s < L; ++s) {
        double re = 0.0, im = 0.0;
        for (int32_t t = 0; t < L; ++t) {
            int64_t r = ((int64_t)s * t) % L;
            double wr = roots[2 * r], wi = roots[2 * r + 1];
            re += b[2 * t] * wr - b[2 * t + 1] * wi;
            im += b[2 * t] * wi + b[2 * t + 1] * wr;
        }
        u[2 * s] = re;
        u[2 * s + 1] = im;
    }
}

void orc_upchan(int32_t L, const double *b, double *u)
{
    double *roots = (double *)malloc(sizeof(double) * 2 * (size_t)L);
    orc_roots(L, roots);
    orc_upchan_tab(L, roots, b, u);
    free(roots);
}

static int orc_check(const orc_geom *g)
{
    if (!g || g->n_feed <= 0 || g->pad <= 0 || g->n_cyl <= 0 || g->n_pol <= 0 ||
        g->n_beam_ns <= 0 || g->n_beam_ew <= 0 || g->n_dft <= 0 || g->n_time <= 0)
        return -1;
    if (g->n_time % g->n_dft != 0) return -1;
    if (!g->cyl_x_m || !g->sin_theta_ns || !g->sin_phi_ew) return -1;
    return 0;
}

/*
 * Steps 1-3 for one channel-frame: decode, N-S zero-padded beams at the kept
 * bins, E-W exact phasing.  Returns B[p][j][m][t] (complex, time innermost: the
 * paper's transposed order), allocated here and freed by the caller, or NULL
 * on bad arguments or allocation failure.  `lut` gives the kept bin per N-S
 * beam; NULL means Eq. (1) at f_hz.
 */
static double *orc_beams_time(const orc_geom *g, double f_hz, const int32_t *lut,
                              const uint8_t *in)
{
    if (orc_check(g)) return NULL;
    const int32_t NF = g->n_feed, NB = g->n_feed * g->pad, NC = g->n_cyl,
                  NP = g->n_pol, NM = g->n_beam_ns, NJ = g->n_beam_ew, T = g->n_time;
    const int64_t n_in = (int64_t)NC * NF * NP;

    int32_t *k = (int32_t *)malloc(sizeof(int32_t) * NM);
    double *roots = (double *)malloc(sizeof(double) * 2 * NB);
    double *w = (double *)malloc(sizeof(double) * 2 * NJ * NC);
    double *x = (double *)malloc(sizeof(double) * 2 * (size_t)T * n_in);        /* [t][i] */
    double *line = (double *)malloc(sizeof(double) * 2 * NF);
    double *yb = (double *)malloc(sizeof(double) * 2 * NM);
    /* Y[t][p][m][c]: N-S beams, cylinders innermost for the E-W sum */
    double *Y = (double *)malloc(sizeof(double) * 2 * (size_t)T * NP * NM * NC);
    /* B[p][j][m][t]: after E-W phasing, time innermost (the paper's transpose) */
    double *B = (double *)malloc(sizeof(double) * 2 * (size_t)NP * NJ * NM * T);
    double *bj = (double *)malloc(sizeof(double) * 2 * NJ);
    int ok = k && roots && w && x && line && yb && Y && B && bj;
    if (ok) {
        if (lut) memcpy(k, lut, sizeof(int32_t) * NM);
        else orc_lut(g, f_hz, k);
        for (int32_t m = 0; m < NM; ++m)
            if (k[m] < 0 || k[m] >= NB) ok = 0;
    }
    if (!ok) {
        free(k); free(roots); free(w); free(x); free(line); free(yb); free(Y); free(B); free(bj);
        return NULL;
    }
    orc_roots(NB, roots);
    orc_ew_weights(g, f_hz, w);

    /* 1. decode */
    orc_decode(in, (int64_t)T * n_in, x);

    /* 2. N-S zero-padded beams, one line per (sample, cylinder, pol) */
    for (int32_t t = 0; t < T; ++t)
        for (int32_t c = 0; c < NC; ++c)
            for (int32_t p = 0; p < NP; ++p) {
                for (int32_t n = 0; n < NF; ++n) {
                    int64_t i = ((int64_t)c * NF + n) * NP + p;
                    line[2 * n] = x[2 * ((int64_t)t * n_in + i)];
                    line[2 * n + 1] = x[2 * ((int64_t)t * n_in + i) + 1];
                }
                orc_ns_beams_tab(NF, NB, roots, line, NM, k, yb);
                for (int32_t m = 0; m < NM; ++m) {
                    size_t o = (((size_t)t * NP + p) * NM + m) * NC + c;
                    Y[2 * o] = yb[2 * m];
                    Y[2 * o + 1] = yb[2 * m + 1];
                }
            }

    /* 3. E-W exact phasing per (sample, pol, N-S beam) */
    for (int32_t t = 0; t < T; ++t)
        for (int32_t p = 0; p < NP; ++p)
            for (int32_t m = 0; m < NM; ++m) {
                size_t o = (((size_t)t * NP + p) * NM + m) * NC;
                orc_ew_beams(NC, NJ, w, &Y[2 * o], bj);
                for (int32_t j = 0; j < NJ; ++j) {
                    size_t ob = (((size_t)p * NJ + j) * NM + m) * T + t;
                    B[2 * ob] = bj[2 * j];
                    B[2 * ob + 1] = bj[2 * j + 1];
                }
            }

    free(k); free(roots); free(w); free(x); free(line); free(yb); free(Y); free(bj);
    return B;
}

/*
 * One channel-frame: raw bytes [n_time][n_cyl*n_feed*n_pol] in, Stokes-I
 * powers [n_beam_ew*n_beam_ns][n_dft] out.  `lut` gives the kept bin per N-S
 * beam; NULL means Eq. (1) at f_hz.
 */
int orc_beamform_unit(const orc_geom *g, double f_hz, const int32_t *lut,
                      const uint8_t *in, double *out)
{
    double *B = orc_beams_time(g, f_hz, lut, in);
    if (!B) return orc_check(g) ? -1 : -2;
    const int32_t NP = g->n_pol, NM = g->n_beam_ns, NJ = g->n_beam_ew, L = g->n_dft,
                  T = g->n_time;
    double *roots_l = (double *)malloc(sizeof(double) * 2 * L);
    double *u = (double *)malloc(sizeof(double) * 2 * L);
    if (!roots_l || !u) { free(B); free(roots_l); free(u); return -2; }
    orc_roots(L, roots_l);

    /* 4-5. up-channelise each block of L samples, Stokes I, integrate */
    memset(out, 0, sizeof(double) * (size_t)NJ * NM * L);
    for (int32_t j = 0; j < NJ; ++j)
        for (int32_t m = 0; m < NM; ++m)
            for (int32_t p = 0; p < NP; ++p)
                for (int32_t blk = 0; blk < T / L; ++blk) {
                    size_t ob = (((size_t)p * NJ + j) * NM + m) * T + (size_t)blk * L;
                    orc_upchan_tab(L, roots_l, &B[2 * ob], u);
                    for (int32_t s = 0; s < L; ++s) {
                        int32_t q = (s + L / 2) % L;
                        out[((size_t)j * NM + m) * L + q] +=
                            u[2 * s] * u[2 * s] + u[2 * s + 1] * u[2 * s + 1];
                    }
                }

    free(B); free(roots_l); free(u);
    return 0;
}

/*
 * The complex beams before detection for one channel-frame: the beams of
 * steps 1-3, each up-channelised per block of L samples (step 4), written as
 * out[blk][s][p][j][m] (complex; s the DFT bin, not centre-shifted).
 */
int orc_beams_unit(const orc_geom *g, double f_hz, const int32_t *lut, const uint8_t *in,
                   double *out)
{
    double *B = orc_beams_time(g, f_hz, lut, in);
    if (!B) return orc_check(g) ? -1 : -2;
    const int32_t NP = g->n_pol, NM = g->n_beam_ns, NJ = g->n_beam_ew, L = g->n_dft,
                  T = g->n_time;
    double *roots_l = (double *)malloc(sizeof(double) * 2 * L);
    double *u = (double *)malloc(sizeof(double) * 2 * L);
    if (!roots_l || !u) { free(B); free(roots_l); free(u); return -2; }
    orc_roots(L, roots_l);
    for (int32_t p = 0; p < NP; ++p)
        for (int32_t j = 0; j < NJ; ++j)
            for (int32_t m = 0; m < NM; ++m)
                for (int32_t blk = 0; blk < T / L; ++blk) {
                    size_t ob = (((size_t)p * NJ + j) * NM + m) * T + (size_t)blk * L;
                    orc_upchan_tab(L, roots_l, &B[2 * ob], u);
                    for (int32_t s = 0; s < L; ++s) {
                        size_t o = ((((size_t)blk * L + s) * NP + p) * NJ + j) * NM + m;
                        out[2 * o] = u[2 * s];
                        out[2 * o + 1] = u[2 * s + 1];
                    }
                }
    free(B); free(roots_l); free(u);
    return 0;
}

/*
 * Selected channel-frames of a batch.  in = [n_frames][n_chan][n_time][inputs]
 * bytes; unit u is (frame units[2u], channel units[2u+1]); out = [n_units]
 * [n_beam_ew*n_beam_ns][n_dft].  lut_override = [n_chan][n_beam_ns] or NULL.
 * Units are independent, so they are spread over n_threads OpenMP threads.
 */
int orc_beamform_units(const orc_geom *g, const double *freqs, int32_t n_chan,
                       const int32_t *lut_override, const uint8_t *in,
                       int32_t n_frames, const int32_t *units, int32_t n_units,
                       double *out, int32_t n_threads)
{
    if (orc_check(g) || !freqs || !in || !out || !units || n_chan <= 0 || n_frames <= 0)
        return -1;
    const size_t unit_in = (size_t)g->n_time * g->n_cyl * g->n_feed * g->n_pol;
    const size_t unit_out = (size_t)g->n_beam_ew * g->n_beam_ns * g->n_dft;
    for (int32_t u = 0; u < n_units; ++u)
        if (units[2 * u] < 0 || units[2 * u] >= n_frames ||
            units[2 * u + 1] < 0 || units[2 * u + 1] >= n_chan)
            return -1;
    int status = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads) reduction(min : status)
#endif
    for (int32_t u = 0; u < n_units; ++u) {
        int32_t f = units[2 * u], c = units[2 * u + 1];
        const uint8_t *src = in + ((size_t)f * n_chan + c) * unit_in;
        const int32_t *lut = lut_override ? lut_override + (size_t)c * g->n_beam_ns : NULL;
        int r = orc_beamform_unit(g, freqs[c], lut, src, out + (size_t)u * unit_out);
        if (r < status) status = r;
    }
    return status;
}

/* Every channel-frame of a batch: out = [n_frames][n_chan][beams][n_dft]. */
int orc_beamform(const orc_geom *g, const double *freqs, int32_t n_chan,
                 const int32_t *lut_override, const uint8_t *in, int32_t n_frames,
                 double *out, int32_t n_threads)
{
    if (n_frames <= 0 || n_chan <= 0) return -1;
    int32_t n_units = n_frames * n_chan;
    int32_t *units = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)n_units);
    if (!units) return -2;
    for (int32_t f = 0; f < n_frames; ++f)
        for (int32_t c = 0; c < n_chan; ++c) {
            units[2 * (f * n_chan + c)] = f;
            units[2 * (f * n_chan + c) + 1] = c;
        }
    int r = orc_beamform_units(g, freqs, n_chan, lut_override, in, n_frames, units,
                               n_units, out, n_threads);
    free(units);
    return r;
}

/*
 * The paper's own up-channelisation (Sec. 3, Sec. 3.2): a 128-point DFT of
 * every 128 samples (3.05 kHz fine channels), squared, then integrated to 16
 * sub-channels of 24.4 kHz per 0.983 ms.  With the fine powers from
 * orc_beamform at n_dft = L (centre-shifted fine bin q', summed over blocks and
 * pols), coarse sub-channel q sums the G fine bins nearest its centre:
 * q = ((q' + G/2) / G) mod (L/G), i.e. fine bins q' = G q - G/2 .. G q + G/2 - 1
 * (mod L).  fine = [rows][L], coarse = [rows][L/G].
 */
void orc_group_bins(const double *fine, int64_t rows, int32_t L, int32_t G, double *coarse)
{
    const int32_t nq = L / G;
    for (int64_t r = 0; r < rows; ++r) {
        for (int32_t q = 0; q < nq; ++q) coarse[r * nq + q] = 0.0;
        for (int32_t qf = 0; qf < L; ++qf) {
            int32_t q = ((qf + G / 2) / G) % nq;
            coarse[r * nq + q] += fine[r * L + qf];
        }
    }
}

/*
 * 8-bit output (Sec. 3, Table 1: the integrated beams are rescaled to 8-bit
 * integers; the paper gives no rule).  Reading: an affine rescale per output,
 * code = clamp(rint(P * scale + offset), 0, 255).  The code is an integer
 * decided by floating point, so it is decided in the library's precision:
 * P rounded to FP32, one FP32 fused multiply-add, rint (round half to even).
 * A NaN argument gives code 0.
 */
void orc_rescale_u8(const double *P, const float *scale, const float *offset, int64_t n,
                    uint8_t *out)
{
    for (int64_t i = 0; i < n; ++i) {
        float x = rintf(fmaf((float)P[i], scale[i], offset[i]));
        if (!(x >= 0.0f)) x = 0.0f;
        if (x > 255.0f) x = 255.0f;
        out[i] = (uint8_t)x;
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
