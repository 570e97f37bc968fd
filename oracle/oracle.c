/*
 * ORACLE -- test infrastructure only.  Plain, slow, obviously correct CPU loops
 * that define what the dedispersion library must compute.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load this library; the
 * product path never does.  Shares no code with the HIP library.
 *
 * Everything here is written straight from the paper's definitions:
 *   - eq. p_dedisp (Section 2.1): the dedispersed series of a trial is the sum of
 *     the selected dynamic-spectrum samples, shifted by the output index n.  A
 *     trial's sample set is stored per channel as a contiguous run
 *     {start[d,c] + k : 0 <= k < ntap[d,c]}, optionally weighted per channel or
 *     per tap (the weighted form is the matched-filter family of Section 4).
 *   - eq. snr (Section 2.1) normalises the sum by the noise standard deviation;
 *     the boxcar detector of Section 4 sums W consecutive outputs.  The noise
 *     variance of a boxcar of the dedispersed series is the exact variance of
 *     that linear functional of independent channel noise.
 *   - the adjoint sums are the transposes of the dedispersion sum.
 * Integers accumulate in int64, floating point in double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_U8 = 0, OR_F32 = 1, OR_F64 = 2, OR_I32 = 3 };
enum { OR_W_UNIT = 0, OR_W_CHANNEL = 1, OR_W_TAP = 2 };

static double load_in(const void *x, int dt, int64_t i) {
  switch (dt) {
    case OR_U8: return (double)((const uint8_t *)x)[i];
    case OR_F32: return (double)((const float *)x)[i];
    case OR_F64: return ((const double *)x)[i];
    default: return (double)((const int32_t *)x)[i];
  }
}

static double weight(int wmode, int ktaps, const float *w, int c, int k) {
  if (wmode == OR_W_UNIT) return 1.0;
  if (wmode == OR_W_CHANNEL) return (double)w[c];
  return (double)w[(int64_t)c * ktaps + k];
}

/* Integer dedispersion of uint8 data with unit weights, eq. p_dedisp:
 *   y[d,t] = sum_c sum_{k<ntap[d,c]} x[c, t + start[d,c] + k],  0 <= t < tout.
 * Returns 0, or -1 if a sample index would fall outside [0, nsamp). */
int oracle_dedisperse_u8(int32_t nchan, int64_t nsamp, const uint8_t *x, int64_t xstride,
                         int32_t ndm, const int32_t *start, const int32_t *ntap,
                         int64_t tout, int64_t *y, int64_t ystride) {
  for (int32_t d = 0; d < ndm; ++d) {
    for (int64_t t = 0; t < tout; ++t) {
      int64_t acc = 0;
      for (int32_t c = 0; c < nchan; ++c) {
        int64_t s = start[(int64_t)d * nchan + c];
        int32_t n = ntap[(int64_t)d * nchan + c];
        for (int32_t k = 0; k < n; ++k) {
          int64_t i = t + s + k;
          if (i < 0 || i >= nsamp) return -1;
          acc += x[(int64_t)c * xstride + i];
        }
      }
      y[(int64_t)d * ystride + t] = acc;
    }
  }
  return 0;
}

/* Weighted dedispersion in double precision (same sum, with per-channel or per-tap
 * weights w_{c,k}); the input may be uint8, fp32 or fp64.  `nbatch` independent
 * filterbanks x[b][c][t] (batch stride xbstride) give y[b][d][t]. */
int oracle_dedisperse_f64(int32_t nbatch, int32_t nchan, int64_t nsamp, const void *x, int xdtype,
                          int64_t xstride, int64_t xbstride, int32_t ndm, const int32_t *start,
                          const int32_t *ntap, int wmode, int32_t ktaps, const float *w,
                          int64_t tout, double *y, int64_t ystride, int64_t ybstride) {
  for (int32_t b = 0; b < nbatch; ++b) {
    for (int32_t d = 0; d < ndm; ++d) {
      for (int64_t t = 0; t < tout; ++t) {
        double acc = 0.0;
        for (int32_t c = 0; c < nchan; ++c) {
          int64_t s = start[(int64_t)d * nchan + c];
          int32_t n = ntap[(int64_t)d * nchan + c];
          for (int32_t k = 0; k < n; ++k) {
            int64_t i = t + s + k;
            if (i < 0 || i >= nsamp) return -1;
            acc += weight(wmode, ktaps, w, c, k) *
                   load_in(x, xdtype, (int64_t)b * xbstride + (int64_t)c * xstride + i);
          }
        }
        y[(int64_t)b * ybstride + (int64_t)d * ystride + t] = acc;
      }
    }
  }
  return 0;
}

/* Noise statistics of a width-W boxcar of the dedispersed series of trial d.
 * B_W[t] = sum_{j<W} y[t+j] = sum_c sum_tau a_c[tau] x[c, t + start + tau] with
 * a_c = (w_{d,c} convolved with a length-W box).  With independent channel noise
 * of mean mu_c and standard deviation sigma_c:
 *   mean  M = sum_c mu_c * sum_tau a_c[tau]
 *   var   S^2 = sum_c sigma_c^2 * sum_tau a_c[tau]^2.
 * The convolution is written out explicitly.  Outputs are [ndm][nw]. */
int oracle_boxcar_norm(int32_t nchan, int32_t ndm, const int32_t *ntap, int wmode, int32_t ktaps,
                       const float *w, const double *mu, const double *sigma, int32_t nw,
                       const int32_t *widths, double *M, double *S) {
  int32_t nmax = 0;
  for (int64_t i = 0; i < (int64_t)ndm * nchan; ++i)
    if (ntap[i] > nmax) nmax = ntap[i];
  int32_t wmax = 0;
  for (int32_t j = 0; j < nw; ++j)
    if (widths[j] > wmax) wmax = widths[j];
  double *a = (double *)malloc(sizeof(double) * (size_t)(nmax + wmax + 1));
  if (!a) return -1;
  for (int32_t d = 0; d < ndm; ++d) {
    for (int32_t j = 0; j < nw; ++j) {
      int32_t W = widths[j];
      double m = 0.0, v = 0.0;
      for (int32_t c = 0; c < nchan; ++c) {
        int32_t n = ntap[(int64_t)d * nchan + c];
        int32_t L = n + W - 1;
        if (n == 0) continue;
        for (int32_t tau = 0; tau < L; ++tau) a[tau] = 0.0;
        for (int32_t k = 0; k < n; ++k)
          for (int32_t q = 0; q < W; ++q) a[k + q] += weight(wmode, ktaps, w, c, k);
        double s1 = 0.0, s2 = 0.0;
        for (int32_t tau = 0; tau < L; ++tau) {
          s1 += a[tau];
          s2 += a[tau] * a[tau];
        }
        m += mu[c] * s1;
        v += sigma[c] * sigma[c] * s2;
      }
      M[(int64_t)d * nw + j] = m;
      S[(int64_t)d * nw + j] = sqrt(v);
    }
  }
  free(a);
  return 0;
}

/* Boxcar S/N search over a dedispersed block y[ndm][tout] (values in double;
 * integers are exact).  For each trial d, every width W in `widths` and every
 * start 0 <= t <= tout - W:
 *   B = sum_{j<W} y[d, t + j]   (direct loop),
 *   snr = (B - M[d,W]) / S[d,W].
 * The winner maximises snr; exact ties go to the smaller width (by value), then
 * the smaller t.  Widths longer than tout are skipped.  A trial with no valid
 * window reports snr = -inf, t = -1, w = 0. */
void oracle_boxcar_detect(int32_t ndm, int64_t tout, const double *y, int64_t ystride, int32_t nw,
                          const int32_t *widths, const double *M, const double *S,
                          double *snr_out, int32_t *t_out, int32_t *w_out) {
  for (int32_t d = 0; d < ndm; ++d) {
    double best = -INFINITY;
    int32_t bt = -1, bw = 0;
    const double *yd = y + (int64_t)d * ystride;
    for (int32_t j = 0; j < nw; ++j) {
      int32_t W = widths[j];
      if (W > tout) continue;
      double m = M[(int64_t)d * nw + j], s = S[(int64_t)d * nw + j];
      for (int64_t t = 0; t + W <= tout; ++t) {
        double B = 0.0;
        for (int32_t q = 0; q < W; ++q) B += yd[t + q];
        double r = (B - m) / s;
        int better = r > best || (r == best && (W < bw || (W == bw && t < bt)));
        if (better) {
          best = r;
          bt = (int32_t)t;
          bw = W;
        }
      }
    }
    snr_out[d] = best;
    t_out[d] = bt;
    w_out[d] = bw;
  }
}

/* Adjoint of the weighted dedispersion with respect to the weights:
 *   gw[c,k] = sum_b sum_d sum_t g[b,d,t] * x[b, c, t + start[d,c] + k]   (k < ntap[d,c]).
 * For per-channel weights (wmode 1) the k-sum is folded into gw[c]. */
int oracle_adjoint_w(int32_t nbatch, int32_t nchan, int64_t nsamp, const void *x, int xdtype,
                     int64_t xstride, int64_t xbstride, int32_t ndm, const int32_t *start,
                     const int32_t *ntap, int wmode, int32_t ktaps, int64_t tout, const double *g,
                     int64_t gstride, int64_t gbstride, double *gw) {
  int32_t K = wmode == OR_W_TAP ? ktaps : 1;
  memset(gw, 0, sizeof(double) * (size_t)nchan * K);
  for (int32_t b = 0; b < nbatch; ++b)
    for (int32_t d = 0; d < ndm; ++d)
      for (int32_t c = 0; c < nchan; ++c) {
        int64_t s = start[(int64_t)d * nchan + c];
        int32_t n = ntap[(int64_t)d * nchan + c];
        for (int32_t k = 0; k < n; ++k)
          for (int64_t t = 0; t < tout; ++t) {
            int64_t i = t + s + k;
            if (i < 0 || i >= nsamp) return -1;
            double gv = g[(int64_t)b * gbstride + (int64_t)d * gstride + t];
            double xv = load_in(x, xdtype, (int64_t)b * xbstride + (int64_t)c * xstride + i);
            gw[(int64_t)c * K + (wmode == OR_W_TAP ? k : 0)] += gv * xv;
          }
      }
  return 0;
}

/* Adjoint with respect to the input samples:
 *   gx[b,c,i] = sum_d sum_{k<ntap[d,c]} w_{c,k} * g[b, d, i - start[d,c] - k]
 * (terms with the output index outside [0, tout) are absent). */
int oracle_adjoint_x(int32_t nbatch, int32_t nchan, int64_t nsamp, int32_t ndm,
                     const int32_t *start, const int32_t *ntap, int wmode, int32_t ktaps,
                     const float *w, int64_t tout, const double *g, int64_t gstride,
                     int64_t gbstride, double *gx, int64_t xstride, int64_t xbstride) {
  for (int32_t b = 0; b < nbatch; ++b)
    for (int32_t c = 0; c < nchan; ++c)
      for (int64_t i = 0; i < nsamp; ++i) gx[(int64_t)b * xbstride + (int64_t)c * xstride + i] = 0.0;
  for (int32_t b = 0; b < nbatch; ++b)
    for (int32_t d = 0; d < ndm; ++d)
      for (int32_t c = 0; c < nchan; ++c) {
        int64_t s = start[(int64_t)d * nchan + c];
        int32_t n = ntap[(int64_t)d * nchan + c];
        for (int32_t k = 0; k < n; ++k) {
          double wk = weight(wmode, ktaps, w, c, k);
          for (int64_t t = 0; t < tout; ++t) {
            int64_t i = t + s + k;
            if (i < 0 || i >= nsamp) return -1;
            gx[(int64_t)b * xbstride + (int64_t)c * xstride + i] +=
                wk * g[(int64_t)b * gbstride + (int64_t)d * gstride + t];
          }
        }
      }
  return 0;
}

/* Selected outputs of the weighted sum, one by one: y_e = y[b_e][d_e][t_e]. */
int oracle_dedisperse_points(int32_t nchan, int64_t nsamp, const void *x, int xdtype,
                             int64_t xstride, int64_t xbstride, const int32_t *start,
                             const int32_t *ntap, int wmode, int32_t ktaps, const float *w,
                             int32_t npts, const int32_t *pb, const int32_t *pd,
                             const int64_t *pt, double *out) {
  for (int32_t e = 0; e < npts; ++e) {
    double acc = 0.0;
    for (int32_t c = 0; c < nchan; ++c) {
      int64_t s = start[(int64_t)pd[e] * nchan + c];
      int32_t n = ntap[(int64_t)pd[e] * nchan + c];
      for (int32_t k = 0; k < n; ++k) {
        int64_t i = pt[e] + s + k;
        if (i < 0 || i >= nsamp) return -1;
        acc += weight(wmode, ktaps, w, c, k) *
               load_in(x, xdtype, (int64_t)pb[e] * xbstride + (int64_t)c * xstride + i);
      }
    }
    out[e] = acc;
  }
  return 0;
}
