// Host half of libdedisp: argument checks, error reporting, the sample-set tables
// of every profile rule, the trial-DM rule and the lazy device upload.
//
// All delay arithmetic is double precision with no contraction into fused
// multiply-adds (the library is built with -ffp-contract=off), so that floor and
// ceil of the delays are reproducible from the stated expressions.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <tuple>

#include <mutex>
#include "internal.h"

namespace dd {

static thread_local std::string g_last_error;
thread_local const float *tl_weights = nullptr;

void set_error(const std::string &msg) { g_last_error = msg; }

dedisp_status fail(dedisp_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

dedisp_status hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return DEDISP_ERR_DEVICE;
}

// Delay constant of Section 2.1: t_d = DM / (kappa nu^2), kappa = 2.41e-16 pc cm^-3 s,
// i.e. K = 1 / (kappa * 1e18) seconds for nu in GHz.
static double paper_kdm() { return 1.0 / (2.41e-16 * 1e18); }

// ---------------------------------------------------------------------------------
// Rectangular pulse model for the GREEDY rule (App. A, eq. dispersed pulse)
// ---------------------------------------------------------------------------------
namespace {

struct GaussLegendre {
  static constexpr int N = 16;
  double x[N], w[N];
  GaussLegendre() {
    for (int i = 0; i < N; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (N + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = 0.0;
        for (int k = 1; k <= N; ++k) {
          double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
        }
        double dp = N * (z * p0 - p1) / (z * z - 1.0);
        double dz = p0 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) {
          double pp = dp;
          x[i] = z;
          // recompute derivative at the converged node
          double q0 = 1.0, q1 = 0.0;
          for (int k = 1; k <= N; ++k) {
            double q2 = q1;
            q1 = q0;
            q0 = ((2.0 * k - 1.0) * z * q1 - (k - 1.0) * q2) / k;
          }
          pp = N * (z * q0 - q1) / (z * z - 1.0);
          w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
          break;
        }
      }
    }
  }
};

const GaussLegendre &gl() {
  static GaussLegendre g;
  return g;
}

struct RectModel {
  double kdm, dm, nu_hi, width, scat, sidx, alpha, nu0;
  double td(double nu) const { return kdm * dm * (1.0 / (nu * nu) - 1.0 / (nu_hi * nu_hi)); }
  double taup(double nu) const { return width + scat * std::pow(nu, sidx); }
  // Mean power of the cell [t0, t0+dt] x [flo, fhi].
  double cell(double t0, double dt, double flo, double fhi) const {
    const double t1 = t0 + dt;
    double cuts[8];
    int nc = 0;
    cuts[nc++] = flo;
    // Edges of the delayed rectangle, both decreasing in nu: td(nu) and td(nu)+tau'(nu).
    for (int e = 0; e < 2; ++e) {
      for (int k = 0; k < 2; ++k) {
        double tc = k == 0 ? t0 : t1;
        auto g = [&](double nu) { return (e == 0 ? td(nu) : td(nu) + taup(nu)) - tc; };
        double ga = g(flo), gb = g(fhi);
        if ((ga > 0 && gb < 0) || (ga < 0 && gb > 0)) {
          double a = flo, b = fhi;
          for (int it = 0; it < 200 && b - a > 0; ++it) {
            double m = 0.5 * (a + b);
            if (m <= a || m >= b) break;
            if ((g(m) > 0) == (ga > 0)) a = m; else b = m;
          }
          cuts[nc++] = 0.5 * (a + b);
        }
      }
    }
    cuts[nc++] = fhi;
    std::sort(cuts, cuts + nc);
    const GaussLegendre &G = gl();
    double tot = 0.0;
    for (int i = 0; i + 1 < nc; ++i) {
      double a = cuts[i], b = cuts[i + 1];
      if (!(b > a)) continue;
      double h = 0.5 * (b - a), m = 0.5 * (a + b), part = 0.0;
      for (int q = 0; q < GaussLegendre::N; ++q) {
        double nu = m + h * G.x[q];
        double lo = td(nu), tp = taup(nu), hi = lo + tp;
        double ov = std::min(t1, hi) - std::max(t0, lo);
        if (ov > 0) part += G.w[q] * std::pow(nu / nu0, -alpha) * ov * (width / tp);
      }
      tot += h * part;
    }
    return tot / dt;
  }
};

}  // namespace

// ---------------------------------------------------------------------------------
// Tables
// ---------------------------------------------------------------------------------
static dedisp_status build_tables(dedisp_plan p) {
  const int32_t C = p->nchan, D = p->ndm;
  const double bw = p->chan_bw, dt = p->dt, k = p->kdm;
  std::vector<double> ft(C), fl(C);
  double fh = -1.0;
  for (int32_t c = 0; c < C; ++c) {
    ft[c] = p->freq[c] + 0.5 * bw;
    fl[c] = p->freq[c] - 0.5 * bw;
    fh = std::max(fh, ft[c]);
  }
  p->start.assign((size_t)D * C, 0);
  p->ntap.assign((size_t)D * C, 0);
  const int rule = p->prof.rule;
  if (rule == DEDISP_RULE_EXPLICIT) {
    for (size_t i = 0; i < (size_t)D * C; ++i) {
      p->start[i] = p->prof.start[i];
      p->ntap[i] = p->prof.ntap[i];
      if (p->ntap[i] < 0) return fail(DEDISP_ERR_INVALID_ARG, "explicit ntap < 0");
      if (p->start[i] < 0) return fail(DEDISP_ERR_INVALID_ARG, "explicit start < 0");
    }
  } else {
    for (int32_t d = 0; d < D; ++d) {
      const double dm = p->dm[d];
      for (int32_t c = 0; c < C; ++c) {
        // start = floor(t_A / dt), t_A the delay of the channel's top edge
        // relative to the top of the band (Section 3).
        const double ta = k * dm * (1.0 / (ft[c] * ft[c]) - 1.0 / (fh * fh)) / dt;
        const double sA = std::floor(ta);
        if (!(sA < 2147483647.0)) return fail(DEDISP_ERR_OVERFLOW, "delay exceeds int32 samples");
        int32_t n = 1;
        if (rule == DEDISP_RULE_SMEAR) {
          const double sm = k * dm * (1.0 / (fl[c] * fl[c]) - 1.0 / (ft[c] * ft[c])) / dt;
          n = (int32_t)std::max(1.0, std::ceil(sm));
        } else if (rule == DEDISP_RULE_ALLNONZERO || rule == DEDISP_RULE_GREEDY) {
          const double taup =
              p->prof.width_s + p->prof.scatter_s_1ghz * std::pow(fl[c], p->prof.scatter_index);
          const double tb = (k * dm * (1.0 / (fl[c] * fl[c]) - 1.0 / (fh * fh)) + taup) / dt;
          n = (int32_t)std::max(1.0, std::ceil(tb) - sA);
        } else if (rule == DEDISP_RULE_FIXED) {
          n = p->prof.ktaps;
        }
        p->start[(size_t)d * C + c] = (int32_t)sA;
        p->ntap[(size_t)d * C + c] = n;
      }
    }
    if (rule == DEDISP_RULE_GREEDY) {
      // Section 2.2: predict each candidate cell's power with the rectangular
      // pulse model, add cells in decreasing order of power while
      // eq. sel_criterion holds.  Candidates are the ALLNONZERO runs above.
      RectModel m{k, 0.0, fh, p->prof.width_s, p->prof.scatter_s_1ghz, p->prof.scatter_index,
                  p->prof.spectral_index, p->prof.nu0_ghz > 0 ? p->prof.nu0_ghz : 1.0};
      if (!(p->prof.width_s > 0)) return fail(DEDISP_ERR_INVALID_ARG, "greedy rule needs width_s > 0");
      std::vector<std::tuple<double, int32_t, int32_t>> cand;
      for (int32_t d = 0; d < D; ++d) {
        m.dm = p->dm[d];
        cand.clear();
        for (int32_t c = 0; c < C; ++c) {
          const int32_t s0 = p->start[(size_t)d * C + c], n0 = p->ntap[(size_t)d * C + c];
          for (int32_t j = s0; j < s0 + n0; ++j) {
            double v = m.cell(j * dt, dt, fl[c], ft[c]);
            if (v > 0.0) cand.emplace_back(v, c, j);
          }
        }
        std::sort(cand.begin(), cand.end(), [](const auto &a, const auto &b) {
          if (std::get<0>(a) != std::get<0>(b)) return std::get<0>(a) > std::get<0>(b);
          if (std::get<1>(a) != std::get<1>(b)) return std::get<1>(a) < std::get<1>(b);
          return std::get<2>(a) < std::get<2>(b);
        });
        std::vector<int32_t> lo(C, INT32_MAX), hi(C, -1), cnt(C, 0);
        double total = 0.0;
        size_t nsel = 0;
        for (size_t i = 0; i < cand.size(); ++i) {
          const double v = std::get<0>(cand[i]);
          if (nsel > 0) {
            const double N = (double)nsel;
            if (!(v > (std::sqrt((N + 1.0) / N) - 1.0) * total)) break;
          }
          total += v;
          ++nsel;
          const int32_t c = std::get<1>(cand[i]), j = std::get<2>(cand[i]);
          lo[c] = std::min(lo[c], j);
          hi[c] = std::max(hi[c], j);
          cnt[c] += 1;
        }
        for (int32_t c = 0; c < C; ++c) {
          if (cnt[c] == 0) {
            p->ntap[(size_t)d * C + c] = 0;
            continue;
          }
          if (hi[c] - lo[c] + 1 != cnt[c])
            return fail(DEDISP_ERR_UNSUPPORTED, "greedy selection is not contiguous in a channel");
          p->start[(size_t)d * C + c] = lo[c];
          p->ntap[(size_t)d * C + c] = cnt[c];
        }
      }
    }
  }
  // An empty run contributes nothing; store it at start 0 so that no kernel
  // ever forms an address from its (irrelevant) start.
  for (size_t i = 0; i < p->ntap.size(); ++i)
    if (p->ntap[i] == 0) p->start[i] = 0;
  int32_t span = 0, nmax = 0, smin = INT32_MAX;
  int64_t summax = 0, rows = 0;
  for (int32_t c = 0; c < C; ++c) {
    int32_t cm = 0, cl = INT32_MAX;
    for (int32_t d = 0; d < D; ++d) {
      const int32_t s = p->start[(size_t)d * C + c], n = p->ntap[(size_t)d * C + c];
      if (n > 0) span = std::max(span, s + n);
      smin = std::min(smin, s);
      cm = std::max(cm, n);
      cl = std::min(cl, n);
    }
    nmax = std::max(nmax, cm);
    summax += cm;
    rows += cm - cl + 1;
  }
  p->max_span = std::max(span, 1);
  p->max_ntap = nmax;
  p->min_start = smin;
  p->sum_max_ntap = summax;
  p->window_rows = rows;
  if (p->wmode == DEDISP_W_TAP) {
    for (size_t i = 0; i < p->ntap.size(); ++i)
      if (p->ntap[i] != p->ktaps)
        return fail(DEDISP_ERR_UNSUPPORTED, "per-tap weights need ntap == ktaps everywhere");
  }
  return DEDISP_OK;
}

bool alloc_fails() {
  static std::mutex mu;
  static std::string last;
  static long count = 0;
  const char *v = getenv("DEDISP_TEST_FAIL_ALLOC");
  std::lock_guard<std::mutex> lk(mu);
  if (!v || !*v) {
    last.clear();
    count = 0;
    return false;
  }
  if (last != v) {
    last = v;
    count = 0;
  }
  return ++count == strtol(v, nullptr, 10);
}

bool log_enabled() {
  const char *v = getenv("DEDISP_LOG");
  return v && *v && strcmp(v, "0") != 0;
}

void log_plan(const dedisp_plan_s *p) {
  static const char *const kRules[] = {"smear", "allnonzero", "greedy", "explicit", "fixed"};
  static const char *const kWeights[] = {"unit", "channel", "tap"};
  const int rule = p->prof.rule >= 0 && p->prof.rule <= DEDISP_RULE_FIXED ? p->prof.rule : 0;
  const int wm = p->wmode >= 0 && p->wmode <= DEDISP_W_TAP ? p->wmode : 0;
  int32_t nmin = INT32_MAX;
  for (int32_t n : p->ntap) nmin = std::min(nmin, n);
  fprintf(stderr,
          "dedisp: plan %p: %d trials x %d channels, DM %.6g..%.6g, rule %s, weights %s, "
          "samples per channel %d..%d, longest run %d samples (outputs = block length - %d)\n",
          (const void *)p, p->ndm, p->nchan, p->dm.front(), p->dm.back(), kRules[rule],
          kWeights[wm], p->ntap.empty() ? 0 : nmin, p->max_ntap, p->max_span, p->max_span - 1);
}

hipError_t dev_malloc(void **p, size_t bytes) {
  if (alloc_fails()) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}

hipError_t dev_malloc_async(void **p, size_t bytes, hipStream_t s) {
  if (alloc_fails()) return hipErrorOutOfMemory;
  return hipMallocAsync(p, bytes, s);
}

dedisp_status ensure_device(dedisp_plan p) {
  std::lock_guard<std::mutex> lk(p->mu);
  int dev = 0;
  DD_HIP(hipGetDevice(&dev));
  if (p->uploaded) {
    if (dev != p->device) return fail(DEDISP_ERR_INVALID_ARG, "plan used on a second device");
    return DEDISP_OK;
  }
  const size_t n = (size_t)p->ndm * p->nchan;
  DD_HIP(dev_malloc((void **)&p->dev.start, n * sizeof(int32_t)));
  DD_HIP(dev_malloc((void **)&p->dev.ntap, n * sizeof(int32_t)));
  DD_HIP(hipMemcpy(p->dev.start, p->start.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
  DD_HIP(hipMemcpy(p->dev.ntap, p->ntap.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
  if (!p->weights.empty()) {
    DD_HIP(dev_malloc((void **)&p->dev.weights, p->weights.size() * sizeof(float)));
    DD_HIP(hipMemcpy(p->dev.weights, p->weights.data(), p->weights.size() * sizeof(float),
                     hipMemcpyHostToDevice));
  }
  p->device = dev;
  p->uploaded = true;
  return DEDISP_OK;
}

}  // namespace dd

using dd::fail;

extern "C" {

dedisp_status dedisp_profile_init(dedisp_profile *prof) {
  if (!prof) return fail(DEDISP_ERR_INVALID_ARG, "null profile");
  std::memset(prof, 0, sizeof(*prof));
  prof->rule = DEDISP_RULE_SMEAR;
  prof->scatter_index = -4.0;
  prof->ktaps = 1;
  prof->wmode = DEDISP_W_UNIT;
  return DEDISP_OK;
}

dedisp_status dedisp_plan_create(dedisp_plan *out, int32_t nchan, const double *freq_ghz,
                                 double chan_bw_ghz, double dt_s, int32_t ndm, const double *dm,
                                 const dedisp_profile *prof) {
  if (!out) return fail(DEDISP_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (nchan <= 0 || ndm <= 0) return fail(DEDISP_ERR_INVALID_ARG, "nchan and ndm must be > 0");
  if (!freq_ghz || !dm) return fail(DEDISP_ERR_INVALID_ARG, "null freq or dm array");
  if (!(chan_bw_ghz > 0) || !std::isfinite(chan_bw_ghz))
    return fail(DEDISP_ERR_INVALID_ARG, "chan_bw must be finite and > 0");
  if (!(dt_s > 0) || !std::isfinite(dt_s)) return fail(DEDISP_ERR_INVALID_ARG, "dt must be finite and > 0");
  for (int32_t c = 0; c < nchan; ++c)
    if (!std::isfinite(freq_ghz[c]) || !(freq_ghz[c] - 0.5 * chan_bw_ghz > 0))
      return fail(DEDISP_ERR_INVALID_ARG, "channel frequencies must be finite with positive low edge");
  for (int32_t d = 0; d < ndm; ++d)
    if (!std::isfinite(dm[d]) || dm[d] < 0) return fail(DEDISP_ERR_INVALID_ARG, "DMs must be finite and >= 0");
  dedisp_profile pr;
  if (prof) pr = *prof; else dedisp_profile_init(&pr);
  if (pr.rule < 0 || pr.rule > DEDISP_RULE_FIXED) return fail(DEDISP_ERR_INVALID_ARG, "bad rule");
  if (pr.wmode < 0 || pr.wmode > DEDISP_W_TAP) return fail(DEDISP_ERR_INVALID_ARG, "bad weight mode");
  if (!(pr.k_dm >= 0) || !std::isfinite(pr.k_dm)) return fail(DEDISP_ERR_INVALID_ARG, "bad k_dm");
  if (pr.rule == DEDISP_RULE_EXPLICIT && (!pr.start || !pr.ntap))
    return fail(DEDISP_ERR_INVALID_ARG, "explicit rule needs start and ntap");
  if ((pr.rule == DEDISP_RULE_FIXED || pr.wmode == DEDISP_W_TAP) && (pr.ktaps < 1 || pr.ktaps > 64))
    return fail(DEDISP_ERR_INVALID_ARG, "ktaps must be in [1, 64]");
  if (pr.wmode != DEDISP_W_UNIT && !pr.weights) return fail(DEDISP_ERR_INVALID_ARG, "weights required");
  if (!std::isfinite(pr.width_s) || pr.width_s < 0 || !std::isfinite(pr.scatter_s_1ghz) ||
      pr.scatter_s_1ghz < 0 || !std::isfinite(pr.scatter_index) || !std::isfinite(pr.spectral_index))
    return fail(DEDISP_ERR_INVALID_ARG, "bad pulse-model parameters");

  dedisp_plan p = dd::alloc_fails() ? nullptr : new (std::nothrow) dedisp_plan_s;
  if (!p) return fail(DEDISP_ERR_OOM, "host allocation failed");
  try {
    if (dd::alloc_fails()) throw std::bad_alloc();   // the tables' storage
    p->nchan = nchan;
    p->ndm = ndm;
    p->chan_bw = chan_bw_ghz;
    p->dt = dt_s;
    p->kdm = pr.k_dm > 0 ? pr.k_dm : dd::paper_kdm();
    p->freq.assign(freq_ghz, freq_ghz + nchan);
    p->dm.assign(dm, dm + ndm);
    p->prof = pr;
    p->wmode = pr.wmode;
    p->ktaps = pr.wmode == DEDISP_W_TAP ? pr.ktaps : 1;
    if (pr.wmode == DEDISP_W_CHANNEL) p->weights.assign(pr.weights, pr.weights + nchan);
    if (pr.wmode == DEDISP_W_TAP) p->weights.assign(pr.weights, pr.weights + (size_t)nchan * pr.ktaps);
    for (float w : p->weights)
      if (!std::isfinite(w)) {
        delete p;
        return fail(DEDISP_ERR_INVALID_ARG, "non-finite weight");
      }
    // The stored profile must not keep caller pointers.
    p->prof.start = nullptr;
    p->prof.ntap = nullptr;
    p->prof.weights = nullptr;
    dedisp_profile tmp = pr;
    p->prof = tmp;
    dedisp_status st = dd::build_tables(p);
    p->prof.start = nullptr;
    p->prof.ntap = nullptr;
    p->prof.weights = nullptr;
    if (st != DEDISP_OK) {
      delete p;
      return st;
    }
  } catch (const std::bad_alloc &) {
    delete p;
    return fail(DEDISP_ERR_OOM, "host allocation failed");
  }
  if (dd::log_enabled()) dd::log_plan(p);
  *out = p;
  return DEDISP_OK;
}

dedisp_status dedisp_plan_destroy(dedisp_plan p) {
  if (!p) return fail(DEDISP_ERR_INVALID_ARG, "null plan");
  if (p->uploaded) {
    (void)hipFree(p->dev.start);
    (void)hipFree(p->dev.ntap);
    if (p->dev.weights) (void)hipFree(p->dev.weights);
  }
  if (p->tiled) dd::free_tiled(p->tiled);
  if (p->f32) dd::free_f32(p->f32);
  if (p->f32_adj) dd::free_f32(p->f32_adj);
  if (p->mfma) dd::free_mfma(p->mfma);
  delete p;
  return DEDISP_OK;
}

dedisp_status dedisp_plan_tables(dedisp_plan p, int32_t *start, int32_t *ntap) {
  if (!p) return fail(DEDISP_ERR_INVALID_ARG, "null plan");
  const size_t n = (size_t)p->ndm * p->nchan;
  if (start) std::memcpy(start, p->start.data(), n * sizeof(int32_t));
  if (ntap) std::memcpy(ntap, p->ntap.data(), n * sizeof(int32_t));
  return DEDISP_OK;
}

dedisp_status dedisp_plan_info(dedisp_plan p, int32_t *nchan, int32_t *ndm, int32_t *max_span,
                               int32_t *ktaps, int32_t *wmode) {
  if (!p) return fail(DEDISP_ERR_INVALID_ARG, "null plan");
  if (nchan) *nchan = p->nchan;
  if (ndm) *ndm = p->ndm;
  if (max_span) *max_span = p->max_span;
  if (ktaps) *ktaps = p->ktaps;
  if (wmode) *wmode = p->wmode;
  return DEDISP_OK;
}

dedisp_status dedisp_plan_out_len(dedisp_plan p, int64_t nsamp, int64_t *nout) {
  if (!p || !nout) return fail(DEDISP_ERR_INVALID_ARG, "null argument");
  *nout = nsamp - p->max_span + 1;
  if (*nout < 1) return fail(DEDISP_ERR_SHAPE, "block shorter than the longest sample run");
  return DEDISP_OK;
}

dedisp_status dedisp_trial_dms(double dm0, double dm_max, double eps, int32_t nchan,
                               const double *freq_ghz, double chan_bw_ghz, double dt_s,
                               double tau_av_s, int32_t include_dm_tau, double k_dm, int32_t cap,
                               double *out, int32_t *n_out) {
  if (!freq_ghz || !out || !n_out || nchan <= 0 || cap <= 0)
    return fail(DEDISP_ERR_INVALID_ARG, "bad trial-DM arguments");
  if (!(eps > 0) || !std::isfinite(eps) || !(dm0 >= 0) || !std::isfinite(dm0) || std::isnan(dm_max) ||
      !(chan_bw_ghz > 0) || !(dt_s > 0) || !(tau_av_s >= 0))
    return fail(DEDISP_ERR_INVALID_ARG, "bad trial-DM parameters");
  const double K = k_dm > 0 ? k_dm : dd::paper_kdm();
  // Mean of nu_c^-3 over channel centres, and the two smearing DMs of Section 5.2.
  double m3 = 0.0;
  for (int32_t c = 0; c < nchan; ++c) {
    if (!(freq_ghz[c] > 0)) return fail(DEDISP_ERR_INVALID_ARG, "frequencies must be > 0");
    m3 += 1.0 / (freq_ghz[c] * freq_ghz[c] * freq_ghz[c]);
  }
  m3 /= nchan;
  const double diag = dt_s / (K * 2.0 * chan_bw_ghz) / m3;
  const double tau = tau_av_s / (K * 2.0 * chan_bw_ghz) / m3;
  const double a2 = diag * diag + (include_dm_tau ? tau * tau : 0.0);
  const double step = 2.0 * eps / nchan;
  int32_t n = 0;
  double running = 0.0, cur = dm0;
  while (cur <= dm_max && n < cap) {
    out[n++] = cur;
    running += std::sqrt(cur * cur + a2);
    cur = dm0 + step * running;
  }
  *n_out = n;
  return DEDISP_OK;
}

const char *dedisp_status_string(dedisp_status s) {
  switch (s) {
    case DEDISP_OK: return "ok";
    case DEDISP_ERR_INVALID_ARG: return "invalid argument";
    case DEDISP_ERR_SHAPE: return "input block too short";
    case DEDISP_ERR_OVERFLOW: return "int32 overflow possible";
    case DEDISP_ERR_OOM: return "out of memory";
    case DEDISP_ERR_DEVICE: return "device error";
    case DEDISP_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char *dedisp_last_error(void) { return dd::g_last_error.c_str(); }

}  // extern "C"
