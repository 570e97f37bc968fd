// C-ABI entry points that run on the GPU: argument checks, workspace carving and
// the launch sequences.  Kernels live in kernels_basic.hip / kernels_search.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using dd::fail;

namespace dd {

static dedisp_status make_widths(const int32_t *widths, int32_t nw, int64_t nout, WidthList *wl) {
  if (!widths || nw <= 0 || nw > kMaxWidths)
    return fail(DEDISP_ERR_INVALID_ARG, "need 1..64 boxcar widths");
  std::vector<int32_t> v(widths, widths + nw);
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  if (v.front() < 1) return fail(DEDISP_ERR_INVALID_ARG, "boxcar widths must be >= 1");
  if (v.back() > nout) return fail(DEDISP_ERR_INVALID_ARG, "boxcar width longer than the output");
  wl->n = (int32_t)v.size();
  for (int i = 0; i < wl->n; ++i) wl->w[i] = v[i];
  return DEDISP_OK;
}

hipError_t ArgStage::copy(void *d_dst, const void *src, size_t n, hipStream_t s) {
  if (done) {
    hipError_t e = hipEventSynchronize(done);
    if (e != hipSuccess) return e;
  } else {
    hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  if (n > cap) {
    if (host) (void)hipHostFree(host);
    host = nullptr;
    cap = 0;
    hipError_t e = alloc_fails() ? hipErrorOutOfMemory : hipHostMalloc(&host, n, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    cap = n;
  }
  memcpy(host, src, n);
  hipError_t e = hipMemcpyAsync(d_dst, host, n, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipEventRecord(done, s);
}

void ArgStage::release() {
  if (done) {
    (void)hipEventSynchronize(done);
    (void)hipEventDestroy(done);
  }
  if (host) (void)hipHostFree(host);
  host = nullptr;
  done = nullptr;
  cap = 0;
}

static int32_t nchunks(int64_t nout) { return (int32_t)((nout + kBoxChunk - 1) / kBoxChunk); }

size_t detect_work_bytes(int32_t ndm, int32_t nw, int64_t nout) {
  const size_t tables = 2 * sizeof(double) * (size_t)ndm * nw;
  const size_t parts = kCandBytes * (size_t)ndm * nchunks(nout);
  return ((tables + 255) & ~(size_t)255) + parts;
}

// Runs norm + boxcar + reduce on a materialised y.
static dedisp_status run_detect(dedisp_plan p, const void *y, int32_t y_dtype, int64_t nout,
                                int64_t y_stride, const WidthList &wl, const double *mu,
                                const double *sigma, double *snr, int32_t *t, int32_t *w,
                                void *work, hipStream_t s) {
  double *M = (double *)work;
  double *S = M + (size_t)p->ndm * wl.n;
  const size_t tables = 2 * sizeof(double) * (size_t)p->ndm * wl.n;
  void *parts = (char *)work + ((tables + 255) & ~(size_t)255);
  const int32_t nc = nchunks(nout);
  DD_HIP(launch_norm(p, wl, mu, sigma, M, S, s));
  DD_HIP(launch_boxcar(p, y, y_dtype, nout, y_stride, wl, M, S, parts, nc, s));
  DD_HIP(launch_reduce(p->ndm, nc, parts, snr, t, w, s));
  return DEDISP_OK;
}

// Dedispersion dispatch shared by dedisp_dedisperse and the unfused search.
static dedisp_status run_dedisperse(dedisp_plan p, const void *in, int32_t in_dtype, int64_t nsamp,
                                    int64_t in_stride, int64_t in_bstride, int32_t nbatch,
                                    void *out, int32_t out_dtype, int64_t out_stride,
                                    int64_t out_bstride, int64_t nout, hipStream_t s,
                                    KernelTimer *kt = nullptr) {
  // fp32 output: the tiled kernel (weights folded into window rows) when the plan
  // fits it; the tile setting -2 keeps the general kernels below
  if (out_dtype == DEDISP_F32 && p->tile_choice != -2) {
    dedisp_status st = run_dedisperse_f32_tiled(p, in, in_dtype, nsamp, in_stride, in_bstride,
                                                nbatch, (float *)out, out_stride, out_bstride,
                                                nout, s, kt);
    if (st != DEDISP_ERR_UNSUPPORTED) return st;
  }
  if (in_dtype == DEDISP_U8 && (p->wmode == DEDISP_W_UNIT || p->wmode == DEDISP_W_CHANNEL)) {
    if (p->wmode == DEDISP_W_CHANNEL && out_dtype != DEDISP_F32)
      return fail(DEDISP_ERR_UNSUPPORTED, "channel weights produce F32 output");
    if (p->wmode == DEDISP_W_UNIT && out_dtype == DEDISP_I32 &&
        255.0 * (double)p->sum_max_ntap >= 2147483647.0)
      return fail(DEDISP_ERR_OVERFLOW, "int32 dedispersion sum could overflow");
    // int32 output: the matrix-core kernel when the plan fits it
    if (p->wmode == DEDISP_W_UNIT && out_dtype == DEDISP_I32 && p->tile_choice != -2) {
      dedisp_status st = run_dedisperse_u8_mfma(p, (const uint8_t *)in, nsamp, in_stride,
                                                in_bstride, nbatch, (int32_t *)out, out_stride,
                                                out_bstride, nout, s, kt);
      if (st != DEDISP_ERR_UNSUPPORTED) return st;
    }
    if (nsamp * 255.0 >= 2147483647.0)
      return fail(DEDISP_ERR_OVERFLOW, "block too long for the int32 prefix");
    const int64_t pstride = nsamp + 1;
    int32_t *P = nullptr;
    DD_HIP(dev_malloc_async((void **)&P, sizeof(int32_t) * (size_t)pstride * p->nchan * nbatch, s));
    hipError_t e = launch_prefix_u8((const uint8_t *)in, in_stride, in_bstride, p->nchan, nbatch,
                                    nsamp, P, s);
    if (e == hipSuccess && kt) e = kt->begin();
    if (e == hipSuccess)
      e = launch_dedisp_prefix(p, P, pstride, pstride * p->nchan, nbatch, nout, out, out_dtype,
                               out_stride, out_bstride, s);
    if (e == hipSuccess && kt) e = kt->end();
    hipError_t e2 = hipFreeAsync(P, s);
    if (e != hipSuccess) return hip_fail(e, "dedisperse launch");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    return DEDISP_OK;
  }
  if (in_dtype == DEDISP_F32 && out_dtype == DEDISP_F32) {
    if (p->wmode == DEDISP_W_TAP) {
      const int64_t nz = nsamp - p->ktaps + 1;
      float *z = nullptr;
      DD_HIP(dev_malloc_async((void **)&z, sizeof(float) * (size_t)nz * p->nchan * nbatch, s));
      hipError_t e = launch_fir_f32(p, (const float *)in, in_stride, in_bstride, nbatch, nz, z, s);
      if (e == hipSuccess)
        e = launch_dedisp_1tap_f32(p, z, nz, nz * p->nchan, nbatch, nout, (float *)out, out_stride,
                                   out_bstride, s);
      hipError_t e2 = hipFreeAsync(z, s);
      if (e != hipSuccess) return hip_fail(e, "dedisperse launch");
      if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
      return DEDISP_OK;
    }
    DD_HIP(launch_dedisp_direct_f32(p, (const float *)in, in_stride, in_bstride, nbatch, nout,
                                    (float *)out, out_stride, out_bstride, s));
    return DEDISP_OK;
  }
  return fail(DEDISP_ERR_UNSUPPORTED, "unsupported input / weight / output combination");
}

// Predicted int32 overflow of exact uint8 sums (checked before any device work): a
// trial's output is at most 255 sum_c max_d ntap[d,c], and the search adds up to
// `span` consecutive outputs in int32 (window sums from a running prefix over a lane's
// starts and the widths' halo).
static dedisp_status check_int32_sums(const dedisp_plan_s *p, int32_t in_dtype, int32_t out_dtype,
                                      int64_t span) {
  if (in_dtype != DEDISP_U8 || p->wmode != DEDISP_W_UNIT || out_dtype != DEDISP_I32)
    return DEDISP_OK;
  if (255.0 * (double)p->sum_max_ntap * (double)span >= 2147483647.0)
    return fail(DEDISP_ERR_OVERFLOW, span == 1 ? "int32 dedispersion sum could overflow"
                                               : "int32 boxcar window sum could overflow");
  return DEDISP_OK;
}

// Under DEDISP_LOG, a line whenever a plan's search runs in another configuration than
// the last one reported for it.
static void log_search(dedisp_plan p, int64_t nout, int32_t nw) {
  if (!log_enabled() || p->last_search_tile == p->logged_tile) return;
  p->logged_tile = p->last_search_tile;
  fprintf(stderr,
          "dedisp: search on plan %p: shape %d of the candidate list (-1: unfused path), "
          "%lld outputs, %d widths\n",
          (const void *)p, p->last_search_tile, (long long)nout, nw);
}

// Outputs the fused search adds in int32 at most: a lane's starts and the halo of
// the widths (at most 64).
constexpr int64_t kSearchSpan = 64;

static dedisp_status check_block(dedisp_plan p, const void *in, int32_t in_dtype, int64_t nsamp,
                                 int64_t in_stride, int64_t *nout) {
  if (!p) return fail(DEDISP_ERR_INVALID_ARG, "null plan");
  if (!in) return fail(DEDISP_ERR_INVALID_ARG, "null input");
  if (in_dtype != DEDISP_U8 && in_dtype != DEDISP_F32)
    return fail(DEDISP_ERR_INVALID_ARG, "input dtype must be U8 or F32");
  if (nsamp < 1 || in_stride < nsamp) return fail(DEDISP_ERR_INVALID_ARG, "bad nsamp / stride");
  if (nsamp < p->max_span) return fail(DEDISP_ERR_SHAPE, "block shorter than the longest sample run");
  *nout = nsamp - p->max_span + 1;
  if (*nout > INT32_MAX) return fail(DEDISP_ERR_UNSUPPORTED, "output longer than 2^31");
  return DEDISP_OK;
}

}  // namespace dd

extern "C" {

dedisp_status dedisp_dedisperse(dedisp_plan p, const void *d_in, int32_t in_dtype, int64_t nsamp,
                                int64_t in_stride, int64_t in_bstride, int32_t nbatch, void *d_out,
                                int32_t out_dtype, int64_t out_stride, int64_t out_bstride,
                                const float *d_weights, void *stream) {
  int64_t nout = 0;
  dedisp_status st = dd::check_block(p, d_in, in_dtype, nsamp, in_stride, &nout);
  if (st != DEDISP_OK) return st;
  if (!d_out) return fail(DEDISP_ERR_INVALID_ARG, "null output");
  if (nbatch < 1) return fail(DEDISP_ERR_INVALID_ARG, "nbatch must be >= 1");
  if (nbatch > 1 && in_bstride < in_stride * p->nchan) return fail(DEDISP_ERR_INVALID_ARG, "bad batch stride");
  if (out_stride < nout || (nbatch > 1 && out_bstride < out_stride * p->ndm))
    return fail(DEDISP_ERR_INVALID_ARG, "bad output stride");
  if (out_dtype != DEDISP_I32 && out_dtype != DEDISP_F32)
    return fail(DEDISP_ERR_INVALID_ARG, "output dtype must be I32 or F32");
  if ((st = dd::check_int32_sums(p, in_dtype, out_dtype, 1)) != DEDISP_OK) return st;
  if ((st = dd::ensure_device(p)) != DEDISP_OK) return st;
  dd::WeightOverride wo(d_weights);
  return dd::run_dedisperse(p, d_in, in_dtype, nsamp, in_stride, in_bstride, nbatch, d_out,
                            out_dtype, out_stride, out_bstride, nout, (hipStream_t)stream);
}

dedisp_status dedisp_work_bytes(dedisp_plan p, int64_t nsamp, int32_t nw, size_t *bytes) {
  if (!p || !bytes) return fail(DEDISP_ERR_INVALID_ARG, "null argument");
  if (nw <= 0 || nw > dd::kMaxWidths) return fail(DEDISP_ERR_INVALID_ARG, "need 1..64 widths");
  const int64_t nout = nsamp - p->max_span + 1;
  if (nout < 1) return fail(DEDISP_ERR_SHAPE, "block shorter than the longest sample run");
  size_t b = dd::detect_work_bytes(p->ndm, nw, nout);
  b = std::max(b, dd::search_work_bytes(p, nw, nout));
  *bytes = b;
  return DEDISP_OK;
}

dedisp_status dedisp_detect(dedisp_plan p, const void *d_y, int32_t y_dtype, int64_t nout,
                            int64_t y_stride, const int32_t *widths, int32_t nw,
                            const double *d_chan_mean, const double *d_chan_sigma, double *d_snr,
                            int32_t *d_t, int32_t *d_w, void *d_work, size_t work_bytes,
                            void *stream) {
  if (!p || !d_y || !d_chan_mean || !d_chan_sigma || !d_snr || !d_t || !d_w || !d_work)
    return fail(DEDISP_ERR_INVALID_ARG, "null argument");
  if (y_dtype != DEDISP_I32 && y_dtype != DEDISP_F32)
    return fail(DEDISP_ERR_INVALID_ARG, "y dtype must be I32 or F32");
  if (nout < 1 || y_stride < nout) return fail(DEDISP_ERR_INVALID_ARG, "bad nout / stride");
  dd::WidthList wl;
  dedisp_status st = dd::make_widths(widths, nw, nout, &wl);
  if (st != DEDISP_OK) return st;
  if (work_bytes < dd::detect_work_bytes(p->ndm, wl.n, nout))
    return fail(DEDISP_ERR_INVALID_ARG, "workspace too small");
  if ((st = dd::ensure_device(p)) != DEDISP_OK) return st;
  return dd::run_detect(p, d_y, y_dtype, nout, y_stride, wl, d_chan_mean, d_chan_sigma, d_snr, d_t,
                        d_w, d_work, (hipStream_t)stream);
}

dedisp_status dedisp_merge_candidates(int32_t ndm, const double *d_snr_b, const int32_t *d_t_b,
                                      const int32_t *d_w_b, int64_t t_offset, double *d_snr,
                                      int64_t *d_t, int32_t *d_w, void *stream) {
  if (ndm <= 0) return fail(DEDISP_ERR_INVALID_ARG, "ndm must be > 0");
  if (!d_snr_b || !d_t_b || !d_w_b || !d_snr || !d_t || !d_w)
    return fail(DEDISP_ERR_INVALID_ARG, "null argument");
  if (t_offset < 0 || t_offset > INT64_MAX - INT32_MAX)
    return fail(DEDISP_ERR_INVALID_ARG, "bad t_offset");
  DD_HIP(dd::launch_merge_cand(ndm, d_snr_b, d_t_b, d_w_b, t_offset, d_snr, d_t, d_w,
                               (hipStream_t)stream));
  return DEDISP_OK;
}

dedisp_status dedisp_check_search_tables(dedisp_plan p, int32_t shape, int64_t *pieces) {
  if (!p) return fail(DEDISP_ERR_INVALID_ARG, "null plan");
  if (pieces) *pieces = 0;
  return dd::mfma_check_tables(p, shape, pieces);
}

dedisp_status dedisp_search(dedisp_plan p, const void *d_in, int32_t in_dtype, int64_t nsamp,
                            int64_t in_stride, const int32_t *widths, int32_t nw,
                            const double *d_chan_mean, const double *d_chan_sigma, double *d_snr,
                            int32_t *d_t, int32_t *d_w, void *d_work, size_t work_bytes,
                            void *stream) {
  int64_t nout = 0;
  dedisp_status st = dd::check_block(p, d_in, in_dtype, nsamp, in_stride, &nout);
  if (st != DEDISP_OK) return st;
  if (!d_chan_mean || !d_chan_sigma || !d_snr || !d_t || !d_w || !d_work)
    return fail(DEDISP_ERR_INVALID_ARG, "null argument");
  dd::WidthList wl;
  if ((st = dd::make_widths(widths, nw, nout, &wl)) != DEDISP_OK) return st;
  size_t need = 0;
  if ((st = dedisp_work_bytes(p, nsamp, nw, &need)) != DEDISP_OK) return st;
  if (work_bytes < need) return fail(DEDISP_ERR_INVALID_ARG, "workspace too small");
  if ((st = dd::check_int32_sums(p, in_dtype, DEDISP_I32, dd::kSearchSpan)) != DEDISP_OK)
    return st;
  if ((st = dd::ensure_device(p)) != DEDISP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (in_dtype == DEDISP_U8 && p->tile_choice != -2 && dd::search_supported(p, wl)) {
    st = dd::run_search_tiled(p, (const uint8_t *)d_in, nsamp, in_stride, nout, wl, d_chan_mean,
                              d_chan_sigma, d_snr, d_t, d_w, d_work, s);
    if (st != DEDISP_ERR_UNSUPPORTED) {   // unsupported shapes fall through
      if (st == DEDISP_OK) dd::log_search(p, nout, wl.n);
      return st;
    }
  }
  p->last_search_tile = -1;
  dd::log_search(p, nout, wl.n);
  // General path: materialise y in a stream-ordered temporary, then detect.
  const int32_t ydt = (in_dtype == DEDISP_U8 && p->wmode == DEDISP_W_UNIT) ? DEDISP_I32 : DEDISP_F32;
  void *y = nullptr;
  DD_HIP(dd::dev_malloc_async((void **)&y, 4 * (size_t)nout * p->ndm, s));
  dd::KernelTimer kt(p, s);
  st = dd::run_dedisperse(p, d_in, in_dtype, nsamp, in_stride, 0, 1, y, ydt, nout, 0, nout, s, &kt);
  if (st == DEDISP_OK)
    st = dd::run_detect(p, y, ydt, nout, nout, wl, d_chan_mean, d_chan_sigma, d_snr, d_t, d_w,
                        d_work, s);
  hipError_t e2 = hipFreeAsync(y, s);
  if (st != DEDISP_OK) return st;
  if (e2 != hipSuccess) return dd::hip_fail(e2, "hipFreeAsync");
  return DEDISP_OK;
}

dedisp_status dedisp_search_noalloc(dedisp_plan p, const void *d_in, int32_t in_dtype,
                                    int64_t nsamp, int64_t in_stride, const int32_t *widths,
                                    int32_t nw, const double *d_chan_mean,
                                    const double *d_chan_sigma, double *d_snr, int32_t *d_t,
                                    int32_t *d_w, void *stream) {
  int64_t nout = 0;
  dedisp_status st = dd::check_block(p, d_in, in_dtype, nsamp, in_stride, &nout);
  if (st != DEDISP_OK) return st;
  if (in_dtype != DEDISP_U8) return fail(DEDISP_ERR_UNSUPPORTED, "the allocation-free search takes uint8 input");
  if (!d_chan_mean || !d_chan_sigma || !d_snr || !d_t || !d_w)
    return fail(DEDISP_ERR_INVALID_ARG, "null argument");
  dd::WidthList wl;
  if ((st = dd::make_widths(widths, nw, nout, &wl)) != DEDISP_OK) return st;
  if ((st = dd::check_int32_sums(p, in_dtype, DEDISP_I32, dd::kSearchSpan)) != DEDISP_OK)
    return st;
  return dd::run_search_noalloc(p, (const uint8_t *)d_in, nsamp, in_stride, nout, wl, d_chan_mean,
                                d_chan_sigma, d_snr, d_t, d_w, (hipStream_t)stream);
}

dedisp_status dedisp_dedisperse_backward(dedisp_plan p, const float *d_grad_y, int64_t nout,
                                         int64_t gy_stride, int64_t gy_bstride, int32_t nbatch,
                                         const void *d_in, int32_t in_dtype, int64_t nsamp,
                                         int64_t in_stride, int64_t in_bstride, float *d_grad_in,
                                         double *d_grad_w, const float *d_weights, void *stream) {
  int64_t nout_p = 0;
  dedisp_status st = dd::check_block(p, d_in, in_dtype, nsamp, in_stride, &nout_p);
  if (st != DEDISP_OK) return st;
  if (!d_grad_y) return fail(DEDISP_ERR_INVALID_ARG, "null gradient");
  if (nout != nout_p) return fail(DEDISP_ERR_SHAPE, "gradient length differs from the output length");
  if (nbatch < 1 || gy_stride < nout || (nbatch > 1 && gy_bstride < gy_stride * p->ndm))
    return fail(DEDISP_ERR_INVALID_ARG, "bad gradient strides");
  if (nbatch > 1 && in_bstride < in_stride * p->nchan) return fail(DEDISP_ERR_INVALID_ARG, "bad batch stride");
  if (d_grad_w && p->wmode == DEDISP_W_UNIT)
    return fail(DEDISP_ERR_INVALID_ARG, "unit weights have no weight gradient");
  if ((st = dd::ensure_device(p)) != DEDISP_OK) return st;
  dd::WeightOverride wo(d_weights);
  hipStream_t s = (hipStream_t)stream;
  if (p->wmode == DEDISP_W_TAP) {
    // zbar = transpose of the one-sample sum, in fp64 (the weight gradient formed from
    // it cancels heavily); then the FIR transposes.
    const int64_t nz = nsamp - p->ktaps + 1;
    double *z = nullptr;
    DD_HIP(dd::dev_malloc_async((void **)&z, sizeof(double) * (size_t)nz * p->nchan * nbatch, s));
    hipError_t e = hipSuccess;
    st = p->tile_choice == -2 ? DEDISP_ERR_UNSUPPORTED
                              : dd::run_adjoint_z_tiled(p, d_grad_y, nout, gy_stride, gy_bstride,
                                                        nbatch, nz, z, s);
    if (st == DEDISP_ERR_UNSUPPORTED)
      e = dd::launch_adjoint_z(p, d_grad_y, nout, gy_stride, gy_bstride, nbatch, nz, z, s);
    else if (st != DEDISP_OK) {
      (void)hipFreeAsync(z, s);
      return st;
    }
    if (e == hipSuccess && d_grad_w)
      e = dd::launch_grad_w_tap(p, z, nz, d_in, in_dtype, in_stride, in_bstride, nbatch, d_grad_w, s);
    if (e == hipSuccess && d_grad_in)
      e = dd::launch_grad_x_tap(p, z, nz, nsamp, nbatch, d_grad_in, in_stride, in_bstride, s);
    hipError_t e2 = hipFreeAsync(z, s);
    if (e != hipSuccess) return dd::hip_fail(e, "backward launch");
    if (e2 != hipSuccess) return dd::hip_fail(e2, "hipFreeAsync");
    return DEDISP_OK;
  }
  DD_HIP(dd::launch_adjoint_direct(p, d_grad_y, nout, gy_stride, gy_bstride, nbatch, d_in, in_dtype,
                                   nsamp, in_stride, in_bstride, d_grad_in, d_grad_w, s));
  return DEDISP_OK;
}

dedisp_status dedisp_backward_sparse(dedisp_plan p, int32_t nnz, const int32_t *d_b,
                                     const int32_t *d_d, const int32_t *d_t, const float *d_val,
                                     const void *d_in, int32_t in_dtype, int64_t nsamp,
                                     int64_t in_stride, int64_t in_bstride, int32_t nbatch,
                                     double *d_grad_w, void *stream) {
  int64_t nout = 0;
  dedisp_status st = dd::check_block(p, d_in, in_dtype, nsamp, in_stride, &nout);
  if (st != DEDISP_OK) return st;
  if (nnz < 0 || (nnz > 0 && (!d_b || !d_d || !d_t || !d_val)) || !d_grad_w)
    return fail(DEDISP_ERR_INVALID_ARG, "null argument");
  if (p->wmode == DEDISP_W_UNIT) return fail(DEDISP_ERR_INVALID_ARG, "unit weights have no weight gradient");
  if (nbatch < 1 || (nbatch > 1 && in_bstride < in_stride * p->nchan))
    return fail(DEDISP_ERR_INVALID_ARG, "bad batch size / stride");
  if ((st = dd::ensure_device(p)) != DEDISP_OK) return st;
  DD_HIP(dd::launch_sparse_grad_w(p, nnz, d_b, d_d, d_t, d_val, d_in, in_dtype, in_stride,
                                  in_bstride, nbatch, nout, d_grad_w, (hipStream_t)stream));
  return DEDISP_OK;
}

dedisp_status dedisp_last_search_tile(dedisp_plan p, int32_t *tile) {
  if (!p || !tile) return fail(DEDISP_ERR_INVALID_ARG, "null argument");
  *tile = p->last_search_tile;
  return DEDISP_OK;
}

dedisp_status dedisp_set_kernel_events(dedisp_plan p, void *const *ev_start, void *const *ev_stop,
                                       int32_t n) {
  if (!p || n < 0 || (n > 0 && (!ev_start || !ev_stop)))
    return fail(DEDISP_ERR_INVALID_ARG, "bad event arrays");
  p->ev_start.assign((hipEvent_t *)ev_start, (hipEvent_t *)ev_start + n);
  p->ev_stop.assign((hipEvent_t *)ev_stop, (hipEvent_t *)ev_stop + n);
  p->ev_next = 0;
  return DEDISP_OK;
}

dedisp_status dedisp_dedisperse_gather(dedisp_plan p, int32_t nnz, const int32_t *d_b,
                                       const int32_t *d_d, const int32_t *d_t, const void *d_in,
                                       int32_t in_dtype, int64_t nsamp, int64_t in_stride,
                                       int64_t in_bstride, int32_t nbatch, float *d_out,
                                       const float *d_weights, void *stream) {
  int64_t nout = 0;
  dedisp_status st = dd::check_block(p, d_in, in_dtype, nsamp, in_stride, &nout);
  if (st != DEDISP_OK) return st;
  if (nnz < 0 || (nnz > 0 && (!d_b || !d_d || !d_t || !d_out)))
    return fail(DEDISP_ERR_INVALID_ARG, "null argument");
  if (nbatch < 1 || (nbatch > 1 && in_bstride < in_stride * p->nchan))
    return fail(DEDISP_ERR_INVALID_ARG, "bad batch size / stride");
  if (nnz == 0) return DEDISP_OK;
  if ((st = dd::ensure_device(p)) != DEDISP_OK) return st;
  dd::WeightOverride wo(d_weights);
  DD_HIP(dd::launch_gather(p, nnz, d_b, d_d, d_t, d_in, in_dtype, in_stride, in_bstride, nbatch,
                           nout, d_out, (hipStream_t)stream));
  return DEDISP_OK;
}

}  // extern "C"
