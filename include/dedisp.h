/*
 * libdedisp -- programmable-profile incoherent dedispersion and boxcar detection
 * on AMD Instinct MI355X (gfx950).
 *
 * The method is the multi-sample incoherent dedisperser analysed in Clarke,
 * Macquart & Trott, "Performance of a novel fast transients detection system":
 * for every trial DM a set of dynamic-spectrum samples is summed (eq. p_dedisp,
 * Section 2.1), the sample set of each channel being a contiguous run of
 * `ntap` samples starting at the cold-plasma delay of the channel's top edge
 * (t_A, Section 3).  The dedispersed series is then searched with boxcar
 * windows of integer widths (the boxcar detector of Section 4), each window
 * normalised by its exact noise standard deviation (eqs. P_N_dedisp and snr).
 *
 * Conventions shared by every call:
 *   - Every call returns a dedisp_status; DEDISP_OK is 0.  No exception crosses
 *     the ABI.  dedisp_last_error() gives a thread-local description of the last
 *     failure.
 *   - "host" pointers are read during the call only; "device" pointers are HIP
 *     device memory owned by the caller, which must stay alive until `stream`
 *     has executed the enqueued work.  Calls enqueue asynchronously on the HIP
 *     stream `stream` (a hipStream_t, NULL = the default stream) and return.
 *   - Filterbank layout: channel-major, x[b][c][t] at byte offset
 *     ((b * bstride + c * stride) + t) * sizeof(elem), strides in elements.
 *   - Dedispersed layout: y[b][d][t], t in [0, nout), strides in elements.
 *   - A plan holds only immutable tables (host copies and lazily uploaded
 *     device copies); calls on different streams may share it provided each
 *     has its own workspace.
 *   - Environment: DEDISP_LOG (set, not "0") prints one line on stderr per plan
 *     created and whenever a plan's search runs in another shape than the last
 *     one printed; DEDISP_TEST_FAIL_ALLOC=k makes the k-th host or device
 *     allocation (counted from when the variable took that value) fail with
 *     DEDISP_ERR_OOM, for tests of the failure paths.
 */
#ifndef DEDISP_H
#define DEDISP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dedisp_plan_s *dedisp_plan;
typedef struct dedisp_batch_s *dedisp_batch;

typedef enum {
  DEDISP_OK = 0,
  DEDISP_ERR_INVALID_ARG = 1, /* null pointer, non-positive size, non-finite value, bad enum */
  DEDISP_ERR_SHAPE = 2,       /* input block shorter than the longest sample run */
  DEDISP_ERR_OVERFLOW = 3,    /* an int32 sum could exceed 2^31 - 1 */
  DEDISP_ERR_OOM = 4,         /* host or device allocation failed */
  DEDISP_ERR_DEVICE = 5,      /* a HIP call failed (message in dedisp_last_error) */
  DEDISP_ERR_UNSUPPORTED = 6  /* a valid request the library does not implement */
} dedisp_status;

typedef enum { DEDISP_U8 = 0, DEDISP_F32 = 1, DEDISP_I32 = 2 } dedisp_dtype;

/* How the sample run of each (trial, channel) is chosen.
 *   SMEAR      ntap = max(1, ceil(K DM (nu_lo^-2 - nu_top^-2) / dt)): the channel's
 *              dispersion smear in samples (Section 3, Delta tau_c between edges).
 *   ALLNONZERO every sample holding non-zero pulse power for a rectangular pulse
 *              of width tau'(nu) = width_s + scatter_s_1ghz * nu^scatter_index:
 *              ntap = max(1, ceil(t_B/dt) - floor(t_A/dt)) (eq. num_samples), with
 *              t_B taken at the channel's low edge.
 *   GREEDY     the Section 2.2 selection: predicted cell powers of the rectangular
 *              pulse model (App. A, eq. dispersed pulse) added in decreasing order
 *              while eq. sel_criterion holds; channels may get ntap = 0.
 *   EXPLICIT   caller-supplied start/ntap tables.
 *   FIXED      ntap = ktaps for every (trial, channel) (per-tap weighted profiles).
 * For every rule except EXPLICIT, start = floor(K DM (nu_top,c^-2 - nu_hi^-2) / dt). */
typedef enum {
  DEDISP_RULE_SMEAR = 0,
  DEDISP_RULE_ALLNONZERO = 1,
  DEDISP_RULE_GREEDY = 2,
  DEDISP_RULE_EXPLICIT = 3,
  DEDISP_RULE_FIXED = 4
} dedisp_rule;

/* Sample weights: UNIT (the paper's unweighted sums; exact int32 for uint8
 * input), CHANNEL (w[c]), TAP (w[c][k], k < ktaps; requires ntap == ktaps). */
typedef enum { DEDISP_W_UNIT = 0, DEDISP_W_CHANNEL = 1, DEDISP_W_TAP = 2 } dedisp_wmode;

typedef struct {
  int32_t rule;            /* dedisp_rule */
  double k_dm;             /* delay constant in s GHz^2 cm^3 / pc; 0 => 1/(2.41e-16 * 1e18) */
  double width_s;          /* ALLNONZERO / GREEDY: intrinsic pulse width tau */
  double scatter_s_1ghz;   /* ALLNONZERO / GREEDY: scatter width at 1 GHz */
  double scatter_index;    /* ALLNONZERO / GREEDY: scatter frequency index (e.g. -4) */
  double spectral_index;   /* GREEDY: alpha of P ~ (nu/nu0)^-alpha (eq. intrinsic_power) */
  double nu0_ghz;          /* GREEDY: reference frequency; 0 => 1 GHz */
  const int32_t *start;    /* EXPLICIT: host [ndm * nchan], copied at create */
  const int32_t *ntap;     /* EXPLICIT: host [ndm * nchan], copied at create, >= 0 */
  int32_t ktaps;           /* FIXED rule tap count; TAP weights per channel */
  int32_t wmode;           /* dedisp_wmode */
  const float *weights;    /* host [nchan] (CHANNEL) or [nchan * ktaps] (TAP), copied */
} dedisp_profile;

/* Fill `prof` with defaults: SMEAR rule, paper K, unit weights, scatter_index -4. */
dedisp_status dedisp_profile_init(dedisp_profile *prof);

/* Build a plan: the sample-set tables for `ndm` trial DMs over `nchan` channels.
 *   freq_ghz   host [nchan] channel centre frequencies (any order), GHz
 *   chan_bw_ghz channel width (> 0), GHz; dt_s sample time (> 0)
 *   dm         host [ndm] trial DMs (>= 0, finite), pc cm^-3
 * Host-only work; device tables are uploaded on first use.  Errors:
 * INVALID_ARG for bad sizes/values, OOM. */
dedisp_status dedisp_plan_create(dedisp_plan *out, int32_t nchan, const double *freq_ghz,
                                 double chan_bw_ghz, double dt_s, int32_t ndm, const double *dm,
                                 const dedisp_profile *prof);
dedisp_status dedisp_plan_destroy(dedisp_plan plan);

/* Copy the tables to host arrays start/ntap [ndm * nchan] (either may be NULL). */
dedisp_status dedisp_plan_tables(dedisp_plan plan, int32_t *start, int32_t *ntap);

/* Plan shape: number of channels, trials, the longest run max(start + ntap), the
 * tap count of TAP weights (1 otherwise) and the weight mode.  Any may be NULL. */
dedisp_status dedisp_plan_info(dedisp_plan plan, int32_t *nchan, int32_t *ndm, int32_t *max_span,
                               int32_t *ktaps, int32_t *wmode);

/* Valid output length for a block of nsamp samples: nout = nsamp - max(start + ntap) + 1
 * (eq. p_dedisp restricted to outputs whose samples all lie in the block).
 * SHAPE if nout < 1. */
dedisp_status dedisp_plan_out_len(dedisp_plan plan, int64_t nsamp, int64_t *nout);

/* eq. p_dedisp: y[b][d][t] = sum_c sum_{k < ntap[d,c]} w_{c,k} x[b][c][t + start[d,c] + k]
 * for 0 <= t < nout.  Supported (input, weights) -> output:
 *   U8 + UNIT    -> I32 (exact) or F32
 *   U8 + CHANNEL -> F32 (per-channel products summed in fp32 blocks, fp64 across blocks)
 *   F32 + TAP    -> F32 (FIR over the taps, then the one-sample sum)
 *   F32 + UNIT / CHANNEL -> F32
 * d_in device, d_out device [nbatch][ndm][nout].  Errors: SHAPE when
 * nsamp < max_span, OVERFLOW when an int32 sum could exceed 2^31 - 1,
 * UNSUPPORTED for other combinations, DEVICE on HIP failure.
 * d_weights (device, nullable): when non-NULL, replaces the plan's CHANNEL or TAP
 * weights for this call (same layout); used when the weights are being learned. */
dedisp_status dedisp_dedisperse(dedisp_plan plan, const void *d_in, int32_t in_dtype,
                                int64_t nsamp, int64_t in_stride, int64_t in_bstride,
                                int32_t nbatch, void *d_out, int32_t out_dtype, int64_t out_stride,
                                int64_t out_bstride, const float *d_weights, void *stream);

/* Streaming (Section 2.1's detector runs on data as they arrive): a block of a
 * stream searched by dedisp_search or dedisp_detect gives each trial's best window
 * of that block (starts relative to the block's first output).  This merges such a
 * result into a running best over the stream: for every trial d < ndm whose block
 * candidate holds a window (d_t_b[d] >= 0), the candidate (d_snr_b, d_t_b + t_offset,
 * d_w_b) replaces (d_snr, d_t, d_w) when d_t[d] < 0 or it ranks above it in the
 * search's order (larger S/N, then smaller W, then smaller start).  Block candidate
 * arrays are device f64 / i32 / i32 [ndm]; the running best device f64 / i64 / i32
 * [ndm], initialised by the caller to (-inf, -1, 0).  t_offset >= 0 is the stream
 * index of the block's first output.  A block that overlaps the previous one by
 * max_span - 1 + W_max - 1 samples searches every window of the stream at least once,
 * and the running best then equals the search of the whole stream.  Enqueued on
 * `stream`; DEDISP_ERR_INVALID_ARG for ndm <= 0, a null array or a negative t_offset. */
dedisp_status dedisp_merge_candidates(int32_t ndm, const double *d_snr_b, const int32_t *d_t_b,
                                      const int32_t *d_w_b, int64_t t_offset, double *d_snr,
                                      int64_t *d_t, int32_t *d_w, void *stream);

/* Workspace (device bytes) needed by dedisp_detect / dedisp_search for nsamp
 * samples and nw widths: the noise tables, per-(trial, time tile) candidates and,
 * for the search of uint8 blocks with unit weights, the largest of the tile kernels'
 * own buffers (the matrix-core search writes a converted copy of the block,
 * nchan x about nsamp bytes, into it on every call). */
dedisp_status dedisp_work_bytes(dedisp_plan plan, int64_t nsamp, int32_t nw, size_t *bytes);

/* Boxcar S/N search (eq. snr with the Section 4 boxcar) of a dedispersed block:
 * for every trial d, width W (host widths[nw], 1 <= W <= nout, nw <= 64) and
 * start t (0 <= t <= nout - W):
 *   B = sum_{j<W} y[d][t+j],  snr = (B - M[d,W]) / S[d,W],
 *   M = sum_c mu_c sum_tau a[tau],  S^2 = sum_c sigma_c^2 sum_tau a[tau]^2,
 * where a is the trial's channel weight run convolved with a length-W box, and
 * mu/sigma are device fp64 [nchan] per-channel noise mean / std.  Per trial the
 * best (snr, t, W) is written to device d_snr (f64), d_t, d_w (i32) [ndm];
 * exact ties go to the smaller W, then the smaller t.  y is I32 or F32. */
dedisp_status dedisp_detect(dedisp_plan plan, const void *d_y, int32_t y_dtype, int64_t nout,
                            int64_t y_stride, const int32_t *widths, int32_t nw,
                            const double *d_chan_mean, const double *d_chan_sigma, double *d_snr,
                            int32_t *d_t, int32_t *d_w, void *d_work, size_t work_bytes,
                            void *stream);

/* Fused dedisperse + detect for one uint8 (UNIT weights) or other supported
 * block without materialising y.  Same results as dedisp_dedisperse followed by
 * dedisp_detect. */
dedisp_status dedisp_search(dedisp_plan plan, const void *d_in, int32_t in_dtype, int64_t nsamp,
                            int64_t in_stride, const int32_t *widths, int32_t nw,
                            const double *d_chan_mean, const double *d_chan_sigma, double *d_snr,
                            int32_t *d_t, int32_t *d_w, void *d_work, size_t work_bytes,
                            void *stream);

/* Allocation-free fused search, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments and results as dedisp_search for uint8 input with unit weights and
 * widths up to 32, without the workspace: the search runs on the matrix cores with a
 * library-owned device array of DEDISP_NOALLOC_SCRATCH_BYTES per GPU as its
 * workspace (held until the process ends), and the call allocates nothing.
 * Requirements and errors:
 *   - the plan's device tables must already exist on the current device: run
 *     dedisp_search (or dedisp_autotune) with the plan once first; otherwise
 *     INVALID_ARG, with nothing launched;
 *   - the workspace the block needs (16 B per trial and width for the noise tables,
 *     16 B per trial and time tile of about 1000 outputs for the candidates) must fit
 *     the array, else INVALID_ARG; other inputs UNSUPPORTED.
 * Every call on one GPU uses that GPU's array: calls that overlap on one GPU (on
 * different streams, or from different threads) race; calls in stream order do not.
 * The shape is the plan's tuned or forced matrix-core shape, else the first one. */
#define DEDISP_NOALLOC_SCRATCH_BYTES (16u << 20)
dedisp_status dedisp_search_noalloc(dedisp_plan plan, const void *d_in, int32_t in_dtype,
                                    int64_t nsamp, int64_t in_stride, const int32_t *widths,
                                    int32_t nw, const double *d_chan_mean,
                                    const double *d_chan_sigma, double *d_snr, int32_t *d_t,
                                    int32_t *d_w, void *stream);

/* Adjoint of dedisp_dedisperse (the transpose of eq. p_dedisp), for gradients:
 *   grad_w[c][k] += sum_b sum_d sum_t g[b][d][t] x[b][c][t + start + k]   (fp64, device,
 *                   [nchan][K], K = ktaps for TAP weights, 1 otherwise)
 *   grad_in[b][c][i] = sum_d sum_k w_{c,k} g[b][d][i - start - k]           (fp32, device)
 * grad_w is overwritten (not accumulated); either output may be NULL.
 * g is device fp32 [nbatch][ndm][nout]; x is the forward input (U8 or F32);
 * d_weights as in dedisp_dedisperse. */
dedisp_status dedisp_dedisperse_backward(dedisp_plan plan, const float *d_grad_y, int64_t nout,
                                         int64_t gy_stride, int64_t gy_bstride, int32_t nbatch,
                                         const void *d_in, int32_t in_dtype, int64_t nsamp,
                                         int64_t in_stride, int64_t in_bstride, float *d_grad_in,
                                         double *d_grad_w, const float *d_weights, void *stream);

/* Weight gradient for a sparse output gradient with nnz entries (b, d, t, val)
 * (device arrays): grad_w[c][k] = sum_e val_e x[b_e][c][t_e + start[d_e,c] + k].
 * Used when the loss reads a few known outputs (a matched-filter S/N at known
 * pulse positions).  grad_w is overwritten.  Entries whose b, d or t fall
 * outside [0, nbatch) x [0, ndm) x [0, nout) contribute nothing. */
dedisp_status dedisp_backward_sparse(dedisp_plan plan, int32_t nnz, const int32_t *d_b,
                                     const int32_t *d_d, const int32_t *d_t, const float *d_val,
                                     const void *d_in, int32_t in_dtype, int64_t nsamp,
                                     int64_t in_stride, int64_t in_bstride, int32_t nbatch,
                                     double *d_grad_w, void *stream);

/* Gather selected outputs y[b_e][d_e][t_e] (e < nnz) of the dedispersion sum
 * without computing the rest (the forward of the sparse path), summed in fp64
 * and rounded to fp32 into d_out [nnz].  Out-of-range entries yield NaN. */
dedisp_status dedisp_dedisperse_gather(dedisp_plan plan, int32_t nnz, const int32_t *d_b,
                                       const int32_t *d_d, const int32_t *d_t, const void *d_in,
                                       int32_t in_dtype, int64_t nsamp, int64_t in_stride,
                                       int64_t in_bstride, int32_t nbatch, float *d_out,
                                       const float *d_weights, void *stream);

/* Trial DMs by eq. trial DMs (Section 5.3):
 *   DM_n = DM_0 + (2 eps / C) sum_{i<n} sqrt(DM_i^2 + DM_diag^2 + DM_tau^2),
 * DM_diag = dt / (2 K dnu) / mean(nu_c^-3), DM_tau the same with tau_av_s for dt,
 * nu_c the channel centres; DM_tau is used only when include_dm_tau != 0.
 * Trials are produced while DM_n <= dm_max and at most `cap` of them; host
 * out[cap] receives them and *n_out their number.  k_dm = 0 => paper K. */
dedisp_status dedisp_trial_dms(double dm0, double dm_max, double eps, int32_t nchan,
                               const double *freq_ghz, double chan_bw_ghz, double dt_s,
                               double tau_av_s, int32_t include_dm_tau, double k_dm, int32_t cap,
                               double *out, int32_t *n_out);

/* Batched search over many beams, each with its own plan (own DM grid) and
 * block length (Section 5.3 grids per beam), as one launch over every beam's tiles: on
 * the matrix cores a persistent launch whose workgroups claim (beam, tile) work items
 * from a device counter (the environment variable DEDISP_BATCH_LAUNCH=grid, read at
 * create, selects one workgroup per tile instead).  plans[nbeam] must share nchan and
 * use UNIT weights with uint8 input.  widths host [nw]. */
dedisp_status dedisp_batch_create(dedisp_batch *out, int32_t nbeam, const dedisp_plan *plans,
                                  const int64_t *nsamp, const int32_t *widths, int32_t nw);
dedisp_status dedisp_batch_destroy(dedisp_batch batch);
dedisp_status dedisp_batch_work_bytes(dedisp_batch batch, size_t *bytes);
/* d_in: host array [nbeam] of device pointers to each beam's uint8 block
 * (row stride in_stride[b]); d_chan_mean/sigma device fp64 [nchan] shared by all
 * beams; outputs device, concatenated over beams in beam order (sum of ndm_b).
 * If use_graph != 0 the launch sequence is captured once into a hipGraph and
 * replayed on later calls with the same pointers.  Calls on one batch share its
 * work-item counter and graph argument table: they must not overlap in time (issue
 * them on one stream, or order the streams). */
dedisp_status dedisp_batch_run(dedisp_batch batch, const void *const *d_in, const int64_t *in_stride,
                               const double *d_chan_mean, const double *d_chan_sigma,
                               double *d_snr, int32_t *d_t, int32_t *d_w, void *d_work,
                               size_t work_bytes, int32_t use_graph, void *stream);
/* Total trials across beams (length of the batch outputs). */
dedisp_status dedisp_batch_info(dedisp_batch batch, int64_t *total_trials, int64_t *total_sums);

/* Choose the search kernel's tile shape for this plan and block length by timing
 * the candidates on `stream` with caller-provided scratch input; the choice is
 * stored in the plan (and cached per shape in the file named by the environment
 * variable DEDISP_TUNE_CACHE, if set).  d_in must hold nsamp valid samples. */
dedisp_status dedisp_autotune(dedisp_plan plan, const void *d_in, int64_t nsamp, int64_t in_stride,
                              const int32_t *widths, int32_t nw, const double *d_chan_mean,
                              const double *d_chan_sigma, void *d_work, size_t work_bytes,
                              void *stream, int32_t *chosen);
/* Test support, host only (no device work): builds the host tables of matrix-core shape
 * `shape` (0 .. 4, the search's candidates 8 .. 12) for the plan and checks them: the
 * register staging's units and the direct staging's copy blocks fill the same LDS
 * pieces with the same window bytes, every K block's segments are read inside their
 * channel's staged region, window origins are multiples of 8 and the converted rows
 * reach every copy block.  *pieces (optional): LDS pieces compared.  Returns OK,
 * UNSUPPORTED when the plan does not fit the shape or a check fails (message in
 * dedisp_last_error), INVALID_ARG for a null plan or a shape out of range. */
dedisp_status dedisp_check_search_tables(dedisp_plan plan, int32_t shape, int64_t *pieces);

/* Force a shape of the fused uint8 search (index into its candidate list: the
 * shapes of the packed-add kernel, then those of the int8 matrix-core kernel; the
 * autotuner times them all), -1 for the default (the matrix-core shape of two
 * workgroups per CU, else the first matrix-core shape, else packed-add shape 0,
 * the first that takes the plan), or -2 to always use the
 * general kernels: the unfused search (dedisperse into a temporary, then detect),
 * the prefix-difference uint8 dedispersion, the untiled fp32 dedispersion and the
 * untiled per-tap adjoint. */
dedisp_status dedisp_set_tile(dedisp_plan plan, int32_t tile);
/* Tile configuration used by the last dedisp_search on this plan (-1: unfused path). */
dedisp_status dedisp_last_search_tile(dedisp_plan plan, int32_t *tile);

/* Instrumentation.  When set, every dedisp_search call on this plan records
 * ev_start[i] on its stream immediately before its dominant kernel (the
 * dedispersion sum, or the fused search kernel) and ev_stop[i] immediately
 * after it, with i cycling over [0, n).  The events are caller-created
 * hipEvent_t handles that must outlive their use; n = 0 disables.  This is the
 * one piece of mutable plan state: do not change it while calls are in flight. */
dedisp_status dedisp_set_kernel_events(dedisp_plan plan, void *const *ev_start,
                                       void *const *ev_stop, int32_t n);

const char *dedisp_status_string(dedisp_status s);
const char *dedisp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DEDISP_H */
