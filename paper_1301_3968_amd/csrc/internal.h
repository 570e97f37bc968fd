// Internal declarations shared by the host plan code and the HIP launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dedisp.h"

namespace dd {

// Thread-local error text behind dedisp_last_error().
void set_error(const std::string &msg);
dedisp_status fail(dedisp_status s, const std::string &msg);
dedisp_status hip_fail(hipError_t e, const char *what);

// Test hook: when the environment variable DEDISP_TEST_FAIL_ALLOC holds k >= 1, the
// k-th allocation attempt counted from the moment the variable took that value fails
// (every host or device allocation the library makes goes through this check first).
bool alloc_fails();
// DEDISP_LOG set (and not "0"): one line per plan created and per change of a plan's
// search configuration, on stderr.
bool log_enabled();
void log_plan(const dedisp_plan_s *p);
// hipMalloc and hipMallocAsync behind the test hook.
hipError_t dev_malloc(void **p, size_t bytes);
hipError_t dev_malloc_async(void **p, size_t bytes, hipStream_t s);

#define DD_HIP(call)                                            \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return ::dd::hip_fail(e_, #call);     \
  } while (0)

constexpr int kMaxWidths = 64;

// Boxcar widths passed to kernels by value: sorted ascending, unique.
struct WidthList {
  int32_t n;
  int32_t w[kMaxWidths];
};

// Per-(DM tile, channel group) descriptors of the tiled search kernel and of the
// tiled fp32 dedispersion.
struct TiledTables;
struct F32Tables;
struct MfmaTables;

struct DevTables {
  int32_t *start = nullptr;   // [ndm][nchan]
  int32_t *ntap = nullptr;    // [ndm][nchan]
  float *weights = nullptr;   // [nchan] or [nchan][ktaps]
};

}  // namespace dd

struct dedisp_plan_s {
  int32_t nchan = 0, ndm = 0;
  double chan_bw = 0, dt = 0, kdm = 0;
  std::vector<double> freq, dm;
  dedisp_profile prof{};
  std::vector<int32_t> start, ntap;     // [ndm][nchan]
  std::vector<float> weights;           // copied weights
  int32_t ktaps = 1;
  int32_t wmode = DEDISP_W_UNIT;
  int32_t max_span = 0;                 // max(start + ntap)
  int32_t min_start = 0;
  int32_t max_ntap = 0;
  int64_t sum_max_ntap = 0;             // sum_c max_d ntap[d,c]
  int64_t window_rows = 0;              // sum_c (max_d ntap[d,c] - min_d ntap[d,c] + 1)
  int32_t tile_choice = -1;             // forced / tuned tile configuration (-2: general path)
  int32_t last_search_tile = -1;        // tile configuration of the last search (-1: general)
  int32_t logged_tile = INT32_MIN;      // search configuration last reported under DEDISP_LOG

  // Device copies, uploaded on first use (per plan, on the current device).
  std::mutex mu;
  bool uploaded = false;
  int device = -1;
  dd::DevTables dev;
  dd::TiledTables *tiled = nullptr;     // optimised-search tables (built lazily)
  dd::F32Tables *f32 = nullptr;         // tiled fp32 dedispersion tables (built lazily)
  dd::F32Tables *f32_adj = nullptr;     // tables of the transposed (adjoint) gather
  dd::MfmaTables *mfma = nullptr;       // matrix-core uint8 dedispersion tables

  // Instrumentation events around the dominant kernel (dedisp_set_kernel_events).
  std::vector<hipEvent_t> ev_start, ev_stop;
  size_t ev_next = 0;
};

namespace dd {
dedisp_status ensure_device(dedisp_plan p);

// Records the instrumentation events (if any) around one dominant-kernel launch.
struct KernelTimer {
  dedisp_plan_s *p;
  hipStream_t s;
  size_t slot = 0;
  bool on = false;
  KernelTimer(dedisp_plan_s *plan, hipStream_t stream) : p(plan), s(stream) {
    if (!p->ev_start.empty()) {
      on = true;
      slot = p->ev_next % p->ev_start.size();
      p->ev_next++;
    }
  }
  hipError_t begin() { return on ? hipEventRecord(p->ev_start[slot], s) : hipSuccess; }
  hipError_t end() { return on ? hipEventRecord(p->ev_stop[slot], s) : hipSuccess; }
};

// Per-call replacement of the plan's device weights (learned weights), scoped to
// the calling thread for the duration of one entry point.
extern thread_local const float *tl_weights;
struct WeightOverride {
  const float *prev;
  explicit WeightOverride(const float *w) : prev(tl_weights) { if (w) tl_weights = w; }
  ~WeightOverride() { tl_weights = prev; }
};
inline const float *weights_of(const dedisp_plan_s *p) {
  return tl_weights ? tl_weights : p->dev.weights;
}
void free_tiled(TiledTables *t);
void free_f32(F32Tables *t);
void free_mfma(MfmaTables *t);

// Launchers (kernels_*.hip).  All enqueue on `stream` and return hipError_t.
hipError_t launch_prefix_u8(const uint8_t *x, int64_t in_stride, int64_t in_bstride, int32_t nchan,
                            int32_t nbatch, int64_t nsamp, int32_t *P, hipStream_t s);
hipError_t launch_dedisp_prefix(const dedisp_plan_s *p, const int32_t *P, int64_t pstride,
                                int64_t pbstride, int32_t nbatch, int64_t nout, void *y,
                                int32_t out_dtype, int64_t out_stride, int64_t out_bstride,
                                hipStream_t s);
hipError_t launch_dedisp_direct_f32(const dedisp_plan_s *p, const float *x, int64_t in_stride,
                                    int64_t in_bstride, int32_t nbatch, int64_t nout, float *y,
                                    int64_t out_stride, int64_t out_bstride, hipStream_t s);
hipError_t launch_fir_f32(const dedisp_plan_s *p, const float *x, int64_t in_stride,
                          int64_t in_bstride, int32_t nbatch, int64_t nz, float *z,
                          hipStream_t s);
hipError_t launch_dedisp_1tap_f32(const dedisp_plan_s *p, const float *z, int64_t zstride,
                                  int64_t zbstride, int32_t nbatch, int64_t nout, float *y,
                                  int64_t out_stride, int64_t out_bstride, hipStream_t s);
// The converted block the matrix-core search's direct staging reads: xs[c][t] =
// x[c][t] ^ 0x80 for t < nsamp, 0x80 up to the row length xs_stride (a multiple of 16).
struct ConvertJob {
  const uint8_t *x;
  int64_t in_stride, nsamp;
  uint8_t *xs;
  int64_t xs_stride;
  int32_t nchan;
};
// Noise tables M, S [ndm][nw]; with cv, the same launch (extra workgroups) also writes
// the converted block.
hipError_t launch_norm(const dedisp_plan_s *p, const WidthList &wl, const double *mu,
                       const double *sigma, double *M, double *S, hipStream_t s,
                       const ConvertJob *cv = nullptr);
hipError_t launch_boxcar(const dedisp_plan_s *p, const void *y, int32_t y_dtype, int64_t nout,
                         int64_t y_stride, const WidthList &wl, const double *M, const double *S,
                         void *partials, int32_t nchunk, hipStream_t s);
hipError_t launch_reduce(int32_t ndm, int32_t nchunk, const void *partials, double *snr,
                         int32_t *t, int32_t *w, hipStream_t s);
hipError_t launch_merge_cand(int32_t ndm, const double *snr_b, const int32_t *t_b,
                             const int32_t *w_b, int64_t t_offset, double *snr, int64_t *t,
                             int32_t *w, hipStream_t s);
hipError_t launch_adjoint_z(const dedisp_plan_s *p, const float *g, int64_t nout, int64_t gstride,
                            int64_t gbstride, int32_t nbatch, int64_t nz, double *z,
                            hipStream_t s);
hipError_t launch_grad_w_tap(const dedisp_plan_s *p, const double *z, int64_t nz, const void *x,
                             int32_t in_dtype, int64_t in_stride, int64_t in_bstride,
                             int32_t nbatch, double *gw, hipStream_t s);
hipError_t launch_grad_x_tap(const dedisp_plan_s *p, const double *z, int64_t nz, int64_t nsamp,
                             int32_t nbatch, float *gx, int64_t in_stride, int64_t in_bstride,
                             hipStream_t s);
hipError_t launch_adjoint_direct(const dedisp_plan_s *p, const float *g, int64_t nout,
                                 int64_t gstride, int64_t gbstride, int32_t nbatch, const void *x,
                                 int32_t in_dtype, int64_t nsamp, int64_t in_stride,
                                 int64_t in_bstride, float *gx, double *gw, hipStream_t s);
hipError_t launch_sparse_grad_w(const dedisp_plan_s *p, int32_t nnz, const int32_t *b,
                                const int32_t *d, const int32_t *t, const float *val,
                                const void *x, int32_t in_dtype, int64_t in_stride,
                                int64_t in_bstride, int32_t nbatch, int64_t nout, double *gw,
                                hipStream_t s);
hipError_t launch_gather(const dedisp_plan_s *p, int32_t nnz, const int32_t *b, const int32_t *d,
                         const int32_t *t, const void *x, int32_t in_dtype, int64_t in_stride,
                         int64_t in_bstride, int32_t nbatch, int64_t nout, float *out,
                         hipStream_t s);

// Tiled fused search for uint8 input with unit weights (kernels_search.hip).
bool search_supported(const dedisp_plan_s *p, const WidthList &wl);
size_t search_work_bytes(const dedisp_plan_s *p, int32_t nw, int64_t nout);
dedisp_status run_search_tiled(dedisp_plan p, const uint8_t *x, int64_t nsamp, int64_t in_stride,
                               int64_t nout, const WidthList &wl, const double *mu,
                               const double *sigma, double *snr, int32_t *t, int32_t *w,
                               void *work, hipStream_t s);

// Tiled fp32 dedispersion for weighted profiles (kernels_f32.hip): uint8 or fp32
// input, fp32 output.  Returns DEDISP_ERR_UNSUPPORTED (launching nothing) when the
// plan does not fit the tiled kernel.
dedisp_status run_dedisperse_f32_tiled(dedisp_plan p, const void *in, int32_t in_dtype,
                                       int64_t nsamp, int64_t in_stride, int64_t in_bstride,
                                       int32_t nbatch, float *out, int64_t out_stride,
                                       int64_t out_bstride, int64_t nout, hipStream_t s,
                                       KernelTimer *kt);
// uint8 input, unit weights, int32 output on the int8 matrix cores (kernels_mfma.hip).
// Returns DEDISP_ERR_UNSUPPORTED (launching nothing) when the plan does not fit.
dedisp_status run_dedisperse_u8_mfma(dedisp_plan p, const uint8_t *x, int64_t nsamp,
                                     int64_t in_stride, int64_t in_bstride, int32_t nbatch,
                                     int32_t *out, int64_t out_stride, int64_t out_bstride,
                                     int64_t nout, hipStream_t s, KernelTimer *kt);
// Fused search on the matrix-core kernel, shape k of mfma_search_count() (noise
// tables, the tile kernel, the reduction over time tiles; kernels_mfma.hip).
// Returns DEDISP_ERR_UNSUPPORTED (launching nothing) when the plan does not fit.
int mfma_search_count();
// Host-only consistency check of a matrix-core shape's tables (kernels_mfma.hip).
dedisp_status mfma_check_tables(const dedisp_plan_s *p, int k, int64_t *pieces);
size_t mfma_search_work_bytes(const dedisp_plan_s *p, int32_t nw, int64_t nout);
dedisp_status run_search_mfma(dedisp_plan p, int k, const uint8_t *x, int64_t nsamp,
                              int64_t in_stride, int64_t nout, const WidthList &wl,
                              const double *mu, const double *sigma, double *snr, int32_t *t,
                              int32_t *w, void *work, hipStream_t s, bool dma = true);
// Fused search of a uint8 block with unit weights on the matrix cores, with the
// library's per-device scratch array as its workspace (kernels_mfma.hip): allocates
// nothing; fails when the plan's device tables are not built yet or the workspace
// would exceed the array.
dedisp_status run_search_noalloc(dedisp_plan p, const uint8_t *x, int64_t nsamp,
                                 int64_t in_stride, int64_t nout, const WidthList &wl,
                                 const double *mu, const double *sigma, double *snr, int32_t *t,
                                 int32_t *w, hipStream_t s);
// Multi-beam fused search on the matrix cores (kernels_mfma.hip): one shape for all
// beams (`prefer` if it takes them all, else the first that does); *out stays null
// when no shape takes every beam.
struct MfmaBatch;
dedisp_status mfma_batch_create(const std::vector<dedisp_plan> &plans,
                                const std::vector<int64_t> &nsamp, const WidthList &wl, int prefer,
                                MfmaBatch **out);
size_t mfma_batch_work_bytes(const MfmaBatch *B);
dedisp_status mfma_batch_enqueue(MfmaBatch *B, const void *const *in, const int64_t *stride,
                                 const double *mu, const double *sigma, double *snr, int32_t *t,
                                 int32_t *w, const std::vector<int64_t> &out_off, void *work,
                                 hipStream_t s, bool for_graph, KernelTimer *kt);
dedisp_status mfma_batch_upload(MfmaBatch *B);
void mfma_batch_free(MfmaBatch *B);
// zbar[b][c][tau] = sum_d g[b][d][tau - start[d][c]] for tau in [0, nz) on the same
// tiled kernel, every term added in fp64, fp64 output; DEDISP_ERR_UNSUPPORTED
// (launching nothing) when it does not fit.
dedisp_status run_adjoint_z_tiled(dedisp_plan p, const float *g, int64_t nout, int64_t gstride,
                                  int64_t gbstride, int32_t nbatch, int64_t nz, double *z,
                                  hipStream_t s);

// Pinned host staging for a small argument table that a call copies to the device
// on its stream.  copy() first waits for the previous copy out of the staging buffer
// to have executed (not for the rest of that call's work), so the host never
// overwrites bytes a queued copy has yet to read.
struct ArgStage {
  void *host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  hipError_t copy(void *d_dst, const void *src, size_t n, hipStream_t s);
  void release();
};

// Size of one per-chunk detection candidate record in the workspace.
constexpr size_t kCandBytes = 16;
constexpr int kBoxChunk = 256;  // starts per detection block

}  // namespace dd
