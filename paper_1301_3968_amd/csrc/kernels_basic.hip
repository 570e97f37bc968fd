// General-purpose kernels of libdedisp for gfx950: prefix pre-pass, the
// dedispersion sum for every weight mode, the boxcar detector, its reduction and
// the adjoint (gradient) kernels.  The tiled search kernel for uint8 data with
// unit weights lives in kernels_search.hip.
//
// Sums follow eq. p_dedisp (Section 2.1): for trial d, channel c contributes the
// run of ntap[d,c] samples starting at start[d,c] + t.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "internal.h"
#include "norm_reduce.h"

namespace dd {
namespace {

constexpr int kThreads = 256;

// ----------------------------------------------------------------------------------
// Per-channel inclusive prefix of uint8 samples: P[c][0] = 0, P[c][i+1] = P[c][i] + x[c][i].
// One block per (channel, batch); each thread scans a contiguous chunk.
// Values are exact in int32 for blocks shorter than 2^31 / 255 samples.
// ----------------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
k_prefix_u8(const uint8_t *__restrict__ x, int64_t in_stride, int64_t in_bstride, int64_t nsamp,
            int32_t *__restrict__ P, int64_t pstride, int64_t pbstride) {
  const int c = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const uint8_t *row = x + (int64_t)b * in_bstride + (int64_t)c * in_stride;
  int32_t *out = P + (int64_t)b * pbstride + (int64_t)c * pstride;
  const int64_t chunk = (nsamp + kThreads - 1) / kThreads;
  const int64_t i0 = min((int64_t)tid * chunk, nsamp), i1 = min(i0 + chunk, nsamp);
  int32_t s = 0;
  for (int64_t i = i0; i < i1; ++i) s += row[i];
  __shared__ int32_t part[kThreads];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    int32_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = tid == 0 ? 0 : part[tid - 1];
  if (tid == 0) out[0] = 0;
  for (int64_t i = i0; i < i1; ++i) {
    run += row[i];
    out[i + 1] = run;
  }
}

// y[d][t] = sum_c (P[c][t+s+n] - P[c][t+s]) (int32, exact), or with channel
// weights sum_c w_c * (window sum), accumulated in fp32 over blocks of 32
// channels and in fp64 across blocks.
template <bool kWeighted, typename OutT>
__global__ void __launch_bounds__(kThreads)
k_dedisp_prefix(const int32_t *__restrict__ P, int64_t pstride, int64_t pbstride,
                const int32_t *__restrict__ start, const int32_t *__restrict__ ntap,
                const float *__restrict__ w, int32_t nchan, int64_t nout, OutT *__restrict__ y,
                int64_t out_stride, int64_t out_bstride) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int d = blockIdx.y, b = blockIdx.z;
  if (t >= nout) return;
  const int32_t *Pb = P + (int64_t)b * pbstride;
  const int32_t *sd = start + (int64_t)d * nchan;
  const int32_t *nd = ntap + (int64_t)d * nchan;
  if constexpr (!kWeighted) {
    int32_t acc = 0;
    for (int c = 0; c < nchan; ++c) {
      const int32_t *row = Pb + (int64_t)c * pstride + t + sd[c];
      acc += row[nd[c]] - row[0];
    }
    y[(int64_t)b * out_bstride + (int64_t)d * out_stride + t] = (OutT)acc;
  } else {
    double tot = 0.0;
    for (int c0 = 0; c0 < nchan; c0 += 32) {
      float part = 0.0f;
      const int c1 = min(nchan, c0 + 32);
      for (int c = c0; c < c1; ++c) {
        const int32_t *row = Pb + (int64_t)c * pstride + t + sd[c];
        part = __fmaf_rn(w[c], (float)(row[nd[c]] - row[0]), part);
      }
      tot += (double)part;
    }
    y[(int64_t)b * out_bstride + (int64_t)d * out_stride + t] = (OutT)tot;
  }
}

// fp32 input, unit or channel weights: direct tap sums, fp32 within a block of
// 32 channels, fp64 across blocks.
template <bool kWeighted>
__global__ void __launch_bounds__(kThreads)
k_dedisp_direct_f32(const float *__restrict__ x, int64_t in_stride, int64_t in_bstride,
                    const int32_t *__restrict__ start, const int32_t *__restrict__ ntap,
                    const float *__restrict__ w, int32_t nchan, int64_t nout, float *__restrict__ y,
                    int64_t out_stride, int64_t out_bstride) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int d = blockIdx.y, b = blockIdx.z;
  if (t >= nout) return;
  const float *xb = x + (int64_t)b * in_bstride;
  const int32_t *sd = start + (int64_t)d * nchan;
  const int32_t *nd = ntap + (int64_t)d * nchan;
  double tot = 0.0;
  for (int c0 = 0; c0 < nchan; c0 += 32) {
    float part = 0.0f;
    const int c1 = min(nchan, c0 + 32);
    for (int c = c0; c < c1; ++c) {
      const float *row = xb + (int64_t)c * in_stride + t + sd[c];
      float s = 0.0f;
      for (int k = 0; k < nd[c]; ++k) s += row[k];
      part = kWeighted ? __fmaf_rn(w[c], s, part) : part + s;
    }
    tot += (double)part;
  }
  y[(int64_t)b * out_bstride + (int64_t)d * out_stride + t] = (float)tot;
}

// FIR over the taps: z[b][c][i] = sum_{k<K} w[c][k] x[b][c][i+k], 0 <= i < nz.
__global__ void __launch_bounds__(kThreads)
k_fir_f32(const float *__restrict__ x, int64_t in_stride, int64_t in_bstride,
          const float *__restrict__ w, int32_t K, int64_t nz, float *__restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y, b = blockIdx.z;
  if (i >= nz) return;
  const float *row = x + (int64_t)b * in_bstride + (int64_t)c * in_stride + i;
  const float *wc = w + (int64_t)c * K;
  float acc = 0.0f;
  for (int k = 0; k < K; ++k) acc = __fmaf_rn(wc[k], row[k], acc);
  z[((int64_t)b * gridDim.y + c) * nz + i] = acc;
}

// One-sample sum over FIR outputs: y[b][d][t] = sum_c z[b][c][t + s[d,c]].
__global__ void __launch_bounds__(kThreads)
k_dedisp_1tap_f32(const float *__restrict__ z, int64_t zstride, int64_t zbstride,
                  const int32_t *__restrict__ start, int32_t nchan, int64_t nout,
                  float *__restrict__ y, int64_t out_stride, int64_t out_bstride) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int d = blockIdx.y, b = blockIdx.z;
  if (t >= nout) return;
  const float *zb = z + (int64_t)b * zbstride + t;
  const int32_t *sd = start + (int64_t)d * nchan;
  double tot = 0.0;
  for (int c0 = 0; c0 < nchan; c0 += 32) {
    float part = 0.0f;
    const int c1 = min(nchan, c0 + 32);
    for (int c = c0; c < c1; ++c) part += zb[(int64_t)c * zstride + sd[c]];
    tot += (double)part;
  }
  y[(int64_t)b * out_bstride + (int64_t)d * out_stride + t] = (float)tot;
}

// ----------------------------------------------------------------------------------
// Boxcar noise statistics: M[d][j], S[d][j] for width W_j (eqs. P_N_dedisp and snr
// extended to W consecutive outputs).  a = (channel weight run) * box_W.
// ----------------------------------------------------------------------------------
__device__ __forceinline__ void norm_terms(int wmode, int K, const float *__restrict__ w, int c, int n,
                                           int W, double &s1, double &s2) {
  if (wmode == DEDISP_W_TAP) {
    // explicit convolution of the tap weights with a length-W box
    s1 = 0.0;
    s2 = 0.0;
    for (int tau = 0; tau < n + W - 1; ++tau) {
      double a = 0.0;
      const int k0 = max(0, tau - W + 1), k1 = min(n - 1, tau);
      for (int k = k0; k <= k1; ++k) a += (double)w[(int64_t)c * K + k];
      s1 += a;
      s2 += a * a;
    }
  } else {
    // n-box convolved with W-box: a trapezoid 1, 2, .., m, .., m, .., 2, 1
    const int lo = min(n, W), hi = max(n, W);
    const double ld = lo;
    s1 = (double)n * (double)W;
    s2 = 2.0 * ((ld - 1.0) * ld * (2.0 * ld - 1.0) / 6.0) + (double)(hi - lo + 1) * ld * ld;
    if (wmode == DEDISP_W_CHANNEL) {
      const double wc = (double)w[c];
      s1 *= wc;
      s2 *= wc * wc;
    }
  }
}

// Noise statistics of every (trial, width), for tap weights or widths above 63 (the
// bucketed kernel below takes the rest).  One workgroup per kNormTrials trials;
// per trial, 32 width lanes (each taking widths j and j + 32) times kNormSplit
// channel residues.  The trials' tap counts and the channel statistics are staged
// in LDS a chunk of channels at a time; the kNormSplit partial sums of a (trial,
// width) are added in a fixed order, so results do not vary between runs.
constexpr int kNormTrials = 1, kNormSplit = 16, kNormChunk = 512;
constexpr int kNormThreads = kNormTrials * 32 * kNormSplit;

// Sum and sum of squares of the n-box convolved with the W-box: a trapezoid
// 1, 2, .., L, .., L, .., 2, 1 with L = min(n, W) (exact integers).
__device__ __forceinline__ void trapezoid(int n, int W, double &s1, double &s2) {
  const int L = min(n, W), H = max(n, W);
  s1 = (double)n * (double)W;
  if (L < 1024) {
    s2 = (double)((L - 1) * L * (2 * L - 1) / 3) + (double)(H - L + 1) * (double)L * (double)L;
  } else {
    const double ld = L;
    s2 = (ld - 1.0) * ld * (2.0 * ld - 1.0) / 3.0 + (double)(H - L + 1) * ld * ld;
  }
}

__global__ void __launch_bounds__(kNormThreads)
k_norm(const int32_t *__restrict__ ntap, int32_t nchan, int32_t ndm, int32_t wmode, int32_t K,
       const float *__restrict__ w, const double *__restrict__ mu,
       const double *__restrict__ sigma, WidthList wl, double *__restrict__ M,
       double *__restrict__ S) {
  __shared__ int32_t sn[kNormTrials][kNormChunk];
  __shared__ double smu[kNormChunk], svar[kNormChunk];
  __shared__ double part[kNormTrials][2][64][kNormSplit];
  const int tid = threadIdx.x, d0 = blockIdx.x * kNormTrials;
  const int tj = tid / (32 * kNormSplit), rest = tid % (32 * kNormSplit);
  const int split = rest / 32, jlane = rest % 32;
  const int d = d0 + tj;
  int Wh[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) Wh[h] = (jlane + 32 * h < wl.n) ? wl.w[jlane + 32 * h] : 0;
  double m[2] = {0.0, 0.0}, v[2] = {0.0, 0.0};
  for (int c0 = 0; c0 < nchan; c0 += kNormChunk) {
    const int cn = min(kNormChunk, nchan - c0);
    __syncthreads();
    for (int i = tid; i < kNormTrials * kNormChunk; i += kNormThreads) {
      const int t = i / kNormChunk, c = i - t * kNormChunk;
      sn[t][c] = (c < cn && d0 + t < ndm) ? ntap[(int64_t)(d0 + t) * nchan + c0 + c] : 0;
    }
    for (int c = tid; c < cn; c += kNormThreads) {
      smu[c] = mu[c0 + c];
      svar[c] = sigma[c0 + c] * sigma[c0 + c];
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int W = Wh[h];
      if (W == 0) continue;
      double mm = m[h], vv = v[h];
      for (int c = split; c < cn; c += kNormSplit) {
        const int n = sn[tj][c];
        if (n == 0) continue;
        double s1, s2;
        if (wmode == DEDISP_W_TAP) {
          norm_terms(wmode, K, w, c0 + c, n, W, s1, s2);
        } else {
          trapezoid(n, W, s1, s2);
          if (wmode == DEDISP_W_CHANNEL) {
            const double wc = (double)w[c0 + c];
            s1 *= wc;
            s2 *= wc * wc;
          }
        }
        mm += smu[c] * s1;
        vv += svar[c] * s2;
      }
      m[h] = mm;
      v[h] = vv;
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    part[tj][0][jlane + 32 * h][split] = m[h];
    part[tj][1][jlane + 32 * h][split] = v[h];
  }
  __syncthreads();
  if (split != 0 || d >= ndm) return;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = jlane + 32 * h;
    if (j >= wl.n) continue;
    double mm = 0.0, vv = 0.0;
#pragma unroll
    for (int q = 0; q < kNormSplit; ++q) {
      mm += part[tj][0][j][q];
      vv += part[tj][1][j][q];
    }
    M[(int64_t)d * wl.n + j] = mm;
    S[(int64_t)d * wl.n + j] = sqrt(vv);
  }
}

// Workgroup j of the conversion (256 threads, 16 bytes each): row j / per_row, bytes
// 4096 (j mod per_row) .. of the converted block.
constexpr int kConvThreads = 256;
__device__ __forceinline__ void convert_block(const ConvertJob &cv, int64_t j, int64_t per_row) {
  const int64_t c = j / per_row;
  const int64_t p = 16 * ((j - c * per_row) * kConvThreads + threadIdx.x);
  if (p >= cv.xs_stride) return;
  const uint8_t *row = cv.x + c * cv.in_stride;
  uint32_t v[4];
  if (p + 16 <= cv.nsamp && ((uintptr_t)(row + p) & 3) == 0) {
    const __attribute__((address_space(1))) uint32_t *r =
        (const __attribute__((address_space(1))) uint32_t *)(row + p);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = r[k] ^ 0x80808080u;
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t u = 0;
      for (int i = 0; i < 4; ++i) {
        const int64_t q = p + 4 * k + i;
        u |= (uint32_t)((q < cv.nsamp ? row[q] : 0) ^ 0x80) << (8 * i);
      }
      v[k] = u;
    }
  }
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  *(v4u *)(cv.xs + c * cv.xs_stride + p) = (v4u){v[0], v[1], v[2], v[3]};
}

__global__ void __launch_bounds__(kConvThreads) k_convert_u8(ConvertJob cv, int64_t per_row) {
  convert_block(cv, blockIdx.x, per_row);
}

// Workgroups 0 .. ndm - 1: the noise tables of trial blockIdx.x; workgroups from ndm on
// (when cv.xs is set): the conversion, workgroup ndm + j taking conversion block j.
__global__ void __launch_bounds__(64 * kBucketWaves)
k_norm_buckets(const int32_t *__restrict__ ntap, int32_t nchan, int32_t wmode,
               const float *__restrict__ w, const double *__restrict__ mu,
               const double *__restrict__ sigma, WidthList wl, double *__restrict__ M,
               double *__restrict__ S, int32_t ndm, ConvertJob conv, int64_t per_row) {
  static_assert(64 * kBucketWaves == kConvThreads, "one workgroup shape for both roles");
  if ((int)blockIdx.x >= ndm) {   // the whole workgroup, before any barrier
    convert_block(conv, (int64_t)blockIdx.x - ndm, per_row);
    return;
  }
  const int d = blockIdx.x;
  norm_buckets_trial(ntap + (int64_t)d * nchan, nchan, wmode, w, mu, sigma, wl,
                     M + (int64_t)d * wl.n, S + (int64_t)d * wl.n);
}

struct Cand {
  double snr;
  int32_t t;
  int32_t w;
};

// Boxcar search of one chunk of kBoxChunk starts of one trial.  Thread t grows
// the window sum B one output at a time (the same summation order as a direct
// sum), evaluating snr = (B - M)/S at every listed width.
template <typename YT>
__global__ void __launch_bounds__(kBoxChunk)
k_boxcar(const YT *__restrict__ y, int64_t nout, int64_t y_stride, WidthList wl,
         const double *__restrict__ M, const double *__restrict__ S, Cand *__restrict__ part,
         int32_t nchunk) {
  const int d = blockIdx.y, chunk = blockIdx.x, tid = threadIdx.x;
  const int64_t t = (int64_t)chunk * kBoxChunk + tid;
  const YT *yd = y + (int64_t)d * y_stride;
  double best = -INFINITY;
  int bw = 0, bt = -1;
  if (t < nout) {
    double acc = 0.0;
    int j = 0;
    const int wmax = wl.w[wl.n - 1];
    for (int q = 0; q < wmax && t + q < nout; ++q) {
      acc += (double)yd[t + q];
      if (q + 1 == wl.w[j]) {
        const double r = (acc - M[d * wl.n + j]) / S[d * wl.n + j];
        if (better(r, wl.w[j], (int)t, best, bw, bt)) {
          best = r;
          bw = wl.w[j];
          bt = (int)t;
        }
        ++j;
      }
    }
  }
  __shared__ double s_snr[kBoxChunk];
  __shared__ int s_w[kBoxChunk], s_t[kBoxChunk];
  s_snr[tid] = best;
  s_w[tid] = bw;
  s_t[tid] = bt;
  __syncthreads();
  for (int off = kBoxChunk / 2; off > 0; off >>= 1) {
    if (tid < off) {
      const int o = tid + off;
      if (s_t[o] >= 0 && (s_t[tid] < 0 || better(s_snr[o], s_w[o], s_t[o], s_snr[tid], s_w[tid], s_t[tid]))) {
        s_snr[tid] = s_snr[o];
        s_w[tid] = s_w[o];
        s_t[tid] = s_t[o];
      }
    }
    __syncthreads();
  }
  if (tid == 0) part[(int64_t)d * nchunk + chunk] = Cand{s_snr[0], s_t[0], s_w[0]};
}

// Per trial, the best of its chunk candidates.
static_assert(kThreads == kReduceThreads, "k_reduce runs best_of_row with kThreads threads");
__global__ void __launch_bounds__(kThreads)
k_reduce(int32_t ndm, int32_t nchunk, const Cand *__restrict__ part, double *__restrict__ snr,
         int32_t *__restrict__ tout, int32_t *__restrict__ wout) {
  const int d = blockIdx.x;
  best_of_row(part + (int64_t)d * nchunk, nchunk, snr + d, tout + d, wout + d);
}

// Per trial, the block's best candidate (start t_b + t_offset in the stream) replaces
// the running best when it ranks above it (the ranking of the search: larger S/N, then
// smaller width, then earlier start; a candidate with t < 0 holds no window).
__global__ void __launch_bounds__(kThreads)
k_merge_cand(int32_t ndm, const double *__restrict__ snr_b, const int32_t *__restrict__ t_b,
             const int32_t *__restrict__ w_b, int64_t t_offset, double *__restrict__ snr,
             int64_t *__restrict__ t, int32_t *__restrict__ w) {
  const int d = blockIdx.x * kThreads + threadIdx.x;
  if (d >= ndm || t_b[d] < 0) return;
  const int64_t tb = t_b[d] + t_offset;
  const double sb = snr_b[d];
  const int wb = w_b[d];
  bool take = t[d] < 0;
  if (!take) {
    if (sb != snr[d]) take = sb > snr[d];
    else if (wb != w[d]) take = wb < w[d];
    else take = tb < t[d];
  }
  if (take) {
    snr[d] = sb;
    t[d] = tb;
    w[d] = wb;
  }
}

// ----------------------------------------------------------------------------------
// Adjoint kernels (transposes of the dedispersion sum), all in gather form so that
// every output is written by exactly one thread in a fixed summation order.
// ----------------------------------------------------------------------------------

// zbar[b][c][i] = sum_d g[b][d][i - s[d,c]] over trials whose output index lies in
// [0, nout), added and stored in fp64.
__global__ void __launch_bounds__(kThreads)
k_adjoint_z(const float *__restrict__ g, int64_t nout, int64_t gstride, int64_t gbstride,
            const int32_t *__restrict__ start, int32_t nchan, int32_t ndm, int64_t nz,
            double *__restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y, b = blockIdx.z;
  if (i >= nz) return;
  const float *gb = g + (int64_t)b * gbstride;
  double acc = 0.0;
  for (int d = 0; d < ndm; ++d) {
    const int64_t t = i - start[(int64_t)d * nchan + c];
    if (t >= 0 && t < nout) acc += (double)gb[(int64_t)d * gstride + t];
  }
  z[((int64_t)b * nchan + c) * nz + i] = acc;
}

// gw[c][k] = sum_b sum_i zbar[b][c][i] x[b][c][i+k] (zbar fp64) with fp64 products and sums, in
// two passes.  Pass 1: one workgroup per (chunk of kGwChunk samples, slice of at most
// KB taps, channel, batch element).  Piece by piece (kGwPiece samples) the workgroup
// copies zbar and the x it meets into LDS with coalesced loads; a thread then takes
// kGwRun consecutive samples and the x window they meet into registers and keeps one
// fp64 accumulator per tap of the slice.  The workgroup reduces them and writes its
// partial sums.  Pass 2 adds the partials of each (c, k) in a fixed order, so the
// result does not depend on the schedule.
constexpr int kGwRun = 8, kGwPiece = kThreads * kGwRun, kGwIter = 4;
constexpr int kGwChunk = kGwPiece * kGwIter, kGwMaxK = 64;

template <typename XT, int KB>
__global__ void __launch_bounds__(kThreads)
k_grad_w_tap_part(const double *__restrict__ z, int64_t nz, const XT *__restrict__ x,
                  int64_t in_stride, int64_t in_bstride, int32_t nchan, int32_t K,
                  int32_t nslice, double *__restrict__ part) {
  constexpr int XW = (kGwRun + KB - 1 + 3) / 4 * 4;   // x window of a run, whole float4s
  static_assert(KB <= 16 && kGwRun % 4 == 0, "window within the 16-sample pad");
  __shared__ __attribute__((aligned(16))) double zs[kGwPiece];
  __shared__ __attribute__((aligned(16))) float xs[kGwPiece + 16];
  __shared__ double red[KB][kThreads / 64];
  const int sidx = blockIdx.x / nslice, k0 = (blockIdx.x - sidx * nslice) * KB;
  const int c = blockIdx.y, b = blockIdx.z, tid = threadIdx.x;
  const int kl = min(KB, K - k0);   // taps k0 .. k0 + kl - 1
  const int nsplit = gridDim.x / nslice;
  const XT *xr = x + (int64_t)b * in_bstride + (int64_t)c * in_stride + k0;
  const double *zr = z + ((int64_t)b * nchan + c) * nz;
  const int64_t nx = nz + K - 1 - k0;   // samples of the input row from k0 on
  double acc[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) acc[k] = 0.0;
  // the next piece is loaded into registers while the current one is summed
  double zn[kGwRun];
  float xn[kGwRun], xt = 0.0f;
  auto load_piece = [&](int64_t p0) {
    // zbar[p0 + i] (zero past nz) and x[p0 + k0 + i] (zero past the row)
#pragma unroll
    for (int j = 0; j < kGwRun; ++j) {
      const int i = tid + kThreads * j;
      zn[j] = p0 + i < nz ? zr[p0 + i] : 0.0;
      xn[j] = p0 + i < nx ? (float)xr[p0 + i] : 0.0f;
    }
    if (tid < 16) xt = p0 + kGwPiece + tid < nx ? (float)xr[p0 + kGwPiece + tid] : 0.0f;
  };
  const int64_t c0 = (int64_t)sidx * kGwChunk;
  load_piece(c0);
  for (int it = 0; it < kGwIter; ++it) {
    const int64_t p0 = c0 + (int64_t)it * kGwPiece;
    if (p0 >= nz) break;   // uniform over the workgroup
#pragma unroll
    for (int j = 0; j < kGwRun; ++j) {
      zs[tid + kThreads * j] = zn[j];
      xs[tid + kThreads * j] = xn[j];
    }
    if (tid < 16) xs[kGwPiece + tid] = xt;
    __syncthreads();
    if (it + 1 < kGwIter && p0 + kGwPiece < nz) load_piece(p0 + kGwPiece);
    const double2 *zp = (const double2 *)(zs + kGwRun * tid);
    const float4 *xp = (const float4 *)(xs + kGwRun * tid);
    double zv[kGwRun];
    float xv[XW];
#pragma unroll
    for (int q = 0; q < kGwRun / 2; ++q) *(double2 *)&zv[2 * q] = zp[q];
#pragma unroll
    for (int q = 0; q < XW / 4; ++q) *(float4 *)&xv[4 * q] = xp[q];
#pragma unroll
    for (int q = 0; q < kGwRun; ++q) {
      const double zq = zv[q];
#pragma unroll
      for (int k = 0; k < KB; ++k) acc[k] += zq * (double)xv[q + k];   // k >= kl: never stored
    }
    __syncthreads();
  }
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[k][wave] = v;
  }
  __syncthreads();
  if (tid < kl) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += red[tid][w];
    part[(((int64_t)c * gridDim.z + b) * nsplit + sidx) * K + k0 + tid] = t;
  }
}

// One wave per (c, k): lane l adds partials l, l + 64, ..., then a fixed tree.
__global__ void __launch_bounds__(kThreads)
k_grad_w_tap_sum(const double *__restrict__ part, int32_t nparts, int32_t nchan, int32_t K,
                 double *__restrict__ gw) {
  const int64_t idx = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (idx >= (int64_t)nchan * K) return;   // whole waves leave together
  const int64_t c = idx / K, k = idx - c * K;
  const double *pp = part + c * nparts * K + k;
  double t = 0.0;
  for (int j = lane; j < nparts; j += 64) t += pp[(int64_t)j * K];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
  if (lane == 0) gw[idx] = t;
}

// gx[b][c][i] = sum_k w[c][k] zbar[b][c][i-k] (zbar fp64, fp64 sum, fp32 result).
__global__ void __launch_bounds__(kThreads)
k_grad_x_tap(const double *__restrict__ z, int64_t nz, const float *__restrict__ w, int32_t K,
             int64_t nsamp, int32_t nchan, float *__restrict__ gx, int64_t in_stride,
             int64_t in_bstride) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y, b = blockIdx.z;
  if (i >= nsamp) return;
  const double *zr = z + ((int64_t)b * nchan + c) * nz;
  double acc = 0.0;
  for (int k = 0; k < K; ++k) {
    const int64_t j = i - k;
    if (j >= 0 && j < nz) acc += (double)w[(int64_t)c * K + k] * zr[j];
  }
  gx[(int64_t)b * in_bstride + (int64_t)c * in_stride + i] = (float)acc;
}

// Unit / channel weights, any tap counts: gx[b][c][i] = sum_d w_c sum_{k<n} g[b][d][i-s-k].
__global__ void __launch_bounds__(kThreads)
k_grad_x_direct(const float *__restrict__ g, int64_t nout, int64_t gstride, int64_t gbstride,
                const int32_t *__restrict__ start, const int32_t *__restrict__ ntap,
                const float *__restrict__ w, int32_t nchan, int32_t ndm, int64_t nsamp,
                float *__restrict__ gx, int64_t in_stride, int64_t in_bstride) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int c = blockIdx.y, b = blockIdx.z;
  if (i >= nsamp) return;
  const float *gb = g + (int64_t)b * gbstride;
  double acc = 0.0;
  for (int d = 0; d < ndm; ++d) {
    const int64_t s = start[(int64_t)d * nchan + c];
    const int n = ntap[(int64_t)d * nchan + c];
    for (int k = 0; k < n; ++k) {
      const int64_t t = i - s - k;
      if (t >= 0 && t < nout) acc += (double)gb[(int64_t)d * gstride + t];
    }
  }
  const double wc = w ? (double)w[c] : 1.0;
  gx[(int64_t)b * in_bstride + (int64_t)c * in_stride + i] = (float)(wc * acc);
}

// Channel weights: gw[c] = sum_b sum_d sum_t g[b][d][t] sum_{k<n} x[b][c][t+s+k].
template <typename XT>
__global__ void __launch_bounds__(kThreads)
k_grad_w_channel(const float *__restrict__ g, int64_t nout, int64_t gstride, int64_t gbstride,
                 const int32_t *__restrict__ start, const int32_t *__restrict__ ntap,
                 int32_t nchan, int32_t ndm, int32_t nbatch, const XT *__restrict__ x,
                 int64_t in_stride, int64_t in_bstride, double *__restrict__ gw) {
  const int c = blockIdx.x, tid = threadIdx.x;
  double acc = 0.0;
  for (int b = 0; b < nbatch; ++b)
    for (int d = 0; d < ndm; ++d) {
      const int64_t s = start[(int64_t)d * nchan + c];
      const int n = ntap[(int64_t)d * nchan + c];
      const XT *xr = x + (int64_t)b * in_bstride + (int64_t)c * in_stride + s;
      const float *gr = g + (int64_t)b * gbstride + (int64_t)d * gstride;
      for (int64_t t = tid; t < nout; t += kThreads) {
        double xs = 0.0;
        for (int k = 0; k < n; ++k) xs += (double)xr[t + k];
        acc += (double)gr[t] * xs;
      }
    }
  __shared__ double red[kThreads];
  red[tid] = acc;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) gw[c] = red[0];
}

// Sparse weight gradient: gw[c][k] = sum_e val_e x[b_e][c][t_e + s[d_e,c] + k], fp64,
// entries summed in index order.  One thread per (c, k).
template <typename XT>
__global__ void __launch_bounds__(kThreads)
k_sparse_grad_w(int32_t nnz, const int32_t *__restrict__ eb, const int32_t *__restrict__ ed,
                const int32_t *__restrict__ et, const float *__restrict__ val,
                const int32_t *__restrict__ start, const int32_t *__restrict__ ntap,
                int32_t nchan, int32_t ndm, int32_t K, int32_t tapmode, const XT *__restrict__ x,
                int64_t in_stride, int64_t in_bstride, int32_t nbatch, int64_t nout,
                double *__restrict__ gw) {
  const int idx = blockIdx.x * kThreads + threadIdx.x;
  if (idx >= nchan * K) return;
  const int c = idx / K, k = idx % K;
  double acc = 0.0;
  for (int e = 0; e < nnz; ++e) {
    if (eb[e] < 0 || eb[e] >= nbatch || ed[e] < 0 || ed[e] >= ndm || et[e] < 0 || et[e] >= nout)
      continue;
    const int64_t s = start[(int64_t)ed[e] * nchan + c];
    const int n = ntap[(int64_t)ed[e] * nchan + c];
    const XT *xr = x + (int64_t)eb[e] * in_bstride + (int64_t)c * in_stride + et[e] + s;
    if (tapmode) {
      if (k < n) acc += (double)val[e] * (double)xr[k];
    } else {
      double xs = 0.0;
      for (int q = 0; q < n; ++q) xs += (double)xr[q];
      acc += (double)val[e] * xs;
    }
  }
  gw[idx] = acc;
}

// Selected outputs y[b_e][d_e][t_e] in fp64, rounded to fp32.
template <typename XT>
__global__ void __launch_bounds__(64)
k_gather(int32_t nnz, const int32_t *__restrict__ eb, const int32_t *__restrict__ ed,
         const int32_t *__restrict__ et, const int32_t *__restrict__ start,
         const int32_t *__restrict__ ntap, const float *__restrict__ w, int32_t wmode, int32_t K,
         int32_t nchan, int32_t ndm, const XT *__restrict__ x, int64_t in_stride,
         int64_t in_bstride, int32_t nbatch, int64_t nout, float *__restrict__ out) {
  const int e = blockIdx.x, tid = threadIdx.x;
  if (eb[e] < 0 || eb[e] >= nbatch || ed[e] < 0 || ed[e] >= ndm || et[e] < 0 || et[e] >= nout) {
    if (tid == 0) out[e] = __builtin_nanf("");
    return;
  }
  double acc = 0.0;
  for (int c = tid; c < nchan; c += 64) {
    const int64_t s = start[(int64_t)ed[e] * nchan + c];
    const int n = ntap[(int64_t)ed[e] * nchan + c];
    const XT *xr = x + (int64_t)eb[e] * in_bstride + (int64_t)c * in_stride + et[e] + s;
    for (int k = 0; k < n; ++k) {
      const double wk = wmode == DEDISP_W_TAP ? (double)w[(int64_t)c * K + k]
                        : wmode == DEDISP_W_CHANNEL ? (double)w[c] : 1.0;
      acc += wk * (double)xr[k];
    }
  }
  __shared__ double red[64];
  red[tid] = acc;
  __syncthreads();
  for (int off = 32; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) out[e] = (float)red[0];
}

inline dim3 grid3(int64_t n, int y, int z) {
  return dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)y, (unsigned)z);
}

}  // namespace

// ------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------
hipError_t launch_prefix_u8(const uint8_t *x, int64_t in_stride, int64_t in_bstride, int32_t nchan,
                            int32_t nbatch, int64_t nsamp, int32_t *P, hipStream_t s) {
  const int64_t pstride = nsamp + 1;
  hipLaunchKernelGGL(k_prefix_u8, dim3(nchan, nbatch), dim3(kThreads), 0, s, x, in_stride,
                     in_bstride, nsamp, P, pstride, pstride * nchan);
  return hipGetLastError();
}

hipError_t launch_dedisp_prefix(const dedisp_plan_s *p, const int32_t *P, int64_t pstride,
                                int64_t pbstride, int32_t nbatch, int64_t nout, void *y,
                                int32_t out_dtype, int64_t out_stride, int64_t out_bstride,
                                hipStream_t s) {
  const dim3 g = grid3(nout, p->ndm, nbatch);
  if (p->wmode == DEDISP_W_CHANNEL) {
    hipLaunchKernelGGL((k_dedisp_prefix<true, float>), g, dim3(kThreads), 0, s, P, pstride,
                       pbstride, p->dev.start, p->dev.ntap, weights_of(p), p->nchan, nout,
                       (float *)y, out_stride, out_bstride);
  } else if (out_dtype == DEDISP_I32) {
    hipLaunchKernelGGL((k_dedisp_prefix<false, int32_t>), g, dim3(kThreads), 0, s, P, pstride,
                       pbstride, p->dev.start, p->dev.ntap, nullptr, p->nchan, nout,
                       (int32_t *)y, out_stride, out_bstride);
  } else {
    hipLaunchKernelGGL((k_dedisp_prefix<false, float>), g, dim3(kThreads), 0, s, P, pstride,
                       pbstride, p->dev.start, p->dev.ntap, nullptr, p->nchan, nout, (float *)y,
                       out_stride, out_bstride);
  }
  return hipGetLastError();
}

hipError_t launch_dedisp_direct_f32(const dedisp_plan_s *p, const float *x, int64_t in_stride,
                                    int64_t in_bstride, int32_t nbatch, int64_t nout, float *y,
                                    int64_t out_stride, int64_t out_bstride, hipStream_t s) {
  const dim3 g = grid3(nout, p->ndm, nbatch);
  if (p->wmode == DEDISP_W_CHANNEL)
    hipLaunchKernelGGL(k_dedisp_direct_f32<true>, g, dim3(kThreads), 0, s, x, in_stride,
                       in_bstride, p->dev.start, p->dev.ntap, weights_of(p), p->nchan, nout, y,
                       out_stride, out_bstride);
  else
    hipLaunchKernelGGL(k_dedisp_direct_f32<false>, g, dim3(kThreads), 0, s, x, in_stride,
                       in_bstride, p->dev.start, p->dev.ntap, nullptr, p->nchan, nout, y,
                       out_stride, out_bstride);
  return hipGetLastError();
}

hipError_t launch_fir_f32(const dedisp_plan_s *p, const float *x, int64_t in_stride,
                          int64_t in_bstride, int32_t nbatch, int64_t nz, float *z,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_fir_f32, grid3(nz, p->nchan, nbatch), dim3(kThreads), 0, s, x, in_stride,
                     in_bstride, weights_of(p), p->ktaps, nz, z);
  return hipGetLastError();
}

hipError_t launch_dedisp_1tap_f32(const dedisp_plan_s *p, const float *z, int64_t zstride,
                                  int64_t zbstride, int32_t nbatch, int64_t nout, float *y,
                                  int64_t out_stride, int64_t out_bstride, hipStream_t s) {
  hipLaunchKernelGGL(k_dedisp_1tap_f32, grid3(nout, p->ndm, nbatch), dim3(kThreads), 0, s, z,
                     zstride, zbstride, p->dev.start, p->nchan, nout, y, out_stride, out_bstride);
  return hipGetLastError();
}

hipError_t launch_norm(const dedisp_plan_s *p, const WidthList &wl, const double *mu,
                       const double *sigma, double *M, double *S, hipStream_t s,
                       const ConvertJob *cv) {
  int wmax = 0;
  for (int i = 0; i < wl.n; ++i) wmax = wl.w[i] > wmax ? wl.w[i] : wmax;
  ConvertJob conv{};
  int64_t per_row = 1, nconv = 0;
  if (cv) {
    conv = *cv;
    per_row = (conv.xs_stride / 16 + kConvThreads - 1) / kConvThreads;
    nconv = per_row * conv.nchan;
    if (nconv + p->ndm > 0x7fffffff) return hipErrorInvalidValue;
  }
  if (p->wmode != DEDISP_W_TAP && wmax <= kBucketMaxW) {
    hipLaunchKernelGGL(k_norm_buckets, dim3((unsigned)(p->ndm + nconv)), dim3(64 * kBucketWaves),
                       0, s, p->dev.ntap, p->nchan, p->wmode, weights_of(p), mu, sigma, wl, M, S,
                       p->ndm, conv, per_row);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_norm, dim3((unsigned)((p->ndm + kNormTrials - 1) / kNormTrials)), dim3(kNormThreads), 0, s,
                     p->dev.ntap, p->nchan, p->ndm, p->wmode, p->ktaps, weights_of(p), mu, sigma,
                     wl, M, S);
  if (nconv > 0) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_convert_u8, dim3((unsigned)nconv), dim3(kConvThreads), 0, s, conv, per_row);
  }
  return hipGetLastError();
}

hipError_t launch_boxcar(const dedisp_plan_s *p, const void *y, int32_t y_dtype, int64_t nout,
                         int64_t y_stride, const WidthList &wl, const double *M, const double *S,
                         void *partials, int32_t nchunk, hipStream_t s) {
  const dim3 g((unsigned)nchunk, (unsigned)p->ndm);
  if (y_dtype == DEDISP_I32)
    hipLaunchKernelGGL(k_boxcar<int32_t>, g, dim3(kBoxChunk), 0, s, (const int32_t *)y, nout,
                       y_stride, wl, M, S, (Cand *)partials, nchunk);
  else
    hipLaunchKernelGGL(k_boxcar<float>, g, dim3(kBoxChunk), 0, s, (const float *)y, nout,
                       y_stride, wl, M, S, (Cand *)partials, nchunk);
  return hipGetLastError();
}

hipError_t launch_reduce(int32_t ndm, int32_t nchunk, const void *partials, double *snr,
                         int32_t *t, int32_t *w, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(ndm), dim3(kThreads), 0, s, ndm, nchunk,
                     (const Cand *)partials, snr, t, w);
  return hipGetLastError();
}

hipError_t launch_merge_cand(int32_t ndm, const double *snr_b, const int32_t *t_b,
                             const int32_t *w_b, int64_t t_offset, double *snr, int64_t *t,
                             int32_t *w, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_cand, dim3((unsigned)((ndm + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, ndm, snr_b, t_b, w_b, t_offset, snr, t, w);
  return hipGetLastError();
}

hipError_t launch_adjoint_z(const dedisp_plan_s *p, const float *g, int64_t nout, int64_t gstride,
                            int64_t gbstride, int32_t nbatch, int64_t nz, double *z,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_adjoint_z, grid3(nz, p->nchan, nbatch), dim3(kThreads), 0, s, g, nout,
                     gstride, gbstride, p->dev.start, p->nchan, p->ndm, nz, z);
  return hipGetLastError();
}

hipError_t launch_grad_w_tap(const dedisp_plan_s *p, const double *z, int64_t nz, const void *x,
                             int32_t in_dtype, int64_t in_stride, int64_t in_bstride,
                             int32_t nbatch, double *gw, hipStream_t s) {
  const int K = p->ktaps;
  if (K < 1 || K > kGwMaxK || nz < 1) return hipErrorInvalidValue;
  const int64_t nsplit = (nz + kGwChunk - 1) / kGwChunk;
  const int64_t nparts = nsplit * nbatch;
  const int kb = K <= 8 ? 8 : 16;
  const int nslice = (K + kb - 1) / kb;
  if (nsplit * nslice > INT32_MAX || nparts > INT32_MAX || p->nchan > 65535 || nbatch > 65535)
    return hipErrorInvalidValue;
  double *part = nullptr;
  hipError_t e =
      dev_malloc_async((void **)&part, sizeof(double) * (size_t)p->nchan * nparts * K, s);
  if (e != hipSuccess) return e;
  const dim3 g((unsigned)(nsplit * nslice), (unsigned)p->nchan, (unsigned)nbatch);
#define DD_GW_LAUNCH(XT, KB)                                                     \
  hipLaunchKernelGGL((k_grad_w_tap_part<XT, KB>), g, dim3(kThreads), 0, s, z, nz, \
                     (const XT *)x, in_stride, in_bstride, p->nchan, K, nslice, part)
  if (in_dtype == DEDISP_F32) {
    if (kb == 8) DD_GW_LAUNCH(float, 8);
    else DD_GW_LAUNCH(float, 16);
  } else {
    if (kb == 8) DD_GW_LAUNCH(uint8_t, 8);
    else DD_GW_LAUNCH(uint8_t, 16);
  }
#undef DD_GW_LAUNCH
  e = hipGetLastError();
  if (e == hipSuccess) {
    const int64_t n = (int64_t)p->nchan * K;   // one wave each
    constexpr int kWaves = kThreads / 64;
    hipLaunchKernelGGL(k_grad_w_tap_sum, dim3((unsigned)((n + kWaves - 1) / kWaves)),
                       dim3(kThreads), 0, s, part, (int32_t)nparts, p->nchan, K, gw);
    e = hipGetLastError();
  }
  hipError_t e2 = hipFreeAsync(part, s);
  return e != hipSuccess ? e : e2;
}

hipError_t launch_grad_x_tap(const dedisp_plan_s *p, const double *z, int64_t nz, int64_t nsamp,
                             int32_t nbatch, float *gx, int64_t in_stride, int64_t in_bstride,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_grad_x_tap, grid3(nsamp, p->nchan, nbatch), dim3(kThreads), 0, s, z, nz,
                     weights_of(p), p->ktaps, nsamp, p->nchan, gx, in_stride, in_bstride);
  return hipGetLastError();
}

hipError_t launch_adjoint_direct(const dedisp_plan_s *p, const float *g, int64_t nout,
                                 int64_t gstride, int64_t gbstride, int32_t nbatch, const void *x,
                                 int32_t in_dtype, int64_t nsamp, int64_t in_stride,
                                 int64_t in_bstride, float *gx, double *gw, hipStream_t s) {
  if (gx)
    hipLaunchKernelGGL(k_grad_x_direct, grid3(nsamp, p->nchan, nbatch), dim3(kThreads), 0, s, g,
                       nout, gstride, gbstride, p->dev.start, p->dev.ntap,
                       p->wmode == DEDISP_W_CHANNEL ? weights_of(p) : nullptr, p->nchan, p->ndm,
                       nsamp, gx, in_stride, in_bstride);
  if (gw) {
    if (in_dtype == DEDISP_F32)
      hipLaunchKernelGGL(k_grad_w_channel<float>, dim3(p->nchan), dim3(kThreads), 0, s, g, nout,
                         gstride, gbstride, p->dev.start, p->dev.ntap, p->nchan, p->ndm, nbatch,
                         (const float *)x, in_stride, in_bstride, gw);
    else
      hipLaunchKernelGGL(k_grad_w_channel<uint8_t>, dim3(p->nchan), dim3(kThreads), 0, s, g, nout,
                         gstride, gbstride, p->dev.start, p->dev.ntap, p->nchan, p->ndm, nbatch,
                         (const uint8_t *)x, in_stride, in_bstride, gw);
  }
  return hipGetLastError();
}

hipError_t launch_sparse_grad_w(const dedisp_plan_s *p, int32_t nnz, const int32_t *b,
                                const int32_t *d, const int32_t *t, const float *val,
                                const void *x, int32_t in_dtype, int64_t in_stride,
                                int64_t in_bstride, int32_t nbatch, int64_t nout, double *gw,
                                hipStream_t s) {
  const int K = p->ktaps;
  const int tapmode = p->wmode == DEDISP_W_TAP;
  const int n = p->nchan * K;
  const dim3 g((unsigned)((n + kThreads - 1) / kThreads));
  if (in_dtype == DEDISP_F32)
    hipLaunchKernelGGL(k_sparse_grad_w<float>, g, dim3(kThreads), 0, s, nnz, b, d, t, val,
                       p->dev.start, p->dev.ntap, p->nchan, p->ndm, K, tapmode, (const float *)x,
                       in_stride, in_bstride, nbatch, nout, gw);
  else
    hipLaunchKernelGGL(k_sparse_grad_w<uint8_t>, g, dim3(kThreads), 0, s, nnz, b, d, t, val,
                       p->dev.start, p->dev.ntap, p->nchan, p->ndm, K, tapmode,
                       (const uint8_t *)x, in_stride, in_bstride, nbatch, nout, gw);
  return hipGetLastError();
}

hipError_t launch_gather(const dedisp_plan_s *p, int32_t nnz, const int32_t *b, const int32_t *d,
                         const int32_t *t, const void *x, int32_t in_dtype, int64_t in_stride,
                         int64_t in_bstride, int32_t nbatch, int64_t nout, float *out,
                         hipStream_t s) {
  if (in_dtype == DEDISP_F32)
    hipLaunchKernelGGL(k_gather<float>, dim3(nnz), dim3(64), 0, s, nnz, b, d, t, p->dev.start,
                       p->dev.ntap, weights_of(p), p->wmode, p->ktaps, p->nchan, p->ndm,
                       (const float *)x, in_stride, in_bstride, nbatch, nout, out);
  else
    hipLaunchKernelGGL(k_gather<uint8_t>, dim3(nnz), dim3(64), 0, s, nnz, b, d, t, p->dev.start,
                       p->dev.ntap, weights_of(p), p->wmode, p->ktaps, p->nchan, p->ndm,
                       (const uint8_t *)x, in_stride, in_bstride, nbatch, nout, out);
  return hipGetLastError();
}

}  // namespace dd
