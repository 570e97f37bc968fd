// Noise tables and per-trial reductions shared by the one-plan launches and the
// multi-beam launch (one workgroup per trial in both).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "internal.h"

namespace dd {

// Noise statistics for unit or per-channel weights and widths up to kBucketMaxW, by
// tap-count buckets.  For a channel taking n samples, the length-W boxcar of the
// dedispersed series weights its samples by the n-box convolved with the W-box, whose
// sum of squares is q(W, n) = L^2 H + b(L) with L = min(W, n), H = max(W, n) and
// b(L) = L^2 - L^3 + (L - 1) L (2L - 1) / 3 (the same for either order).  So
//     M[W] = W sum_c m_c n_c,   S[W]^2 = sum_c v_c q(W, n_c),
// with m_c = w_c mu_c, v_c = (w_c sigma_c)^2, and the channels with equal n < 64 can be
// summed first; those with n >= 64 exceed every width (q = W^2 n + b(W)) and enter
// through sum v_c n_c and sum v_c.  One workgroup per trial, its 4 waves taking a
// quarter of the channels each, a chunk at a time: the lanes first take one channel
// each (m_c n_c and the n >= 64 sums, and (n_c, v_c) into LDS), then lane k adds v_c
// over the chunk's channels with n_c = k.  Every sum runs in a fixed order, so results
// do not vary between runs.
constexpr int kBucketMaxW = 63, kBucketWaves = 4, kBucketChunk = 256;

__device__ __forceinline__ int bucket_q(int W, int n) {   // q(W, n) for W, n <= 63
  const int L = min(W, n), H = max(W, n);
  return L * L * H + L * L - L * L * L + (L - 1) * L * (2 * L - 1) / 3;
}

__device__ __forceinline__ double wave_sum(double x) {   // fixed butterfly order
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// The noise tables of one trial (M[W], S[W] for the listed widths) from its tap-count row
// nrow[nchan]; one workgroup of 64 kBucketWaves threads.
__device__ __forceinline__ void norm_buckets_trial(const int32_t *__restrict__ nrow, int nchan,
                                                   int wmode, const float *__restrict__ w,
                                                   const double *__restrict__ mu,
                                                   const double *__restrict__ sigma,
                                                   const WidthList &wl, double *__restrict__ M,
                                                   double *__restrict__ S) {
  __shared__ double cv[kBucketWaves][kBucketChunk];
  __shared__ int32_t cn[kBucketWaves][kBucketChunk];
  __shared__ double sv[kBucketWaves][64];
  __shared__ double sd[kBucketWaves][3];
  const int lane = threadIdx.x & 63;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int per = (nchan + kBucketWaves - 1) / kBucketWaves;
  const int cb = min(nchan, q * per), ce = min(nchan, cb + per);
  double smn = 0.0, svn = 0.0, sv0 = 0.0, bv = 0.0;
  for (int c0 = cb; c0 < ce; c0 += kBucketChunk) {
    const int len = min(kBucketChunk, ce - c0);
    for (int i = lane; i < len; i += 64) {
      const int c = c0 + i, n = nrow[c];
      const double wc = wmode == DEDISP_W_CHANNEL ? (double)w[c] : 1.0;
      const double sg = sigma[c] * wc, v = sg * sg;
      smn += mu[c] * wc * (double)n;
      if (n >= 64) {
        svn += v * (double)n;
        sv0 += v;
      }
      cv[q][i] = v;
      cn[q][i] = n;
    }
    // LDS operations of one wave complete in order: the reads below see the writes
    __builtin_amdgcn_wave_barrier();
#pragma unroll 8
    for (int i = 0; i < len; ++i) bv += (cn[q][i] == lane && lane != 0) ? cv[q][i] : 0.0;
    __builtin_amdgcn_wave_barrier();
  }
  smn = wave_sum(smn);
  svn = wave_sum(svn);
  sv0 = wave_sum(sv0);
  sv[q][lane] = bv;
  if (lane == 0) {
    sd[q][0] = smn;
    sd[q][1] = svn;
    sd[q][2] = sv0;
  }
  __syncthreads();
  if (q != 0) return;
  double tot = 0.0, msum = 0.0, vn = 0.0, v0 = 0.0;
#pragma unroll
  for (int r = 0; r < kBucketWaves; ++r) {
    tot += sv[r][lane];
    msum += sd[r][0];
    vn += sd[r][1];
    v0 += sd[r][2];
  }
  __builtin_amdgcn_wave_barrier();
  sv[0][lane] = tot;   // bucket totals (wave 0 alone reads and writes row 0 now)
  __builtin_amdgcn_wave_barrier();
  // the highest tap count below 64 that any channel takes (buckets above it are empty)
  const uint64_t used = __ballot(lane != 0 && tot != 0.0);
  const int kmax = used ? 63 - __builtin_clzll(used) : 0;
  // lane j takes width j (the list has at most 64 entries)
  if (lane >= wl.n) return;
  const int W = wl.w[lane];
  const int bW = W * W - W * W * W + (W - 1) * W * (2 * W - 1) / 3;
  double v = (double)(W * W) * vn + (double)bW * v0;
  for (int k = 1; k <= kmax; ++k) v += (double)bucket_q(W, k) * sv[0][k];
  M[lane] = (double)W * msum;
  S[lane] = sqrt(v);
}

// Ranking of candidates: larger S/N, then smaller width, then earlier start.
__device__ __forceinline__ bool better(double s1, int w1, int t1, double s2, int w2, int t2) {
  if (s1 != s2) return s1 > s2;
  if (w1 != w2) return w1 < w2;
  return t1 < t2;
}

// The best of one trial's n candidates (C: snr, t, w; t < 0 holds no window) by a
// workgroup of kReduceThreads threads, in a fixed order; (-inf, -1, 0) if none.
constexpr int kReduceThreads = 256;
template <typename C>
__device__ __forceinline__ void best_of_row(const C *__restrict__ row, int n, double *snr,
                                            int32_t *tout, int32_t *wout) {
  const int tid = threadIdx.x;
  double best = -INFINITY;
  int bw = 0, bt = -1;
  for (int i = tid; i < n; i += kReduceThreads) {
    const C c = row[i];
    if (c.t >= 0 && (bt < 0 || better(c.snr, c.w, c.t, best, bw, bt))) {
      best = c.snr;
      bw = c.w;
      bt = c.t;
    }
  }
  __shared__ double s_snr[kReduceThreads];
  __shared__ int s_w[kReduceThreads], s_t[kReduceThreads];
  s_snr[tid] = best;
  s_w[tid] = bw;
  s_t[tid] = bt;
  __syncthreads();
  for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
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
  if (tid == 0) {
    *snr = s_t[0] >= 0 ? s_snr[0] : -INFINITY;
    *tout = s_t[0];
    *wout = s_w[0];
  }
}

}  // namespace dd
