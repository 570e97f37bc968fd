// Boxcar S/N search (eq. snr) over one tile of one trial's dedispersed series,
// by one wave: the best (S/N, width, earliest start) among the tile's starts.
// Shared by the fused search kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

namespace dd {

constexpr int kHalo = 32;   // boxcar widths up to 32

struct CandRec {
  double snr;
  int32_t t;
  int32_t w;
};

// Lane l's double.
__device__ __forceinline__ double rl_double(double x, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One step of a wave maximum of a double: the larger of x and the value the
// 32-bit lane movement F brings to this lane (applied to both halves).
template <typename F>
__device__ __forceinline__ double dmax_step(double x, F move) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = move((uint32_t)u), hi = move((uint32_t)(u >> 32));
  const double o = __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
  return __builtin_fmax(x, o);
}

// The larger of the two doubles a permlane swap of x with itself gives this lane
// (the lane's own value and its partner's, in some order).
template <bool P32>
__device__ __forceinline__ double dmax_swap(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
  uint32_t l0, l1, h0, h1;
  if constexpr (P32) {
    const auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    l0 = pl[0]; l1 = pl[1]; h0 = ph[0]; h1 = ph[1];
  } else {
    const auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    l0 = pl[0]; l1 = pl[1]; h0 = ph[0]; h1 = ph[1];
  }
  const double a = __builtin_bit_cast(double, ((uint64_t)h0 << 32) | l0);
  const double b = __builtin_bit_cast(double, ((uint64_t)h1 << 32) | l1);
  return __builtin_fmax(a, b);
}

// Yw (16-byte aligned) holds the TY = 64 SP outputs of the tile (outputs t0 .. t0 + TY - 1, written by
// this wave before the call, or by any wave before a workgroup barrier), followed by
// kHalo ints that this function sets to zero.  The tile owns starts t0 .. t0 + TT - 1
// (TT <= TY - 31); outputs at or past nout are not part of the series.  M, S: the
// noise mean and deviation of each listed width of trial dg (row dg of [ndm][nw]);
// wmask: bit W - 1 set for each listed width W <= 32.  Returns, in every lane, the
// best candidate (snr -inf, t -1, w 0 if none): larger S/N first, then smaller
// width, then earlier start.
template <int SP>
__device__ __forceinline__ CandRec boxcar_row(int *Yw, int lane, int64_t t0, int TT, int64_t nout,
                                              int dg, uint32_t wmask, int nw,
                                              const double *__restrict__ M,
                                              const double *__restrict__ S) {
  constexpr int TY = 64 * SP;
  // The width this lane speaks for in the S/N step: register index from lane bits
  // 1-4, pair member from bit 5 (lanes l and l ^ 1 agree); its index in the sorted
  // width list is the number of listed widths below it.  Its noise mean and
  // deviation are loaded first, so that the loads are in flight during the sums.
  const int wl = 2 * ((lane >> 1) & 15) + (lane >> 5) + 1;
  const int ji = ((wmask >> (wl - 1)) & 1u) ? __popc(wmask & ((1u << (wl - 1)) - 1u)) : -1;
  double nm = 0.0, ns = 1.0;
  if (ji >= 0 && dg >= 0) {
    nm = M[(int64_t)dg * nw + ji];
    ns = S[(int64_t)dg * nw + ji];
  }
  if (lane < kHalo) Yw[TY + lane] = 0;
  // Only the tile holding the end of the series sees outputs past the last valid
  // one.  Elsewhere every prefix entry is a real output, except the zero halo past
  // TY: windows of lanes whose starts belong to the next tile may run into it and
  // come out short, never larger than the same window in the tile that owns the
  // start, which finds it exactly; so they cannot win falsely.
  const bool tail = t0 + TY + kHalo > nout;
  // LDS operations of one wave complete in order: the reads below see the writes
  __builtin_amdgcn_wave_barrier();
  // Window sums come from the running prefix qv[k] = y[0] + .. + y[k-1] of this
  // lane's SP + 32 outputs.  In the tail tile, prefix entries past the last
  // valid output (all of them for lanes without starts in this tile) are pushed
  // down so that every window that is not a valid (start, width) comes out
  // negative; windows of unit-weight uint8 sums are otherwise >= 0.
  // Yw is 16-byte aligned and SP a multiple of 4: the lane's outputs come in 16-byte
  // reads (4 per instruction instead of 1, a quarter of the bank-conflict cycles)
  static_assert(SP % 4 == 0, "lane runs of whole 16-byte words");
  const int *yl = (const int *)__builtin_assume_aligned(Yw + lane * SP, 16);
  int lim = SP + kHalo;
  if (tail) {
    const int64_t room = nout - (t0 + lane * SP);
    lim = (lane * SP < TT) ? (int)(room < SP + kHalo ? room : SP + kHalo) : -1;
  }
  int qv[SP + kHalo + 1];
  qv[0] = 0;
#pragma unroll
  for (int k = 0; k < SP + kHalo; ++k) qv[k + 1] = qv[k] + yl[k];
  __builtin_amdgcn_wave_barrier();
  if (tail) {
    // An opaque copy of the limit, so that the compiler neither folds this branch into
    // selects run for every row nor hoists the comparisons out of the caller's row loop
    // (their masks would occupy scalar registers across it)
    int lt = lim;
    asm volatile("" : "+v"(lt));
#pragma unroll
    for (int k = 0; k <= SP + kHalo; ++k)
      if (k > lt) qv[k] = (INT_MIN / 4) - (k - lt);
  }
  // Per width: the lane maximum over its starts (made for all 32 widths; the
  // widths not searched are dropped at the S/N step), reduced across the wave
  // by a transposed butterfly: each level
  // halves the registers and doubles the lanes each register is reduced over.
  // Widths are taken in ascending pairs (2r + 1, 2r + 2), so each prefix entry
  // is needed only for a short run of widths, and the first level (lanes l,
  // l ^ 32: the lower half keeps width 2r + 1, the upper half 2r + 2) runs as
  // the maxima are made.
  int mw[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    int m2[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int w = 2 * r + h + 1;
      int m = qv[w] - qv[0];
#pragma unroll
      for (int i = 1; i < SP; ++i) m = max(m, qv[i + w] - qv[i]);
      m2[h] = m;
    }
    const auto p = __builtin_amdgcn_permlane32_swap(m2[0], m2[1], false, false);
    mw[r] = max((int)p[0], (int)p[1]);
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {    // lanes l, l ^ 16: rows 0, 2 keep r, rows 1, 3 r + 8
    const auto p = __builtin_amdgcn_permlane16_swap(mw[r], mw[r + 8], false, false);
    mw[r] = max((int)p[0], (int)p[1]);
  }
  const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0, b1 = (lane & 2) != 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {    // lanes l, l ^ 8 (rotate by 8 within a row)
    int t = __builtin_amdgcn_update_dpp(0, mw[r + 4], 0x128, 0xf, 0xc, false);
    t = __builtin_amdgcn_update_dpp(t, mw[r], 0x128, 0xf, 0x3, false);
    mw[r] = max(b3 ? mw[r + 4] : mw[r], t);
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {    // lanes l, l ^ 4 (a row rotation by n moves lane i - n to i)
    int t = __builtin_amdgcn_update_dpp(0, mw[r + 2], 0x124, 0xf, 0xa, false);
    t = __builtin_amdgcn_update_dpp(t, mw[r], 0x12c, 0xf, 0x5, false);
    mw[r] = max(b2 ? mw[r + 2] : mw[r], t);
  }
  {                                // lanes l, l ^ 2 (quad permutation 2, 3, 0, 1)
    const int send = b1 ? mw[0] : mw[1];
    const int t = __builtin_amdgcn_update_dpp(0, send, 0x4e, 0xf, 0xf, false);
    mw[0] = max(b1 ? mw[1] : mw[0], t);
  }
  // lanes l, l ^ 1 (quad permutation 1, 0, 3, 2)
  const int bmax = max(mw[0], __builtin_amdgcn_update_dpp(0, mw[0], 0xb1, 0xf, 0xf, false));
  // S/N of the width this lane speaks for (NaN, as from 0 / 0, never wins: -inf)
  double snr = -INFINITY;
  if (ji >= 0 && bmax >= 0 && dg >= 0) {
    const double r = ((double)bmax - nm) / ns;
    if (!__builtin_isnan(r)) snr = r;
  }
  // wave maximum of the S/N over the widths, every lane ending with it
  double smax = snr;
  smax = dmax_step(smax, [](uint32_t v) {   // lanes l, l ^ 2 (quad permutation 2, 3, 0, 1)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false);
  });
  smax = dmax_step(smax, [](uint32_t v) {   // quads q, q + 1 of a row (rotation by 4)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, false);
  });
  smax = dmax_step(smax, [](uint32_t v) {   // the whole row (rotation by 8)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false);
  });
  smax = dmax_swap<false>(smax);            // rows 2 k, 2 k + 1
  smax = dmax_swap<true>(smax);             // all four rows
  CandRec rec;
  rec.snr = -INFINITY;
  rec.t = -1;
  rec.w = 0;
  if (smax == -INFINITY) return rec;        // no valid window of a listed width
  // the smallest width with that S/N: lane 2 r (+ 1) speaks for width 2 r + 1,
  // lane 32 + 2 r (+ 1) for width 2 r + 2, so bit W - 1 of wbits is width W's
  const uint64_t hit = __ballot(snr == smax);
  const uint32_t wbits = ((uint32_t)hit & 0x55555555u) | (((uint32_t)(hit >> 32) & 0x55555555u) << 1);
  const int bw = __builtin_amdgcn_readfirstlane(__builtin_ctz(wbits) + 1);
  const int wlane = 32 * ((bw - 1) & 1) + ((bw - 1) & ~1);
  const int bb = __builtin_amdgcn_readlane(bmax, wlane);
  // The winning windows: those of width bw whose S/N equals smax.  With a noise deviation
  // 0 < S < inf the S/N rises strictly with the window sum, so they are the windows of
  // sum bb; with S = 0 (every window above the mean has S/N +inf) or S = inf (every
  // finite window 0) other sums tie, so their S/N is compared itself.
  const double ws = rl_double(ns, wlane), wm = rl_double(nm, wlane);
  const bool strict = ws > 0.0 && ws < INFINITY;
  // earliest such start: per lane a sliding window over its outputs (only valid windows,
  // i + bw <= lim, count), then the lowest lane that has one
  int first = -1;
  {
    int B = 0;
    for (int k = 0; k < bw; ++k) B += yl[k];
    if (strict) {
#pragma unroll
      for (int i = 0; i < SP; ++i) {
        if (first < 0 && B == bb && i + bw <= lim) first = i;
        B += yl[i + bw] - yl[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < SP; ++i) {
        if (first < 0 && ((double)B - wm) / ws == smax && i + bw <= lim) first = i;
        B += yl[i + bw] - yl[i];
      }
    }
  }
  const uint64_t fh = __ballot(first >= 0);
  if (fh == 0ull) return rec;
  const int fl = __builtin_amdgcn_readfirstlane(__builtin_ctzll(fh));
  rec.snr = smax;
  rec.t = (int)(t0 + fl * SP + __builtin_amdgcn_readlane(first, fl));
  rec.w = bw;
  return rec;
}

}  // namespace dd
