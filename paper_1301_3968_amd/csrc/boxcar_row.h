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
#pragma unroll
    for (int k = 0; k <= SP + kHalo; ++k)
      if (k > lim) qv[k] = (INT_MIN / 4) - (k - lim);
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
  // the width this lane speaks for: register index from lane bits 1-4, pair
  // member from bit 5 (lanes l and l ^ 1 agree)
  const int wl = 2 * ((lane >> 1) & 15) + (lane >> 5) + 1;
  // index of width wl in the sorted width list = number of listed widths below it
  const int ji = ((wmask >> (wl - 1)) & 1u) ? __popc(wmask & ((1u << (wl - 1)) - 1u)) : -1;
  double snr = -INFINITY;
  if (ji >= 0 && bmax >= 0 && dg >= 0)
    snr = ((double)bmax - M[(int64_t)dg * nw + ji]) / S[(int64_t)dg * nw + ji];
  // wave argmax over (snr desc, W asc); every lane ends with the result
  int bw = wl, bb = bmax;
#pragma unroll
  for (int sh = 2; sh < 64; sh <<= 1) {
    const double os = __shfl_xor(snr, sh, 64);
    const int ow = __shfl_xor(bw, sh, 64), ob = __shfl_xor(bb, sh, 64);
    if (os > snr || (os == snr && ow < bw)) {
      snr = os;
      bw = ow;
      bb = ob;
    }
  }
  // earliest start of the winning width in this tile: a sliding window of width
  // bw over this lane's outputs (only valid windows, i + bw <= lim, can match)
  int first = -1;
  if (snr != -INFINITY) {
    int B = 0;
    for (int k = 0; k < bw; ++k) B += yl[k];
#pragma unroll
    for (int i = 0; i < SP; ++i) {
      if (first < 0 && B == bb && i + bw <= lim) first = i;
      B += yl[i + bw] - yl[i];
    }
  }
  const unsigned long long hit = __ballot(first >= 0);
  int tbest = -1;
  if (hit != 0ull) {
    const int fl = __builtin_ctzll(hit);
    const int fi = __shfl(first, fl, 64);
    tbest = (int)(t0 + fl * SP + fi);
  }
  CandRec rec;
  rec.snr = (hit != 0ull) ? snr : -INFINITY;
  rec.t = (hit != 0ull) ? tbest : -1;
  rec.w = (hit != 0ull) ? bw : 0;
  return rec;
}

}  // namespace dd
