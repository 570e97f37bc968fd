// Dedispersion of uint8 data with unit weights (eq. p_dedisp) on the int8 matrix cores.
//
// For a tile of 16 trials and a channel c, the samples a trial adds lie in a short band
// of delays: trial d takes x[c][t + start[d,c] + k] for k < ntap[d,c], and over the 16
// trials these delays span [lo_c, lo_c + L_c).  Cutting the band into segments of 16
// delays, the tile's sums over channel c are
//     y[d][t] += sum_{segments s} sum_{j<16} mask_s[d][j] * x[c][t + o_s + j],
// a product of a 16 x 16 0/1 matrix (which delays trial d takes) with a 16 x T Hankel
// matrix of samples.  Four segments (of one or several channels) make the K = 64 of one
// v_mfma_i32_16x16x64_i8; the samples enter as int8 x ^ 0x80 = x - 128, and every
// trial's result is corrected by 128 times its number of samples, so the int32 result
// is exact.
//
// One wave takes 16 trials x 256 outputs as 16 products (blocks b < 16); column n of
// block b is output 16 n + b of the wave's run.  So lane n of a segment needs window
// bytes o + 16 n + b .. o + 16 n + b + 15 for block b: for all 16 blocks, the 32 bytes
// from o + 16 n, two aligned 16-byte LDS reads when o is a multiple of 16; block b then
// takes bytes b .. b + 15 of them, a shift by b that is the same for every lane (three
// byte-align operations per dword, none when b is a multiple of 4).  Segment starts are
// put on a 4-byte grid (one or two more segments than the band needs, rarely), and each
// channel's window is staged into LDS as 4 copies shifted by 0, 4, 8 and 12 bytes, so
// the copy (o / 4) mod 4 holds the segment's bytes at 16-byte alignment.  Channel groups
// are staged while the previous group is multiplied (two LDS buffers).  The host plans,
// per group of 4 segments (a K block), a 144-byte record: the 16-bit mask of every
// (trial, segment) (which of the segment's 16 delays the trial takes) and the LDS
// address of each segment's aligned bytes; the records of a channel group are copied
// into LDS with the windows, and every lane forms its 16 mask bytes and its read
// address from them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "boxcar_row.h"
#include "internal.h"

namespace dd {

// Workgroup shapes: NWD waves along DM (16 trials each), NWT along time (256 outputs
// each), WG workgroups per CU (each with 1 / WG of the CU's LDS).
#define DD_MFMA_CONFIGS(X) \
  X(0, 4, 2, 2)            \
  X(1, 8, 1, 2)            \
  X(2, 8, 2, 1)            \
  X(3, 16, 1, 1)           \
  X(4, 4, 4, 1)
struct MfmaCfg {
  int nwd, nwt, wg;
};
#define DD_MFMA_ENTRY(i, a, b, g) {a, b, g},
static const MfmaCfg kMfmaCfgs[] = {DD_MFMA_CONFIGS(DD_MFMA_ENTRY)};
#undef DD_MFMA_ENTRY
constexpr int kNumMfmaCfgs = sizeof(kMfmaCfgs) / sizeof(kMfmaCfgs[0]);
constexpr int kNT = 16;                     // products (blocks) per wave and K block
constexpr int kTWV = 16 * kNT;              // outputs per wave
constexpr int kCopies = 4;                  // dword-shifted copies of each staged window
constexpr int kMfmaBufBytes = 80 * 1024;    // LDS per staging buffer (two per workgroup) at
                                            // one workgroup per CU
// K-block record: 64 x u16 masks (lane = 16 segment + trial row), then the LDS byte
// address of each of the 4 segments' aligned bytes (lane 16 g + n reads 32 bytes at
// address[g] + 16 n)
constexpr int kRecBytes = 160;
// Staging: one chunk (16 window bytes in all 4 copies) per thread and group, so a
// group stages at most 64 NW chunks (registers: the chunk's raw bytes are held through
// the current group's products).

struct MGroup {
  int32_t unit_begin, nunits;   // staging units (16 window bytes of one channel each)
  int32_t kb_base;              // index into the per-wave K-block ranges
  int32_t kb_first, nkb;        // the group's K blocks (all waves): first and count
  int32_t rec_off;              // LDS byte offset of their records in the buffer
  int32_t pad0, pad1;
};
struct MUnit {
  int32_t c;      // channel
  int32_t src;    // first window sample of the chunk, relative to the tile's first output
  int32_t dst;    // LDS byte offset of the chunk in copy 0
  int32_t cs;     // bytes between the copies of the channel's window
};

struct MfmaCfgTables {
  bool ok = false;
  int tw = 0, ntw = 0, trials = 0;
  std::vector<int32_t> perm, ntot, group_begin, kbr;
  std::vector<MGroup> groups;
  std::vector<MUnit> units;
  int bufbytes = 0;               // LDS bytes of one staging buffer
  std::vector<uint8_t> recs;      // [kb][kRecBytes]
  int32_t *d_perm = nullptr, *d_ntot = nullptr, *d_group_begin = nullptr, *d_kbr = nullptr;
  MGroup *d_groups = nullptr;
  MUnit *d_units = nullptr;
  uint8_t *d_recs = nullptr;
};
struct MfmaTables {
  MfmaCfgTables cfg[kNumMfmaCfgs];
  bool tried[kNumMfmaCfgs] = {};
};

void free_mfma(MfmaTables *t) {
  if (!t) return;
  for (auto &c : t->cfg) {
    (void)hipFree(c.d_perm);
    (void)hipFree(c.d_ntot);
    (void)hipFree(c.d_group_begin);
    (void)hipFree(c.d_kbr);
    (void)hipFree(c.d_groups);
    (void)hipFree(c.d_units);
    (void)hipFree(c.d_recs);
  }
  delete t;
}

namespace {

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
constexpr unsigned kWaitVm0 = 0x0f70;      // s_waitcnt vmcnt(0) (gfx9 encoding)
constexpr int kBufWord3 = 0x00020000;      // raw 32-bit buffer descriptor word 3

struct MfmaArgs {
  const uint8_t *x;
  int64_t in_stride, in_bstride, nsamp;
  int32_t ntw, ntt, bufbytes;
  int32_t pad0;
  const int32_t *group_begin, *kbr, *perm, *ntot;
  const MGroup *groups;
  const MUnit *units;
  const uint8_t *recs;
  int32_t *out;
  int64_t out_stride, out_bstride, nout;
};

template <typename T>
__device__ __forceinline__ T ldc(const T *p, int64_t i) {
  return ((const __attribute__((address_space(4))) T *)p)[i];
}

// The 32 bytes of the row from the 4-byte aligned address at or below row + pos (pos
// may be past the row; bytes outside [0, nsamp) read as 0), as 8 dwords.
__device__ __forceinline__ void load_raw(const uint8_t *row, int64_t nsamp, int64_t pos,
                                         uint32_t raw[8], int *sh) {
  const uintptr_t abs = (uintptr_t)(row + pos);
  *sh = (int)(abs & 3);
  const int64_t p0 = pos - *sh;   // row-relative position of the aligned first byte
  // a global (not flat) pointer: flat loads would also count against the LDS counter
  // and force full LDS waits in the product loop while they are in flight
  const __attribute__((address_space(1))) uint32_t *a =
      (const __attribute__((address_space(1))) uint32_t *)(abs - *sh);
  if (p0 >= 0 && p0 + 32 <= nsamp) {
#pragma unroll
    for (int k = 0; k < 8; ++k) raw[k] = a[k];
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uint32_t v = 0;
      for (int j = 0; j < 4; ++j) {
        const int64_t q = p0 + 4 * k + j;
        if (q >= 0 && q < nsamp) v |= (uint32_t)row[q] << (8 * j);
      }
      raw[k] = v;
    }
  }
}

// One staging task: chunk k of the 4 copies of a window (copy p: window bytes 16 k + 4 p
// .. 16 k + 4 p + 15, as int8 x ^ 0x80), from the raw bytes at the aligned address at or
// below window byte 16 k.  dst: the chunk's offset in copy 0; cs: bytes between copies.
__device__ __forceinline__ void store_chunk(unsigned char *buf, int32_t dst, int32_t cs,
                                            const uint32_t raw[8], int sh) {
  uint32_t e[7];
#pragma unroll
  for (int k = 0; k < 7; ++k)
    e[k] = __builtin_amdgcn_alignbyte(raw[k + 1], raw[k], (uint32_t)sh) ^ 0x80808080u;
#pragma unroll
  for (int p = 0; p < kCopies; ++p) {
    const v4i v = {(int32_t)e[p], (int32_t)e[p + 1], (int32_t)e[p + 2], (int32_t)e[p + 3]};
    *(v4i *)(buf + dst + p * cs) = v;
  }
}

// XCD-aware tile order (blocks b = x mod 8 run on XCD x): XCD x takes a contiguous
// run of tiles in time-major order, so the DM tiles of one time tile share its L2.
__device__ __forceinline__ void tile_of_block(int ntw, int ntt, int *tt, int *tw) {
  const int nb = ntw * ntt;
  const int bi = blockIdx.x;
  const int xcd = bi & 7, kk = bi >> 3, q = nb >> 3, rem = nb & 7;
  const int L = xcd * q + min(xcd, rem) + kk;
  *tt = L / ntw;
  *tw = L - *tt * ntw;
}

template <int N>
struct TileAcc {
  v4i v[N];
};

typedef int32_t v8i __attribute__((ext_vector_type(8)));
typedef int32_t v2i __attribute__((ext_vector_type(2)));

// Shifted samples: T[k] = the lane's bytes shifted down by S bytes, dword k + O (k < 6;
// dwords 6, 7 unused).  Block 4 q + S takes dwords q .. q + 3 of the shifted bytes: from
// the O = 0 tuple at offset q for even q, from the O = 1 tuple at offset q - 1 for odd q,
// so that every operand starts at an even register of its tuple (4-register operands
// must; an odd start would be copied into place).
template <int S, int O>
__device__ __forceinline__ v8i shifted(const v8i &w) {
  // the O = 1 tuple by byte permutes (bytes S .. S + 3 of the dword pair), the O = 0
  // tuple by byte aligns: the same values, which the compiler would otherwise compute
  // once and then copy into the second tuple
  constexpr uint32_t sel = (uint32_t)S | (uint32_t)(S + 1) << 8 | (uint32_t)(S + 2) << 16 |
                           (uint32_t)(S + 3) << 24;
  v8i r;
#pragma unroll
  for (int k = 0; k < 6; ++k)
    r[k] = S == 0 ? w[k + O]
           : O == 0 ? (int32_t)__builtin_amdgcn_alignbyte((uint32_t)w[k + 1], (uint32_t)w[k], (uint32_t)S)
                    : (int32_t)__builtin_amdgcn_perm((uint32_t)w[k + 2], (uint32_t)w[k + 1], sel);
  r[6] = 0;
  r[7] = 0;
  return r;
}

// The products of blocks S, S + 4, S + 8, S + 12.
template <int S>
__device__ __forceinline__ void mfma4(v4i (&acc)[kNT], const v4i &mk, const v8i &w,
                                      const v8i &w1) {
  const v8i e = S == 0 ? w : shifted<S, 0>(w);
  const v8i o = S == 0 ? w1 : shifted<S, 1>(w);
  acc[S] = __builtin_amdgcn_mfma_i32_16x16x64_i8(mk, __builtin_shufflevector(e, e, 0, 1, 2, 3),
                                                 acc[S], 0, 0, 0);
  acc[S + 4] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
      mk, __builtin_shufflevector(o, o, 0, 1, 2, 3), acc[S + 4], 0, 0, 0);
  acc[S + 8] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
      mk, __builtin_shufflevector(e, e, 2, 3, 4, 5), acc[S + 8], 0, 0, 0);
  acc[S + 12] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
      mk, __builtin_shufflevector(o, o, 2, 3, 4, 5), acc[S + 12], 0, 0, 0);
}

// The products of DM tile tw over outputs T0 .. T0 + NWT * 256 - 1 (wave (wd, wt):
// trials 16 wd .. 16 wd + 15 of the tile, outputs T0 + 256 wt + ...; lane l, element r
// of block b: trial row 4 (l / 16) + r, output 16 (l mod 16) + b).  Ends with a
// workgroup barrier, after which the LDS is free.
template <int NWD, int NWT, int WG, typename MA>
__device__ __forceinline__ TileAcc<kNT> mfma_tile(MA &a, int tw, int64_t T0, const uint8_t *xb,
                                                  unsigned char *lds) {
  constexpr int NW = NWD * NWT;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wd = wave % NWD, wt = wave / NWD;
  v4i acc[kNT];
#pragma unroll
  for (int b = 0; b < kNT; ++b) acc[b] = (v4i){0, 0, 0, 0};

  const int gb = ldc(a.group_begin, tw), ge = ldc(a.group_begin, tw + 1);
  // copies the K-block records of group g into LDS (buffer-to-LDS loads, 16 bytes a
  // lane; waited for with the window loads before the group's barrier)
  auto stage_recs = [&](int g, unsigned char *buf) {
    const int kf = ldc(&a.groups[g].kb_first, 0), nkb = ldc(&a.groups[g].nkb, 0);
    const int ro = ldc(&a.groups[g].rec_off, 0);
    const int nch = nkb * (kRecBytes / 16);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(a.recs + (int64_t)kf * kRecBytes), (short)0, nkb * kRecBytes, kBufWord3);
    for (int c0 = 64 * wave; c0 < nch; c0 += 64 * NW) {
      const int ch = c0 + lane;
      if (ch < nch)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void *)(buf + ro + 16 * c0), 16, 16 * ch,
                                                 0, 0, 0);
    }
  };
  // staging: thread t takes chunk t of the group
  uint32_t raw[8];
  int sh = 0, dst = 0, cs = 0;
  bool has = false;
  auto fetch = [&](int g) {
    const int ub = ldc(&a.groups[g].unit_begin, 0), nu = ldc(&a.groups[g].nunits, 0);
    has = tid < nu;
    if (has) {
      const MUnit u = a.units[ub + tid];
      load_raw(xb + (int64_t)u.c * a.in_stride, a.nsamp, T0 + u.src, raw, &sh);
      dst = u.dst;
      cs = u.cs;
    }
  };
  auto store = [&](unsigned char *buf) {
    if (has) store_chunk(buf, dst, cs, raw, sh);
  };
  stage_recs(gb, lds);
  fetch(gb);
  store(lds);
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();
  // the lane's byte offset within a segment's aligned bytes
  const int loff = 16 * (lane & 15) + kTWV * wt;
  for (int g = gb; g < ge; ++g) {
    const int par = (g - gb) & 1;
    unsigned char *buf = lds + par * a.bufbytes;
    if (g + 1 < ge) {
      stage_recs(g + 1, lds + (par ^ 1) * a.bufbytes);
      fetch(g + 1);
    }
    const int kbase = ldc(&a.groups[g].kb_base, 0), kf = ldc(&a.groups[g].kb_first, 0);
    const int ro = ldc(&a.groups[g].rec_off, 0);
    const int k0 = ldc(a.kbr, (int64_t)kbase + wd), k1 = ldc(a.kbr, (int64_t)kbase + wd + 1);
    const unsigned char *rb = buf + ro + (int64_t)(k0 - kf) * kRecBytes;
    // K blocks in pairs through two register sets, each block's mask and samples read
    // while the other block's products run (no copies between the sets)
    auto load = [&](const unsigned char *r, uint32_t &m, v8i &w, int32_t &a1) {
      m = *(const uint16_t *)(r + 2 * lane);
      const int32_t ad = *(const int32_t *)(r + 128 + 4 * (lane >> 4)) + loff;
      a1 = *(const int32_t *)(r + 144 + 4 * (lane >> 4)) + loff;
      w = *(const v8i *)(buf + ad);   // one 8-register tuple (two 16-byte reads)
    };
    auto products = [&](uint32_t m16, const v8i &W, int32_t a1) {
      // the same bytes from 4 bytes on (dwords 1 .. 6), read in place of copies into
      // even-aligned registers for the unshifted blocks at odd dword offsets, which go last
      const v4i lo = *(const v4i *)(buf + a1);
      const v2i hi = *(const v2i *)(buf + a1 + 16);
      // 16 mask bytes of lane (trial row lane % 16, segment lane / 16): bit j -> byte j
      v4i mk;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        mk[k] = (int32_t)((((m16 >> (4 * k)) & 15u) * 0x204081u) & 0x01010101u);
      // Block b = 4 q + s takes bytes b .. b + 15 of the lane's 32: dwords q .. q + 3 of
      // the lane's bytes shifted down by s
      mfma4<1>(acc, mk, W, W);
      mfma4<2>(acc, mk, W, W);
      mfma4<3>(acc, mk, W, W);
      const v8i W1 = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], 0, 0};
      mfma4<0>(acc, mk, W, W1);
    };
    uint32_t ma = 0, mb = 0;
    int32_t aa = 0, ab = 0;
    v8i wa = {0, 0, 0, 0, 0, 0, 0, 0}, wb = {0, 0, 0, 0, 0, 0, 0, 0};
    int kb = k0;
    // while its products run, this wave is issued ahead of waves in their staging stores or
    // boxcar stage (of the CU's other workgroup, or of this one)
    __builtin_amdgcn_s_setprio(1);
    if (kb < k1) load(rb, ma, wa, aa);
    for (; kb + 1 < k1; kb += 2) {
      load(rb + kRecBytes, mb, wb, ab);
      products(ma, wa, aa);
      if (kb + 2 < k1) load(rb + 2 * kRecBytes, ma, wa, aa);
      products(mb, wb, ab);
      rb += 2 * kRecBytes;
    }
    if (kb < k1) products(ma, wa, aa);
    __builtin_amdgcn_s_setprio(0);
    if (g + 1 < ge) store(lds + (par ^ 1) * a.bufbytes);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
  }
  TileAcc<kNT> r;
#pragma unroll
  for (int b = 0; b < kNT; ++b) r.v[b] = acc[b];
  return r;
}

// WG workgroups per CU (their LDS), so WG NW / 4 waves per SIMD: registers up to 512 /
// that.
template <int NWD, int NWT, int WG>
__global__ void __launch_bounds__(64 * NWD * NWT)
__attribute__((amdgpu_waves_per_eu(WG * NWD * NWT / 4, WG * NWD * NWT / 4)))
k_dedisp_mfma(MfmaArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  constexpr int TW = NWT * kTWV;
  int tt, tw;
  tile_of_block(a.ntw, a.ntt, &tt, &tw);
  const int bb = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wd = wave % NWD, wt = wave / NWD;
  const int64_t T0 = (int64_t)tt * TW;
  const TileAcc<kNT> acc =
      mfma_tile<NWD, NWT, WG>(a, tw, T0, a.x + (int64_t)bb * a.in_bstride, lds);
  // Lane l holds, for trial rows 4 (l / 16) + r, the 16 outputs from 16 (l mod 16): the
  // rows go out through LDS (free after the tile's last barrier; each wave has its own
  // 8 rows), so that each store instruction writes 256 consecutive bytes of a row.
  // Swapping the upper lanes of blocks b < 8 with the lower lanes of blocks b + 8 first
  // gives every lane, in pass p, trial row 8 p + 4 ((l / 16) mod 2) + r at outputs
  // 16 (l mod 16) + 8 (l / 32) + b, b < 8.
  constexpr int OROW = kTWV + 4;
  static_assert(NWD * NWT * 8 * OROW * 4 <= 2 * (kMfmaBufBytes / WG), "output rows fit the LDS");
  int *R = (int *)lds + wave * 8 * OROW;
  v4i ps[2][kNT / 2];
#pragma unroll
  for (int b = 0; b < kNT / 2; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const auto p = __builtin_amdgcn_permlane32_swap(acc.v[b][r], acc.v[b + kNT / 2][r], false,
                                                      false);
      ps[0][b][r] = (int32_t)p[0];
      ps[1][b][r] = (int32_t)p[1];
    }
  int32_t *ob = a.out + (int64_t)bb * a.out_bstride;
  const int64_t t0 = T0 + (int64_t)kTWV * wt;
  const int col = 16 * (lane & 15) + 8 * (lane >> 5);
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int *row = R + (4 * ((lane >> 4) & 1) + r) * OROW + col;
      *(v4i *)row = (v4i){ps[pass][0][r], ps[pass][1][r], ps[pass][2][r], ps[pass][3][r]};
      *(v4i *)(row + 4) = (v4i){ps[pass][4][r], ps[pass][5][r], ps[pass][6][r], ps[pass][7][r]};
    }
    // LDS operations of one wave complete in order: the reads below see the writes
    __builtin_amdgcn_wave_barrier();
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
      const int d = a.perm[tw * 16 * NWD + 16 * wd + 8 * pass + k];
      if (d < 0) continue;
      const int32_t corr = 128 * a.ntot[d];
      int32_t *o = ob + (int64_t)d * a.out_stride + t0;
#pragma unroll
      for (int j = 0; j < kTWV / 64; ++j)
        if (t0 + lane + 64 * j < a.nout) o[lane + 64 * j] = R[k * OROW + lane + 64 * j] + corr;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

struct MfmaSearchArgs {
  MfmaArgs m;             // x, tables, ntw, ntt (out and batch strides unused)
  const double *M, *S;    // noise tables [ndm][nw]
  int32_t nw;
  uint32_t wmask;         // bit W - 1 for every listed width W <= 32
  CandRec *part;          // [ndm][ntt]
};

// Time-tile step of the search: the tile's 64 SP outputs less a halo of >= 31 outputs,
// in whole lanes of SP starts (as the boxcar stage needs).
constexpr int search_step(int sp) { return 64 * sp - ((32 + sp - 1) / sp) * sp; }

// Fused search: the products of one tile (outputs T0 .. T0 + TW - 1, T0 = tt * TT),
// then the boxcar search of every trial of the tile over starts T0 .. T0 + TT - 1.
// The series go through LDS in two passes (trial rows 0-7, then 8-15 of every wave),
// as rows of TW + 36 ints; each wave searches whole rows.
template <int NWD, int NWT, int WG, typename SA>
__device__ __forceinline__ void search_tile_mfma(SA &sa, int tt, int tw, unsigned char *lds) {
  constexpr int NW = NWD * NWT, TW = NWT * kTWV, SP = TW / 64;
  constexpr int TT = search_step(SP), YROW = TW + kHalo + 4;
  constexpr int PT = 8;                    // trials of one wave in one pass
  constexpr int ROWS = PT * NWD;           // rows of one pass
  static_assert(TW % 64 == 0 && TT % SP == 0 && TW - TT >= 31, "search tile");
  static_assert(ROWS % NW == 0, "whole rows per wave");
  static_assert(ROWS * YROW * 4 <= 2 * (kMfmaBufBytes / WG), "rows of one pass fit the LDS");
  static_assert(YROW % 4 == 0, "16-byte aligned rows");
  auto &a = sa.m;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wd = wave % NWD, wt = wave / NWD;
  const int64_t T0 = (int64_t)tt * TT;
  const TileAcc<kNT> acc = mfma_tile<NWD, NWT, WG>(a, tw, T0, a.x, lds);
  constexpr int DT = 16 * NWD;
  int *Y = (int *)lds;
  // A lane's 4 trial rows (4 (l / 16) + r) are those of one pass: lanes 0-31 hold the
  // first pass's trials, lanes 32-63 the second's.  Swapping the upper lanes of blocks
  // b < 8 with the lower lanes of blocks b + 8 puts each pass's values into 8
  // registers (b) per row of every lane, so the second pass's values take 32
  // registers (not 64) during the first pass's search, and each pass writes its rows
  // with all lanes.  After the swap, register (b, r) of pass p holds, in lane l, trial
  // row 4 ((l / 16) mod 2) + r of the pass, output 16 (l mod 16) + 8 (l / 32) + b of
  // the wave's run.
  v4i ps[2][kNT / 2];
#pragma unroll
  for (int b = 0; b < kNT / 2; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const auto p = __builtin_amdgcn_permlane32_swap(acc.v[b][r], acc.v[b + kNT / 2][r], false,
                                                      false);
      ps[0][b][r] = (int32_t)p[0];
      ps[1][b][r] = (int32_t)p[1];
    }
  const int col = kTWV * wt + 16 * (lane & 15) + 8 * (lane >> 5);
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * ((lane >> 4) & 1) + r;   // trial row within the pass
      const int d = a.perm[tw * DT + 16 * wd + PT * pass + k];
      const int32_t corr = d >= 0 ? 128 * a.ntot[d] : 0;
      int *row = Y + (PT * wd + k) * YROW + col;
      *(v4i *)row = (v4i){ps[pass][0][r] + corr, ps[pass][1][r] + corr, ps[pass][2][r] + corr,
                          ps[pass][3][r] + corr};
      *(v4i *)(row + 4) = (v4i){ps[pass][4][r] + corr, ps[pass][5][r] + corr,
                                ps[pass][6][r] + corr, ps[pass][7][r] + corr};
    }
    __syncthreads();
    // one row at a time, not unrolled: the search code then stays small enough
    // for the instruction cache
#pragma unroll 1
    for (int k = 0; k < ROWS / NW; ++k) {
      const int rw = wave * (ROWS / NW) + k;
      const int sw = rw / PT, j = rw % PT;   // DM sub-tile, trial row within the pass
      const int dg = a.perm[tw * DT + 16 * sw + PT * pass + j];
      const CandRec rec =
          boxcar_row<SP>(Y + rw * YROW, lane, T0, TT, a.nout, dg, sa.wmask, sa.nw, sa.M, sa.S);
      if (dg >= 0 && lane == 0) sa.part[(int64_t)dg * a.ntt + tt] = rec;
    }
    __syncthreads();
  }
}

template <int NWD, int NWT, int WG>
__global__ void __launch_bounds__(64 * NWD * NWT)
__attribute__((amdgpu_waves_per_eu(WG * NWD * NWT / 4, WG * NWD * NWT / 4)))
k_search_mfma(MfmaSearchArgs sa) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  int tt, tw;
  tile_of_block(sa.m.ntw, sa.m.ntt, &tt, &tw);
  search_tile_mfma<NWD, NWT, WG>(sa, tt, tw, lds);
}

// Multi-beam fused search: one workgroup per (beam, tile).  Beam b owns the blocks
// [base[b], base[b] + its tile count rounded up to 8), base[b] a multiple of 8, so that
// block i of a beam runs on XCD i mod 8 and the beam's tiles take the one-beam
// kernel's XCD-aware order.  Blocks past a beam's tile count exit at once (the whole
// workgroup, before any barrier).
template <int NWD, int NWT, int WG>
__global__ void __launch_bounds__(64 * NWD * NWT)
__attribute__((amdgpu_waves_per_eu(WG * NWD * NWT / 4, WG * NWD * NWT / 4)))
k_search_mfma_batch(const MfmaSearchArgs *__restrict__ beams, const int32_t *__restrict__ base,
                    int32_t nbeam) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const int bi = blockIdx.x;
  int lo = 0, hi = nbeam - 1;   // last beam whose first block <= bi
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ldc(base, mid) <= bi) lo = mid; else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  // the argument table is read through the constant address space (scalar loads)
  typedef const __attribute__((address_space(4))) MfmaSearchArgs CArgs;
  CArgs &sa = ((CArgs *)beams)[lo];
  const int nb = sa.m.ntw * sa.m.ntt;
  const int kl = bi - ldc(base, lo);
  const int xcd = kl & 7, k = kl >> 3, q = nb >> 3, rem = nb & 7;
  if (k >= q + (xcd < rem ? 1 : 0)) return;
  const int L = xcd * q + min(xcd, rem) + k;
  const int tt = L / sa.m.ntw, tw = L - tt * sa.m.ntw;
  search_tile_mfma<NWD, NWT, WG>(sa, tt, tw, lds);
}

}  // namespace

// ---- host ----------------------------------------------------------------------
template <typename T>
static hipError_t upload(T **dst, const std::vector<T> &v) {
  if (v.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void **)dst, sizeof(T) * v.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

// Tables of configuration ci: trial order, per DM tile the channel groups with their
// staging units, and per (group, wave) the K blocks (masks and lane addresses).
static bool build_mfma_cfg(const dedisp_plan_s *p, int ci, MfmaCfgTables &out) {
  const MfmaCfg cf = kMfmaCfgs[ci];
  const int C = p->nchan, D = p->ndm;
  const int NWD = cf.nwd, NW = cf.nwd * cf.nwt, TW = cf.nwt * kTWV, DT = 16 * NWD;
  const int BUF = kMfmaBufBytes / cf.wg;
  const int maxunits = 64 * NW;
  out = MfmaCfgTables();
  out.tw = TW;
  out.trials = DT;
  out.bufbytes = BUF;
  std::vector<int32_t> order(D);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return p->dm[x] < p->dm[y]; });
  const int ntw = (D + DT - 1) / DT;
  out.ntw = ntw;
  out.perm.assign((size_t)ntw * DT, -1);
  for (int i = 0; i < D; ++i) out.perm[i] = order[i];
  out.ntot.assign(D, 0);
  for (int d = 0; d < D; ++d) {
    int64_t s = 0;
    for (int c = 0; c < C; ++c) s += p->ntap[(size_t)d * C + c];
    if (s > (INT32_MAX - 1) / 256) return false;
    out.ntot[d] = (int32_t)s;
  }
  out.group_begin.assign(ntw + 1, 0);
  // per (sub-tile, channel): first segment (window-relative, a multiple of 4) and count
  std::vector<int32_t> so(NWD * C), nseg(NWD * C);
  // per channel: window origin (absolute delay of window byte 0) and copy length
  std::vector<int32_t> wlo(C), clen(C);
  for (int tw = 0; tw < ntw; ++tw) {
    out.group_begin[tw] = (int)out.groups.size();
    for (int c = 0; c < C; ++c) {
      int l[64], h[64];
      int slo = INT32_MAX;
      for (int w = 0; w < NWD; ++w) {
        l[w] = INT32_MAX;
        h[w] = INT32_MIN;
        for (int m = 0; m < 16; ++m) {
          const int d = out.perm[(size_t)tw * DT + 16 * w + m];
          if (d < 0 || p->ntap[(size_t)d * C + c] == 0) continue;
          l[w] = std::min(l[w], p->start[(size_t)d * C + c]);
          h[w] = std::max(h[w], p->start[(size_t)d * C + c] + p->ntap[(size_t)d * C + c]);
        }
        slo = std::min(slo, l[w]);
      }
      clen[c] = 0;
      if (slo == INT32_MAX) {
        for (int w = 0; w < NWD; ++w) nseg[w * C + c] = 0;
        continue;
      }
      wlo[c] = slo;
      int qmax = 0;
      for (int w = 0; w < NWD; ++w) {
        if (l[w] == INT32_MAX) {
          nseg[w * C + c] = 0;
          continue;
        }
        const int o = (l[w] - slo) / 4 * 4;   // on the 4-byte grid, at or below the band
        so[w * C + c] = o;
        nseg[w * C + c] = (h[w] - (slo + o) + 15) / 16;
        qmax = std::max(qmax, (o + 16 * (nseg[w * C + c] - 1)) / 16);
      }
      // lane n of time wave wt reads chunks q + n + 16 wt and q + n + 1 + 16 wt, and 24
      // bytes from 4 bytes further on (up to chunk q + n + 2 + 16 wt)
      clen[c] = 16 * (qmax + 16 * cf.nwt + 2);
      if ((int64_t)kCopies * clen[c] + kRecBytes > BUF || clen[c] / 16 > maxunits) return false;
    }
    int c = 0;
    while (c < C) {
      // channels of the group: windows and K-block records within the LDS buffer
      int used = 0;
      const int cbeg = c;
      std::vector<int> segw(NWD, 0);
      int nunits = 0;
      while (c < C && nunits + clen[c] / 16 <= maxunits) {
        int nrec = 0;   // K-block records with channel c added
        for (int w = 0; w < NWD; ++w) nrec += (segw[w] + nseg[w * C + c] + 3) / 4;
        if ((int64_t)used + (int64_t)kCopies * clen[c] + (int64_t)nrec * kRecBytes > BUF) break;
        for (int w = 0; w < NWD; ++w) segw[w] += nseg[w * C + c];
        used += kCopies * clen[c];
        nunits += clen[c] / 16;
        ++c;
      }
      if (c == cbeg) return false;   // one channel does not fit
      MGroup gi{};
      gi.unit_begin = (int)out.units.size();
      std::vector<int32_t> region(C, 0);
      int off = 0;
      for (int cc = cbeg; cc < c; ++cc) {
        if (!clen[cc]) continue;
        region[cc] = off;
        for (int k = 0; k < clen[cc] / 16; ++k)
          out.units.push_back(MUnit{cc, wlo[cc] + 16 * k, off + 16 * k, clen[cc]});
        off += kCopies * clen[cc];
      }
      gi.nunits = (int)out.units.size() - gi.unit_begin;
      gi.kb_base = (int)out.kbr.size();
      gi.kb_first = (int)(out.recs.size() / kRecBytes);
      gi.rec_off = off;
      for (int w = 0; w < NWD; ++w) {
        out.kbr.push_back((int32_t)(out.recs.size() / kRecBytes));
        // segments of this sub-tile in the group (channel, window-relative start), four
        // per K block
        std::vector<std::pair<int, int>> segs;
        for (int cc = cbeg; cc < c; ++cc)
          for (int sg = 0; sg < nseg[w * C + cc]; ++sg) segs.push_back({cc, so[w * C + cc] + 16 * sg});
        for (size_t s0 = 0; s0 < segs.size(); s0 += 4) {
          std::vector<uint8_t> rec(kRecBytes, 0);
          for (int g = 0; g < 4; ++g) {
            // padding segments: zero masks, a valid address
            const size_t si = s0 + g < segs.size() ? s0 + g : s0;
            const int cc = segs[si].first, o = segs[si].second;
            // copy (o / 4) mod 4 holds window byte o at offset 16 (o / 16); the second
            // address is that of byte o + 4
            const int32_t ad = region[cc] + ((o >> 2) & 3) * clen[cc] + 16 * (o >> 4);
            const int32_t ad1 =
                region[cc] + (((o + 4) >> 2) & 3) * clen[cc] + 16 * ((o + 4) >> 4);
            std::memcpy(rec.data() + 128 + 4 * g, &ad, 4);
            std::memcpy(rec.data() + 144 + 4 * g, &ad1, 4);
            if (s0 + g >= segs.size()) continue;
            const int oa = wlo[cc] + o;   // absolute delay of the segment's first byte
            for (int m = 0; m < 16; ++m) {
              const int d = out.perm[(size_t)tw * DT + 16 * w + m];
              if (d < 0) continue;
              const int st = p->start[(size_t)d * C + cc], nt = p->ntap[(size_t)d * C + cc];
              uint16_t bits = 0;
              for (int j = 0; j < 16; ++j)
                if (oa + j >= st && oa + j < st + nt) bits |= (uint16_t)(1u << j);
              std::memcpy(rec.data() + 2 * (16 * g + m), &bits, 2);
            }
          }
          out.recs.insert(out.recs.end(), rec.begin(), rec.end());
        }
      }
      out.kbr.push_back((int32_t)(out.recs.size() / kRecBytes));
      gi.nkb = (int)(out.recs.size() / kRecBytes) - gi.kb_first;
      out.groups.push_back(gi);
    }
  }
  out.group_begin[ntw] = (int)out.groups.size();
  out.ok = !out.groups.empty();
  return out.ok;
}

static hipError_t allow_lds_mfma(const void *fn, bool *done, std::mutex *mu, int bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= 64) return e;
  std::lock_guard<std::mutex> lk(*mu);
  if (!done[dev]) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) done[dev] = true;
  }
  return e;
}

template <int NWD, int NWT, int WG>
static hipError_t launch_mfma_cfg(const MfmaArgs &a, int nbatch, hipStream_t s) {
  static bool done[64] = {};
  static std::mutex mu;
  hipError_t e = allow_lds_mfma((const void *)k_dedisp_mfma<NWD, NWT, WG>, done, &mu,
                                2 * (kMfmaBufBytes / WG));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_dedisp_mfma<NWD, NWT, WG>), dim3(a.ntw * a.ntt, nbatch),
                     dim3(64 * NWD * NWT), 2 * a.bufbytes, s, a);
  return hipGetLastError();
}

static hipError_t launch_mfma(int ci, const MfmaArgs &a, int nbatch, hipStream_t s) {
  switch (ci) {
#define DD_MFMA_CASE(i, x, y, g) \
  case i: return launch_mfma_cfg<x, y, g>(a, nbatch, s);
    DD_MFMA_CONFIGS(DD_MFMA_CASE)
#undef DD_MFMA_CASE
    default: return hipErrorInvalidValue;
  }
}

// Tables of configuration k, built and uploaded on first use (nullptr if the plan
// does not fit it).  Caller holds p->mu.
static dedisp_status ensure_mfma(dedisp_plan p, int k, MfmaCfgTables **out) {
  *out = nullptr;
  if (!p->mfma) {
    p->mfma = new (std::nothrow) MfmaTables;
    if (!p->mfma) return fail(DEDISP_ERR_OOM, "host allocation failed");
  }
  MfmaCfgTables &c = p->mfma->cfg[k];
  if (!p->mfma->tried[k]) {
    p->mfma->tried[k] = true;
    if (build_mfma_cfg(p, k, c)) {
      DD_HIP(upload(&c.d_perm, c.perm));
      DD_HIP(upload(&c.d_ntot, c.ntot));
      DD_HIP(upload(&c.d_group_begin, c.group_begin));
      DD_HIP(upload(&c.d_kbr, c.kbr));
      DD_HIP(upload(&c.d_groups, c.groups));
      DD_HIP(upload(&c.d_units, c.units));
      DD_HIP(upload(&c.d_recs, c.recs));
    }
  }
  if (c.ok) *out = &c;
  return DEDISP_OK;
}

static void fill_args(dedisp_plan p, const MfmaCfgTables &c, const uint8_t *x, int64_t nsamp,
                      int64_t in_stride, int64_t nout, MfmaArgs &a) {
  a = MfmaArgs{};
  a.x = x;
  a.in_stride = in_stride;
  a.nsamp = nsamp;
  a.ntw = c.ntw;
  a.bufbytes = c.bufbytes;
  a.group_begin = c.d_group_begin;
  a.kbr = c.d_kbr;
  a.perm = c.d_perm;
  a.ntot = c.d_ntot;
  a.groups = c.d_groups;
  a.units = c.d_units;
  a.recs = c.d_recs;
  a.nout = nout;
  (void)p;
}

dedisp_status run_dedisperse_u8_mfma(dedisp_plan p, const uint8_t *x, int64_t nsamp,
                                     int64_t in_stride, int64_t in_bstride, int32_t nbatch,
                                     int32_t *out, int64_t out_stride, int64_t out_bstride,
                                     int64_t nout, hipStream_t s, KernelTimer *kt) {
  if (p->wmode != DEDISP_W_UNIT || nbatch > 65535) return DEDISP_ERR_UNSUPPORTED;
  // the first shape that takes the plan
  int ci = -1;
  MfmaCfgTables *cfg = nullptr;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    for (int k = 0; k < kNumMfmaCfgs && !cfg; ++k) {
      dedisp_status st = ensure_mfma(p, k, &cfg);
      if (st != DEDISP_OK) return st;
      ci = k;
    }
  }
  if (!cfg) return DEDISP_ERR_UNSUPPORTED;
  const int64_t ntt = (nout + cfg->tw - 1) / cfg->tw;
  if (ntt * cfg->ntw > INT32_MAX / 2) return DEDISP_ERR_UNSUPPORTED;
  MfmaArgs a;
  fill_args(p, *cfg, x, nsamp, in_stride, nout, a);
  a.in_bstride = in_bstride;
  a.ntt = (int32_t)ntt;
  a.out = out;
  a.out_stride = out_stride;
  a.out_bstride = out_bstride;
  hipError_t e = kt ? kt->begin() : hipSuccess;
  if (e == hipSuccess) e = launch_mfma(ci, a, nbatch, s);
  if (e == hipSuccess && kt) e = kt->end();
  if (e != hipSuccess) return hip_fail(e, "mfma dedisperse launch");
  return DEDISP_OK;
}

// ---- fused search ----------------------------------------------------------------
struct MfmaSearchLayout {
  int64_t ntt = 0;
  size_t off_part = 0, total = 0;
};

static MfmaSearchLayout search_layout(const dedisp_plan_s *p, int k, int32_t nw, int64_t nout) {
  const MfmaCfg cf = kMfmaCfgs[k];
  const int tw = cf.nwt * kTWV, tstep = search_step(tw / 64);
  MfmaSearchLayout L;
  L.ntt = (nout + tstep - 1) / tstep;
  L.off_part = (2 * sizeof(double) * (size_t)p->ndm * nw + 255) & ~(size_t)255;
  L.total = L.off_part + ((sizeof(CandRec) * (size_t)p->ndm * L.ntt + 255) & ~(size_t)255);
  return L;
}

size_t mfma_search_work_bytes(const dedisp_plan_s *p, int32_t nw, int64_t nout) {
  size_t b = 0;
  for (int k = 0; k < kNumMfmaCfgs; ++k) b = std::max(b, search_layout(p, k, nw, nout).total);
  return b;
}

int mfma_search_count() { return kNumMfmaCfgs; }

template <int NWD, int NWT, int WG>
static hipError_t launch_search_cfg(const MfmaSearchArgs &sa, hipStream_t s) {
  static bool done[64] = {};
  static std::mutex mu;
  hipError_t e = allow_lds_mfma((const void *)k_search_mfma<NWD, NWT, WG>, done, &mu,
                                2 * (kMfmaBufBytes / WG));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_search_mfma<NWD, NWT, WG>), dim3(sa.m.ntw * sa.m.ntt),
                     dim3(64 * NWD * NWT), 2 * sa.m.bufbytes, s, sa);
  return hipGetLastError();
}

static hipError_t launch_search_mfma(int k, const MfmaSearchArgs &sa, hipStream_t s) {
  switch (k) {
#define DD_MFMA_SEARCH_CASE(i, x, y, g) \
  case i: return launch_search_cfg<x, y, g>(sa, s);
    DD_MFMA_CONFIGS(DD_MFMA_SEARCH_CASE)
#undef DD_MFMA_SEARCH_CASE
    default: return hipErrorInvalidValue;
  }
}

dedisp_status run_search_mfma(dedisp_plan p, int k, const uint8_t *x, int64_t nsamp,
                              int64_t in_stride, int64_t nout, const WidthList &wl,
                              const double *mu, const double *sigma, double *snr, int32_t *t,
                              int32_t *w, void *work, hipStream_t s) {
  if (k < 0 || k >= kNumMfmaCfgs || p->wmode != DEDISP_W_UNIT || wl.w[wl.n - 1] > 32)
    return DEDISP_ERR_UNSUPPORTED;
  MfmaCfgTables *cfg = nullptr;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    dedisp_status st = ensure_mfma(p, k, &cfg);
    if (st != DEDISP_OK) return st;
  }
  if (!cfg) return DEDISP_ERR_UNSUPPORTED;
  const MfmaSearchLayout L = search_layout(p, k, wl.n, nout);
  if (L.ntt * cfg->ntw > INT32_MAX / 2) return DEDISP_ERR_UNSUPPORTED;
  MfmaSearchArgs sa{};
  fill_args(p, *cfg, x, nsamp, in_stride, nout, sa.m);
  sa.m.ntt = (int32_t)L.ntt;
  double *M = (double *)work;
  sa.M = M;
  sa.S = M + (size_t)p->ndm * wl.n;
  sa.nw = wl.n;
  sa.wmask = 0;
  for (int i = 0; i < wl.n; ++i) sa.wmask |= 1u << (wl.w[i] - 1);
  sa.part = (CandRec *)((char *)work + L.off_part);
  DD_HIP(launch_norm(p, wl, mu, sigma, M, (double *)sa.S, s));
  KernelTimer kt(p, s);
  DD_HIP(kt.begin());
  DD_HIP(launch_search_mfma(k, sa, s));
  DD_HIP(kt.end());
  DD_HIP(launch_reduce(p->ndm, (int32_t)L.ntt, sa.part, snr, t, w, s));
  return DEDISP_OK;
}

// ---- multi-beam fused search -------------------------------------------------------
struct MfmaBatch {
  int k = 0;                                // matrix-core shape
  int nbeam = 0;
  std::vector<dedisp_plan> plans;
  std::vector<int64_t> nsamp, nout;
  std::vector<size_t> off;                  // workspace offset of each beam
  std::vector<MfmaSearchLayout> lay;
  std::vector<int32_t> base;                // first block of each beam, then the total
  WidthList wl{};
  size_t work_bytes = 0;
  size_t args_off = 0;                      // workspace offset of the eager argument table
  int32_t *d_base = nullptr;
  MfmaSearchArgs *d_args_graph = nullptr;   // argument table of the captured graph
  std::vector<MfmaSearchArgs> args;         // argument table of the last enqueue
  ArgStage stage;                           // pinned staging of the eager table
};

void mfma_batch_free(MfmaBatch *B) {
  if (!B) return;
  B->stage.release();
  (void)hipFree(B->d_base);
  (void)hipFree(B->d_args_graph);
  delete B;
}

size_t mfma_batch_work_bytes(const MfmaBatch *B) { return B->work_bytes; }

dedisp_status mfma_batch_create(const std::vector<dedisp_plan> &plans,
                                const std::vector<int64_t> &nsamp, const WidthList &wl, int prefer,
                                MfmaBatch **out) {
  *out = nullptr;
  if (wl.w[wl.n - 1] > 32) return DEDISP_OK;
  // the preferred shape, else the first that takes every beam
  std::vector<int> order;
  if (prefer >= 0 && prefer < kNumMfmaCfgs) order.push_back(prefer);
  for (int k = 0; k < kNumMfmaCfgs; ++k)
    if (k != prefer) order.push_back(k);
  int chosen = -1;
  for (int k : order) {
    bool all = true;
    for (dedisp_plan p : plans) {
      if (p->wmode != DEDISP_W_UNIT) return DEDISP_OK;
      MfmaCfgTables *cfg = nullptr;
      std::lock_guard<std::mutex> lk(p->mu);
      dedisp_status st = ensure_mfma(p, k, &cfg);
      if (st != DEDISP_OK) return st;
      if (!cfg) {
        all = false;
        break;
      }
    }
    if (all) {
      chosen = k;
      break;
    }
  }
  if (chosen < 0) return DEDISP_OK;
  MfmaBatch *B = new (std::nothrow) MfmaBatch;
  if (!B) return fail(DEDISP_ERR_OOM, "host allocation failed");
  B->k = chosen;
  B->nbeam = (int)plans.size();
  B->plans = plans;
  B->nsamp = nsamp;
  B->wl = wl;
  size_t off = 0;
  int64_t blocks = 0;
  for (int b = 0; b < B->nbeam; ++b) {
    dedisp_plan p = plans[b];
    const int64_t no = nsamp[b] - p->max_span + 1;
    B->nout.push_back(no);
    const MfmaSearchLayout L = search_layout(p, chosen, wl.n, no);
    B->lay.push_back(L);
    B->off.push_back(off);
    off += (L.total + 255) & ~(size_t)255;
    B->base.push_back((int32_t)blocks);
    const int64_t nb = ((int64_t)p->mfma->cfg[chosen].ntw * L.ntt + 7) & ~(int64_t)7;
    blocks += nb;
    if (blocks > INT32_MAX / 2) {
      mfma_batch_free(B);
      return DEDISP_OK;   // too many tiles for one launch: not this path
    }
  }
  B->base.push_back((int32_t)blocks);
  B->args_off = off;
  B->work_bytes = off + sizeof(MfmaSearchArgs) * B->nbeam;
  hipError_t e = upload(&B->d_base, B->base);
  if (e == hipSuccess)
    e = hipMalloc((void **)&B->d_args_graph, sizeof(MfmaSearchArgs) * B->nbeam);
  if (e != hipSuccess) {
    mfma_batch_free(B);
    return hip_fail(e, "batch setup");
  }
  *out = B;
  return DEDISP_OK;
}

template <int NWD, int NWT, int WG>
static hipError_t launch_batch_mfma_cfg(const MfmaBatch *B, const MfmaSearchArgs *table,
                                        hipStream_t s) {
  static bool done[64] = {};
  static std::mutex mu;
  hipError_t e = allow_lds_mfma((const void *)k_search_mfma_batch<NWD, NWT, WG>, done, &mu,
                                2 * (kMfmaBufBytes / WG));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_search_mfma_batch<NWD, NWT, WG>), dim3(B->base.back()),
                     dim3(64 * NWD * NWT), 2 * (kMfmaBufBytes / WG), s, table, B->d_base,
                     B->nbeam);
  return hipGetLastError();
}

static hipError_t launch_batch_mfma(const MfmaBatch *B, const MfmaSearchArgs *table,
                                    hipStream_t s) {
  switch (B->k) {
#define DD_MFMA_BATCH_CASE(i, x, y, g) \
  case i: return launch_batch_mfma_cfg<x, y, g>(B, table, s);
    DD_MFMA_CONFIGS(DD_MFMA_BATCH_CASE)
#undef DD_MFMA_BATCH_CASE
    default: return hipErrorInvalidValue;
  }
}

// Noise tables of every beam, the argument table, one launch over every beam's tiles,
// the per-beam reductions.  Outputs of beam b start at out_off[b].  Eager calls
// (for_graph false) copy the argument table into the caller's workspace through the
// pinned staging buffer; a captured sequence (for_graph true) reads the batch's own
// graph table, which mfma_batch_upload fills once the capture has ended.  The two
// tables are distinct, so eager calls never change what a graph replays.
dedisp_status mfma_batch_enqueue(MfmaBatch *B, const void *const *in, const int64_t *stride,
                                 const double *mu, const double *sigma, double *snr, int32_t *t,
                                 int32_t *w, const std::vector<int64_t> &out_off, void *work,
                                 hipStream_t s, bool for_graph, KernelTimer *kt) {
  B->args.assign(B->nbeam, MfmaSearchArgs{});
  for (int b = 0; b < B->nbeam; ++b) {
    dedisp_plan p = B->plans[b];
    const MfmaCfgTables &c = p->mfma->cfg[B->k];
    MfmaSearchArgs &sa = B->args[b];
    fill_args(p, c, (const uint8_t *)in[b], B->nsamp[b], stride[b], B->nout[b], sa.m);
    sa.m.ntt = (int32_t)B->lay[b].ntt;
    double *M = (double *)((char *)work + B->off[b]);
    sa.M = M;
    sa.S = M + (size_t)p->ndm * B->wl.n;
    sa.nw = B->wl.n;
    sa.wmask = 0;
    for (int i = 0; i < B->wl.n; ++i) sa.wmask |= 1u << (B->wl.w[i] - 1);
    sa.part = (CandRec *)((char *)work + B->off[b] + B->lay[b].off_part);
    DD_HIP(launch_norm(p, B->wl, mu, sigma, M, (double *)sa.S, s));
  }
  MfmaSearchArgs *table = B->d_args_graph;
  if (!for_graph) {
    table = (MfmaSearchArgs *)((char *)work + B->args_off);
    DD_HIP(B->stage.copy(table, B->args.data(), sizeof(MfmaSearchArgs) * B->nbeam, s));
  }
  if (kt) DD_HIP(kt->begin());
  DD_HIP(launch_batch_mfma(B, table, s));
  if (kt) DD_HIP(kt->end());
  for (int b = 0; b < B->nbeam; ++b) {
    const int64_t o = out_off[b];
    DD_HIP(launch_reduce(B->plans[b]->ndm, B->args[b].m.ntt, B->args[b].part, snr + o, t + o,
                         w + o, s));
  }
  return DEDISP_OK;
}

dedisp_status mfma_batch_upload(MfmaBatch *B) {
  DD_HIP(hipMemcpy(B->d_args_graph, B->args.data(), sizeof(MfmaSearchArgs) * B->nbeam,
                   hipMemcpyHostToDevice));
  return DEDISP_OK;
}

}  // namespace dd
