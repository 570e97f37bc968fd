// Dedispersion of uint8 data with unit weights (eq. p_dedisp) on the int8 matrix cores.
//
// For a group of 4 trials and a channel c, the samples the trials add lie in a short band
// of delays: trial d takes x[c][t + start[d,c] + k] for k < ntap[d,c].  One
// v_mfma_i32_32x32x32_i8 product takes 32 rows = 4 trials x 8 output phases u and 32
// columns = 32 output octets n, so that row (d, u), column n is output t = T + 8 n + u of
// trial d; its K = 32 are two segments of 16 consecutive samples (of one or two
// channels), segment g starting at window sample o_g + 8 n for column n.  Then
//     y[d][T + 8 n + u] += sum_{g, i<16} mask_g[d, u][i] * x[c_g][T + 8 n + o_g + i],
// where mask_g[d, u][i] = 1 when sample o_g + i - u lies in trial d's run: the 0/1 matrix
// (which samples each (trial, phase) row takes) is the same for every column and every
// product of the K block, and the samples a column needs start on an 8-byte boundary.
// The samples enter as int8 x ^ 0x80 = x - 128, and every trial's result is corrected
// by 128 times its number of samples, so the int32 result is exact.
//
// Each channel's window is staged into LDS as 2 copies shifted by 0 and 8 bytes,
// interleaved by 16-byte chunks (chunk j of copy k at byte 32 j + 16 k of the channel's
// region), so that the 16 window bytes from any multiple of 8, p, sit 16-byte aligned at
// region + 2 p: a lane's operand of product q is one aligned 16-byte read at its
// segment's base + 16 n + 512 q, and the 32 lanes of a segment read 512 consecutive
// bytes (an LDS read of two such halves runs at the full rate whatever their
// alignment to each other; four quarter-wave runs at different alignments run at about
// half of it).  A wave takes 4 trials x NP products of 256 consecutive outputs;
// segments are put on an 8-byte grid (their band covers start .. start + ntap + 7 for
// the phases; a channel's window starts at a multiple of 8 of the delay).  Channel groups
// are staged while the previous group is multiplied (two LDS buffers): in the fused
// search from a converted copy of the block (x ^ 0x80, written by the noise-table launch)
// with buffer-to-LDS loads, 16 bytes a lane, so that piece m of a region (its 16 bytes
// at region + 16 m) is one load of window bytes 8 m .. 8 m + 15; in the dedispersion, the
// multi-beam search and the allocation-free search from x through registers (aligned
// loads, byte shifts, the conversion, two LDS stores).  The host plans, per pair of
// segments (a K block), a 48-byte record: per segment and trial a 32-bit run mask (bit j
// set when window byte o_g - 8 + j lies in the trial's run; phase u takes bits 8 - u ..
// 23 - u), and the LDS base address of each segment; the records of a channel group are
// copied into LDS with the windows, and every lane forms its 16 mask bytes (two 8-byte
// entries of a 2 KB LDS table indexed by mask bytes) and its read address from them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "boxcar_row.h"
#include "internal.h"
#include "norm_reduce.h"

namespace dd {

// Workgroup shapes: NWD waves along DM (4 trials each), NWT along time (256 NP outputs
// each), WG workgroups per CU (each with 1 / WG of the CU's LDS).
// Every shape keeps 16 waves on a CU (128 registers a lane).
#define DD_MFMA_CONFIGS(X) \
  X(0, 16, 1, 4, 1)        \
  X(1, 8, 1, 4, 2)         \
  X(2, 8, 2, 2, 1)         \
  X(3, 16, 1, 2, 1)        \
  X(4, 8, 1, 2, 2)
struct MfmaCfg {
  int nwd, nwt, np, wg;
};
#define DD_MFMA_ENTRY(i, a, b, n, g) {a, b, n, g},
static const MfmaCfg kMfmaCfgs[] = {DD_MFMA_CONFIGS(DD_MFMA_ENTRY)};
#undef DD_MFMA_ENTRY
constexpr int kNumMfmaCfgs = sizeof(kMfmaCfgs) / sizeof(kMfmaCfgs[0]);
constexpr int kTrialsPerWave = 4;           // trials of a wave (x 8 output phases = 32 rows)
constexpr int kPhases = 8;                  // output phases (rows per trial)
constexpr int kOutsPerProduct = 32 * kPhases;
constexpr int kCopies = 2;                  // 8-byte-shifted copies of each staged window
constexpr int kMfmaBufBytes = 78 * 1024;    // LDS per staging buffer (two per workgroup) at
                                            // one workgroup per CU
constexpr int kLutBytes = 2048;             // after the two buffers: the 8 mask bytes of every
                                            // byte value (byte j is bit j of the value)
constexpr int kSlotBytes = 16;              // the end of the second buffer, never staged into:
                                            // the persistent batch's item broadcast
// K-block record: 8 x u32 run masks (index 4 g + trial for segment g; bit j: window byte
// o_g - 8 + j is in the trial's run), then the LDS byte address of each of the 2 segments'
// first window byte (region + 2 o_g; lane 32 g + n reads 16 bytes at address[g] + 16 n +
// 512 q for product q), padding to a multiple of 16 bytes
constexpr int kRecBytes = 48;
constexpr int kRecBase = 32;                // byte offset of the segment addresses
static_assert(kRecBytes % 16 == 0 && kRecBase + 8 <= kRecBytes, "records copied in 16-byte chunks");
// Staging: up to kUnitsPerThread chunks (16 window bytes in both copies) per thread and
// group, so a group stages at most 64 NW kUnitsPerThread chunks (registers: the chunks'
// raw bytes are held through the current group's products).
constexpr int kUnitsPerThread = 2;

struct MGroup {
  int32_t unit_begin, nunits;   // staging units (16 window bytes of one channel each)
  int32_t kb_base;              // index into the per-wave K-block ranges
  int32_t kb_first, nkb;        // the group's K blocks (all waves): first and count
  int32_t rec_off;              // LDS byte offset of their records in the buffer
  int32_t block_begin, nblocks; // copy blocks (up to 1 KiB of one channel's region each)
};
struct MUnit {
  int32_t c;      // channel
  int32_t src;    // first window sample of the chunk, relative to the tile's first output
  int32_t dst;    // LDS byte offset of the chunk's 2 interleaved copies (32 bytes)
  int32_t pad;
};
// A copy block of the direct staging: up to 64 consecutive 16-byte pieces of a channel's
// region (piece m holds window bytes 8 m .. 8 m + 15), one buffer-to-LDS load of 16 bytes
// a lane from the converted block.
struct MBlock {
  int32_t c;      // channel
  int32_t src;    // window sample of the block's first byte, relative to the tile's first
                  // output (a multiple of 8)
  int32_t dst;    // LDS byte offset of the block
  int32_t nl;     // pieces (lanes), 1 .. 64
};

struct MfmaCfgTables {
  bool ok = false;
  int tw = 0, ntw = 0, trials = 0;
  std::vector<int32_t> perm, ntot, group_begin, kbr;
  std::vector<MGroup> groups;
  std::vector<MUnit> units;
  std::vector<MBlock> blocks;
  int64_t xspan = 0;              // bytes of a converted row a tile's copy blocks reach past
                                  // the tile's first output
  int bufbytes = 0;               // LDS bytes of one staging buffer
  std::vector<uint8_t> recs;      // [kb][kRecBytes]
  int32_t *d_perm = nullptr, *d_ntot = nullptr, *d_group_begin = nullptr, *d_kbr = nullptr;
  MGroup *d_groups = nullptr;
  MUnit *d_units = nullptr;
  MBlock *d_blocks = nullptr;
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
    (void)hipFree(c.d_blocks);
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
  const MBlock *blocks;
  const uint8_t *xs;      // converted block (x ^ 0x80, rows of xs_stride bytes) for the
  int64_t xs_stride;      // direct staging
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

// One staging task: chunk k of the 2 copies of a window (copy p: window bytes 16 k + 8 p
// .. 16 k + 8 p + 15, as int8 x ^ 0x80, stored at dst + 16 p), from the raw bytes at the
// aligned address at or below window byte 16 k.
__device__ __forceinline__ void store_chunk(unsigned char *buf, int32_t dst, const uint32_t raw[8],
                                            int sh) {
  uint32_t e[6];
#pragma unroll
  for (int k = 0; k < 6; ++k)
    e[k] = __builtin_amdgcn_alignbyte(raw[k + 1], raw[k], (uint32_t)sh) ^ 0x80808080u;
#pragma unroll
  for (int p = 0; p < kCopies; ++p) {
    const v4i v = {(int32_t)e[2 * p], (int32_t)e[2 * p + 1], (int32_t)e[2 * p + 2],
                   (int32_t)e[2 * p + 3]};
    *(v4i *)(buf + dst + 16 * p) = v;
  }
}

// XCD-aware tile order (block b runs on XCD b mod 8): XCD x takes a contiguous run of
// tiles in an order that walks the time tiles in groups of kTimeGroup, DM tile by DM tile
// within a group.  The tiles an XCD runs at once are then a few DM tiles of the group's
// time tiles, and the next DM tiles read the group's windows again from the XCD's L2
// while they are still there (every DM tile of one time tile at once, the order before,
// fetched 3.8 times as many bytes from beyond the L2 and ran 2-3 % slower).
constexpr int kTimeGroup = 8;
__device__ __forceinline__ void tile_of_block(int ntw, int ntt, int *tt, int *tw) {
  const int nb = ntw * ntt;
  const int bi = blockIdx.x;
  const int xcd = bi & 7, kk = bi >> 3, q = nb >> 3, rem = nb & 7;
  const int L = xcd * q + min(xcd, rem) + kk;
  const int grp = L / (kTimeGroup * ntw), in = L - grp * kTimeGroup * ntw;
  const int gs = min(kTimeGroup, ntt - grp * kTimeGroup);   // time tiles in this group
  *tw = in / gs;
  *tt = grp * kTimeGroup + (in - *tw * gs);
}

typedef int32_t v16i __attribute__((ext_vector_type(16)));

template <int N>
struct TileAcc {
  v16i v[N];
};

// The products of DM tile tw over outputs T0 .. T0 + NWT * 256 NP - 1.  Wave (wd, wt)
// takes trials 4 wd .. 4 wd + 3 of the tile and outputs T0 + 256 NP wt + ...; lane l,
// register r of product q holds trial 4 wd + r / 4 at output 256 NP wt + 256 q +
// 8 (l mod 32) + 4 (l / 32) + r mod 4.  Ends with a workgroup barrier, after which the
// LDS is free.  DMA: the windows come from the converted block a.xs by buffer-to-LDS
// loads (copy blocks), else from x through registers (staging units).
template <int NWD, int NWT, int NP, int WG, bool DMA, typename MA>
__device__ __forceinline__ TileAcc<NP> mfma_tile(MA &a, int tw, int64_t T0, const uint8_t *xb,
                                                 unsigned char *lds) {
  constexpr int NW = NWD * NWT;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wd = wave % NWD, wt = wave / NWD;
  v16i acc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0;

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
  // staging: thread t takes chunks t, t + 64 NW, ... of the group
  uint32_t raw[kUnitsPerThread][8];
  int sh[kUnitsPerThread] = {}, dst[kUnitsPerThread] = {};
  bool has[kUnitsPerThread] = {};
  auto fetch = [&](int g) {
    const int ub = ldc(&a.groups[g].unit_begin, 0), nu = ldc(&a.groups[g].nunits, 0);
#pragma unroll
    for (int j = 0; j < kUnitsPerThread; ++j) {
      const int ui = tid + 64 * NW * j;
      has[j] = ui < nu;
      if (has[j]) {
        const MUnit u = a.units[ub + ui];
        load_raw(xb + (int64_t)u.c * a.in_stride, a.nsamp, T0 + u.src, raw[j], &sh[j]);
        dst[j] = u.dst;
      }
    }
  };
  auto store = [&](unsigned char *buf) {
#pragma unroll
    for (int j = 0; j < kUnitsPerThread; ++j)
      if (has[j]) store_chunk(buf, dst[j], raw[j], sh[j]);
  };
  // direct staging: wave w takes copy blocks w, w + NW, ... of the group; lane l of a
  // block loads the 16 converted bytes from window byte 8 l of the block into LDS at
  // the block's offset + 16 l (the loads land in LDS without registers and are waited
  // for with the other vector-memory loads before the group's barrier)
  auto dma_block = [&](const v4i d, unsigned char *buf) {   // d: c, src, dst, nl
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(a.xs + (int64_t)d[0] * a.xs_stride), (short)0, (int)a.xs_stride, kBufWord3);
    if (lane < d[3])
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void *)(buf + d[2]), 16,
                                               (int)(T0 + d[1]) + 8 * lane, 0, 0, 0);
  };
  // the block descriptors are read two at a time (one scalar round trip per pair)
  auto dma_stage = [&](int g, unsigned char *buf) {
    const int bb = ldc(&a.groups[g].block_begin, 0), nb = ldc(&a.groups[g].nblocks, 0);
    const v4i *bd = (const v4i *)(a.blocks + bb);
    int b = wave;
    for (; b + NW < nb; b += 2 * NW) {
      const v4i d0 = ldc(bd, b), d1 = ldc(bd, b + NW);
      dma_block(d0, buf);
      dma_block(d1, buf);
    }
    if (b < nb) dma_block(ldc(bd, b), buf);
  };
  // the mask-expansion table (written before the first group's barrier, read only after it)
  typedef uint32_t v2u __attribute__((ext_vector_type(2)));
  unsigned char *lut = lds + 2 * (kMfmaBufBytes / WG);
  for (int e = tid; e < 256; e += 64 * NW) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      lo |= ((uint32_t)(e >> j) & 1u) << (8 * j);
      hi |= ((uint32_t)(e >> (j + 4)) & 1u) << (8 * j);
    }
    *(v2u *)(lut + 8 * e) = (v2u){lo, hi};
  }
  stage_recs(gb, lds);
  if constexpr (DMA) {
    dma_stage(gb, lds);
  } else {
    fetch(gb);
    store(lds);
  }
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();
  // the lane's byte offset from a segment's base: column lane mod 32 of the wave's run
  const int loff = 16 * (lane & 31) + 2 * kOutsPerProduct * NP * wt;
  // the lane's run mask in a record (segment lane / 32, trial (lane mod 32) / 8) and the
  // bit of it that is mask byte 0 (8 - phase)
  const int moff = 16 * (lane >> 5) + 4 * ((lane & 31) >> 3);
  const uint32_t msh = 8 - (lane & 7);
  for (int g = gb; g < ge; ++g) {
    const int par = (g - gb) & 1;
    unsigned char *buf = lds + par * a.bufbytes;
    const int kbase = ldc(&a.groups[g].kb_base, 0), kf = ldc(&a.groups[g].kb_first, 0);
    const int ro = ldc(&a.groups[g].rec_off, 0);
    const int k0 = ldc(a.kbr, (int64_t)kbase + wd), k1 = ldc(a.kbr, (int64_t)kbase + wd + 1);
    const unsigned char *rb = buf + ro + (int64_t)(k0 - kf) * kRecBytes;
    // while its products run, this wave is issued ahead of waves in their staging stores or
    // boxcar stage (of the CU's other workgroup, or of this one)
    __builtin_amdgcn_s_setprio(1);
    // the next K block's mask and segment base are read while this block's products run
    uint32_t m_next = 0;
    int32_t b_next = 0;
    if (k0 < k1) {
      m_next = *(const uint32_t *)(rb + moff);
      b_next = *(const int32_t *)(rb + kRecBase + 4 * (lane >> 5));
    }
    auto kblock = [&](int kb) {
      const uint32_t m32 = m_next;
      const unsigned char *bp = buf + b_next + loff;
      if (kb + 1 < k1) {
        m_next = *(const uint32_t *)(rb + kRecBytes + moff);
        b_next = *(const int32_t *)(rb + kRecBytes + kRecBase + 4 * (lane >> 5));
      }
      // 16 mask bytes of lane (row lane % 32 = trial 8 m + phase u, segment lane / 32):
      // byte j is bit 8 - u + j of the run mask, 8 bytes at a time from the table
      const v2u e0 = *(const v2u *)(lut + 8 * __builtin_amdgcn_ubfe(m32, msh, 8));
      const v2u e1 = *(const v2u *)(lut + 8 * __builtin_amdgcn_ubfe(m32, msh + 8, 8));
      const v4i mk = {(int32_t)e0[0], (int32_t)e0[1], (int32_t)e1[0], (int32_t)e1[1]};
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const v4i bq = *(const v4i *)(bp + 2 * kOutsPerProduct * q);
        acc[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(mk, bq, acc[q], 0, 0, 0);
      }
      rb += kRecBytes;
    };
    // the next group's staging is issued after this group's first K block, so that the
    // scalar reads of its descriptors wait while this group's first products run
    int kb = k0;
    if (kb < k1) kblock(kb++);
    if (g + 1 < ge) {
      stage_recs(g + 1, lds + (par ^ 1) * a.bufbytes);
      if constexpr (DMA) dma_stage(g + 1, lds + (par ^ 1) * a.bufbytes);
      else fetch(g + 1);
    }
    // two K blocks an iteration (half the register copies of the next record's mask and
    // base, and one pointer step for two)
    for (; kb + 1 < k1; kb += 2) {
      kblock(kb);
      kblock(kb + 1);
    }
    if (kb < k1) kblock(kb);
    __builtin_amdgcn_s_setprio(0);
    if constexpr (!DMA) {
      if (g + 1 < ge) store(lds + (par ^ 1) * a.bufbytes);
    }
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
  }
  TileAcc<NP> r;
#pragma unroll
  for (int q = 0; q < NP; ++q) r.v[q] = acc[q];
  return r;
}

// The 4 outputs of trial m (of the wave) that lane l holds in product q: registers
// 4 m .. 4 m + 3, outputs 256 q + 8 (l mod 32) + 4 (l / 32) + 0 .. 3 of the wave's run.
template <int NP>
__device__ __forceinline__ v4i quad_of(const TileAcc<NP> &acc, int q, int m) {
  return (v4i){acc.v[q][4 * m], acc.v[q][4 * m + 1], acc.v[q][4 * m + 2], acc.v[q][4 * m + 3]};
}

// WG workgroups per CU (their LDS), so WG NW / 4 waves per SIMD: registers up to 512 /
// that.
template <int NWD, int NWT, int NP, int WG>
__global__ void __launch_bounds__(64 * NWD * NWT)
__attribute__((amdgpu_waves_per_eu(WG * NWD * NWT / 4, WG * NWD * NWT / 4)))
k_dedisp_mfma(MfmaArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  constexpr int TWV = kOutsPerProduct * NP, TW = NWT * TWV;
  int tt, tw;
  tile_of_block(a.ntw, a.ntt, &tt, &tw);
  const int bb = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wd = wave % NWD, wt = wave / NWD;
  const int64_t T0 = (int64_t)tt * TW;
  const TileAcc<NP> acc =
      mfma_tile<NWD, NWT, NP, WG, false>(a, tw, T0, a.x + (int64_t)bb * a.in_bstride, lds);
  // The rows go out through LDS (free after the tile's last barrier; each wave has its
  // own 2 rows), so that each store instruction writes 256 consecutive bytes of a row.
  constexpr int OROW = TWV + 4;
  static_assert(NWD * NWT * 2 * OROW * 4 <= 2 * (kMfmaBufBytes / WG), "output rows fit the LDS");
  int *R = (int *)lds + wave * 2 * OROW;
  int32_t *ob = a.out + (int64_t)bb * a.out_bstride;
  const int64_t t0 = T0 + (int64_t)TWV * wt;
  const int col = 8 * (lane & 31) + 4 * (lane >> 5);
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int q = 0; q < NP; ++q)
        *(v4i *)(R + m * OROW + kOutsPerProduct * q + col) = quad_of<NP>(acc, q, 2 * pass + m);
    // LDS operations of one wave complete in order: the reads below see the writes
    __builtin_amdgcn_wave_barrier();
#pragma unroll 1
    for (int k = 0; k < 2; ++k) {
      const int d = a.perm[tw * kTrialsPerWave * NWD + kTrialsPerWave * wd + 2 * pass + k];
      if (d < 0) continue;
      const int32_t corr = 128 * a.ntot[d];
      int32_t *o = ob + (int64_t)d * a.out_stride + t0;
#pragma unroll
      for (int j = 0; j < TWV / 64; ++j)
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
  const int32_t *ntap;    // the plan's tap counts [ndm][nchan] (multi-beam noise tables)
  int32_t nchan, ndm;
};

// Time-tile step of the search: the tile's 64 SP outputs less a halo of >= 31 outputs,
// in whole lanes of SP starts (as the boxcar stage needs).
constexpr int search_step(int sp) { return 64 * sp - ((32 + sp - 1) / sp) * sp; }

// Fused search: the products of one tile (outputs T0 .. T0 + TW - 1, T0 = tt * TT),
// then the boxcar search of every trial of the tile over starts T0 .. T0 + TT - 1.
// The series go through LDS in two passes (trials 0-1, then 2-3 of every wave), as rows
// of TW + 36 ints; each wave searches whole rows.
template <int NWD, int NWT, int NP, int WG, bool DMA, typename SA>
__device__ __forceinline__ void search_tile_mfma(SA &sa, int tt, int tw, unsigned char *lds) {
  constexpr int NW = NWD * NWT, TWV = kOutsPerProduct * NP, TW = NWT * TWV, SP = TW / 64;
  constexpr int TT = search_step(SP), YROW = TW + kHalo + 4;
  constexpr int PT = 2;                    // trials of one wave in one pass
  constexpr int ROWS = PT * NWD;           // rows of one pass
  static_assert(TW % 64 == 0 && TT % SP == 0 && TW - TT >= 31, "search tile");
  static_assert(ROWS % NW == 0, "whole rows per wave");
  constexpr bool kOwnRows = NWT == 1 && ROWS / NW == PT;   // wave w searches rows PT w ..
  static_assert(!kOwnRows || NW == NWD, "one wave along time");
  static_assert(ROWS * YROW * 4 <= 2 * (kMfmaBufBytes / WG) - kSlotBytes,
                "rows of one pass fit the LDS (less the item slot)");
  static_assert(YROW % 4 == 0, "16-byte aligned rows");
  auto &a = sa.m;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wd = wave % NWD, wt = wave / NWD;
  const int64_t T0 = (int64_t)tt * TT;
  const TileAcc<NP> acc = mfma_tile<NWD, NWT, NP, WG, DMA>(a, tw, T0, a.x, lds);
  constexpr int DT = kTrialsPerWave * NWD;
  int *Y = (int *)lds;
  const int col = TWV * wt + 8 * (lane & 31) + 4 * (lane >> 5);
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
    for (int m = 0; m < PT; ++m) {
      const int d = a.perm[tw * DT + kTrialsPerWave * wd + PT * pass + m];
      const int32_t corr = d >= 0 ? 128 * a.ntot[d] : 0;
      int *row = Y + (PT * wd + m) * YROW + col;
#pragma unroll
      for (int q = 0; q < NP; ++q)
        *(v4i *)(row + kOutsPerProduct * q) =
            quad_of<NP>(acc, q, PT * pass + m) + (v4i){corr, corr, corr, corr};
    }
    // With one wave along time each wave searches the rows it wrote (rows PT wd ..
    // PT wd + PT - 1), so only its own LDS operations, which complete in order, need
    // to be ordered; rows of several time waves need the workgroup barrier.
    if constexpr (kOwnRows) __builtin_amdgcn_wave_barrier();
    else __syncthreads();
    // one row at a time, not unrolled: the search code then stays small enough
    // for the instruction cache
#pragma unroll 1
    for (int r = 0; r < ROWS / NW; ++r) {
      const int rw = wave * (ROWS / NW) + r;
      const int sw = rw / PT, j = rw % PT;   // wave along DM, trial of the pass
      const int dg = a.perm[tw * DT + kTrialsPerWave * sw + PT * pass + j];
      const CandRec rec =
          boxcar_row<SP>(Y + rw * YROW, lane, T0, TT, a.nout, dg, sa.wmask, sa.nw, sa.M, sa.S);
      if (dg >= 0 && lane == 0) sa.part[(int64_t)dg * a.ntt + tt] = rec;
    }
    // the LDS is free for the next pass's rows (or the next tile) once every wave that
    // reads these rows is done
    if (kOwnRows && pass == 0) __builtin_amdgcn_wave_barrier();
    else __syncthreads();
  }
}

template <int NWD, int NWT, int NP, int WG, bool DMA>
__global__ void __launch_bounds__(64 * NWD * NWT)
__attribute__((amdgpu_waves_per_eu(WG * NWD * NWT / 4, WG * NWD * NWT / 4)))
k_search_mfma(MfmaSearchArgs sa) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  int tt, tw;
  tile_of_block(sa.m.ntw, sa.m.ntt, &tt, &tw);
  search_tile_mfma<NWD, NWT, NP, WG, DMA>(sa, tt, tw, lds);
}

// Multi-beam fused search: one workgroup per (beam, tile).  Beam b owns the blocks
// [base[b], base[b] + its tile count rounded up to 8), base[b] a multiple of 8, so that
// block i of a beam runs on XCD i mod 8 and the beam's tiles take the one-beam
// kernel's XCD-aware order.  Blocks past a beam's tile count exit at once (the whole
// workgroup, before any barrier).
template <int NWD, int NWT, int NP, int WG>
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
  search_tile_mfma<NWD, NWT, NP, WG, false>(sa, tt, tw, lds);
}

// Persistent multi-beam search: a grid that fills the GPU once; each workgroup claims
// work items (beam, tile) from a device counter until the list is exhausted.  Thread 0
// claims an item and passes it to the workgroup through the LDS slot at the end of the
// second staging buffer (never staged into); the exit is uniform over the workgroup, so
// every wave reaches it.  The counter is zeroed by k_reset_counter before the launch.
template <int NWD, int NWT, int NP, int WG>
__global__ void __launch_bounds__(64 * NWD * NWT)
__attribute__((amdgpu_waves_per_eu(WG * NWD * NWT / 4, WG * NWD * NWT / 4)))
k_search_mfma_persist(const MfmaSearchArgs *__restrict__ beams, const int2 *__restrict__ items,
                      int32_t nitems, int32_t *__restrict__ counter) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  int32_t *slot = (int32_t *)(lds + 2 * (kMfmaBufBytes / WG) - kSlotBytes);
  typedef const __attribute__((address_space(4))) MfmaSearchArgs CArgs;
  for (;;) {
    if (threadIdx.x == 0)
      *slot = __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(*slot);
    if (it >= nitems) return;   // the same for every thread of the workgroup
    const int2 w = items[it];
    const int b = __builtin_amdgcn_readfirstlane(w.x), L = __builtin_amdgcn_readfirstlane(w.y);
    CArgs &sa = ((CArgs *)beams)[b];
    const int tt = L / sa.m.ntw, tw = L - tt * sa.m.ntw;
    // the tile ends with a workgroup barrier, after which thread 0 may claim the next item
    search_tile_mfma<NWD, NWT, NP, WG, false>(sa, tt, tw, lds);
  }
}

__global__ void k_reset_counter(int32_t *counter) { *counter = 0; }

// Beam of trial i of the multi-beam list: the last b with tbase[b] <= i.
__device__ __forceinline__ int beam_of_trial(const int32_t *tbase, int nbeam, int i) {
  int lo = 0, hi = nbeam - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ldc(tbase, mid) <= i) lo = mid; else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// Noise tables of every beam's trials in one launch (unit weights): workgroup i takes
// trial i - tbase[b] of beam b.
__global__ void __launch_bounds__(64 * kBucketWaves)
k_norm_beams(const MfmaSearchArgs *__restrict__ beams, const int32_t *__restrict__ tbase,
             int32_t nbeam, WidthList wl, const double *__restrict__ mu,
             const double *__restrict__ sigma) {
  typedef const __attribute__((address_space(4))) MfmaSearchArgs CArgs;
  const int i = blockIdx.x, b = beam_of_trial(tbase, nbeam, i);
  CArgs &sa = ((CArgs *)beams)[b];
  const int d = i - ldc(tbase, b);
  norm_buckets_trial(sa.ntap + (int64_t)d * sa.nchan, sa.nchan, DEDISP_W_UNIT, nullptr, mu,
                     sigma, wl, (double *)sa.M + (int64_t)d * wl.n,
                     (double *)sa.S + (int64_t)d * wl.n);
}

// Per-trial best over the time tiles of every beam in one launch; outputs in the
// order of the trial list (beam by beam).
__global__ void __launch_bounds__(kReduceThreads)
k_reduce_beams(const MfmaSearchArgs *__restrict__ beams, const int32_t *__restrict__ tbase,
               int32_t nbeam, double *__restrict__ snr, int32_t *__restrict__ t,
               int32_t *__restrict__ w) {
  typedef const __attribute__((address_space(4))) MfmaSearchArgs CArgs;
  const int i = blockIdx.x, b = beam_of_trial(tbase, nbeam, i);
  CArgs &sa = ((CArgs *)beams)[b];
  const int d = i - ldc(tbase, b);
  best_of_row(sa.part + (int64_t)d * sa.m.ntt, sa.m.ntt, snr + i, t + i, w + i);
}

}  // namespace

// ---- host ----------------------------------------------------------------------
template <typename T>
static hipError_t upload(T **dst, const std::vector<T> &v) {
  if (v.empty()) return hipSuccess;
  hipError_t e = dev_malloc((void **)dst, sizeof(T) * v.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

// Tables of configuration ci: trial order, per DM tile the channel groups with their
// staging units, and per (group, wave along DM) the K blocks (masks and segment bases).
static bool build_mfma_cfg(const dedisp_plan_s *p, int ci, MfmaCfgTables &out) {
  const MfmaCfg cf = kMfmaCfgs[ci];
  const int C = p->nchan, D = p->ndm;
  constexpr int TPW = kTrialsPerWave;
  const int NWD = cf.nwd, NW = cf.nwd * cf.nwt, TW = cf.nwt * kOutsPerProduct * cf.np;
  const int DT = TPW * NWD;
  constexpr int SEGS = 2;   // segments per K block
  const int BUF = kMfmaBufBytes / cf.wg;
  const int maxunits = 64 * NW * kUnitsPerThread;
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
  // per (wave along DM, channel): first segment (window-relative, a multiple of 8) and count
  std::vector<int32_t> so(NWD * C), nseg(NWD * C);
  // per channel: window origin (absolute delay of window byte 0, a multiple of 8, so
  // that every copy block of the direct staging starts 8-byte aligned in the converted
  // row) and bytes per copy
  std::vector<int32_t> wlo(C), clen(C);
  for (int tw = 0; tw < ntw; ++tw) {
    out.group_begin[tw] = (int)out.groups.size();
    for (int c = 0; c < C; ++c) {
      std::vector<int> l(NWD), h(NWD);
      int slo = INT32_MAX;
      for (int w = 0; w < NWD; ++w) {
        l[w] = INT32_MAX;
        h[w] = INT32_MIN;
        for (int m = 0; m < TPW; ++m) {
          const int d = out.perm[(size_t)tw * DT + TPW * w + m];
          if (d < 0 || p->ntap[(size_t)d * C + c] == 0) continue;
          l[w] = std::min(l[w], p->start[(size_t)d * C + c]);
          // the phase rows u = 1 .. 7 take the run's samples up to 7 later
          h[w] = std::max(h[w], p->start[(size_t)d * C + c] + p->ntap[(size_t)d * C + c] +
                                    kPhases - 1);
        }
        slo = std::min(slo, l[w]);
      }
      clen[c] = 0;
      if (slo == INT32_MAX) {
        for (int w = 0; w < NWD; ++w) nseg[w * C + c] = 0;
        continue;
      }
      wlo[c] = slo / 8 * 8;   // delays are >= 0
      int smax = 0;   // largest segment start
      for (int w = 0; w < NWD; ++w) {
        if (l[w] == INT32_MAX) {
          nseg[w * C + c] = 0;
          continue;
        }
        const int o = (l[w] - wlo[c]) / 8 * 8;   // on the 8-byte grid, at or below the band
        so[w * C + c] = o;
        nseg[w * C + c] = (h[w] - (wlo[c] + o) + 15) / 16;
        smax = std::max(smax, o + 16 * (nseg[w * C + c] - 1));
      }
      // the last lane reads 16 bytes from window byte smax + TW - 8: chunks up to that
      // byte / 16 (copy 1 of a chunk holds its bytes 8 .. 23)
      clen[c] = 16 * ((smax + TW - 8) / 16 + 1);
      if ((int64_t)kCopies * clen[c] + kRecBytes > BUF - kSlotBytes || clen[c] / 16 > maxunits)
        return false;
      // the last piece of the channel's region (window bytes clen - 8 .. clen + 7)
      out.xspan = std::max(out.xspan, (int64_t)wlo[c] + clen[c] + 8);
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
        for (int w = 0; w < NWD; ++w) nrec += (segw[w] + nseg[w * C + c] + SEGS - 1) / SEGS;
        if ((int64_t)used + (int64_t)kCopies * clen[c] + (int64_t)nrec * kRecBytes >
            BUF - kSlotBytes)
          break;
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
          out.units.push_back(MUnit{cc, wlo[cc] + 16 * k, off + 16 * kCopies * k, 0});
        off += kCopies * clen[cc];
      }
      gi.nunits = (int)out.units.size() - gi.unit_begin;
      gi.block_begin = (int)out.blocks.size();
      for (int cc = cbeg; cc < c; ++cc) {
        const int npiece = kCopies * clen[cc] / 16;   // 16-byte pieces of the region
        for (int j = 0; 64 * j < npiece; ++j)
          out.blocks.push_back(
              MBlock{cc, wlo[cc] + 8 * 64 * j, region[cc] + 16 * 64 * j, std::min(64, npiece - 64 * j)});
      }
      gi.nblocks = (int)out.blocks.size() - gi.block_begin;
      gi.kb_base = (int)out.kbr.size();
      gi.kb_first = (int)(out.recs.size() / kRecBytes);
      gi.rec_off = off;
      for (int w = 0; w < NWD; ++w) {
        out.kbr.push_back((int32_t)(out.recs.size() / kRecBytes));
        // segments of this wave's trials in the group (channel, window-relative start),
        // two per K block
        std::vector<std::pair<int, int>> segs;
        for (int cc = cbeg; cc < c; ++cc)
          for (int sg = 0; sg < nseg[w * C + cc]; ++sg) segs.push_back({cc, so[w * C + cc] + 16 * sg});
        for (size_t s0 = 0; s0 < segs.size(); s0 += SEGS) {
          std::vector<uint8_t> rec(kRecBytes, 0);
          for (int g = 0; g < SEGS; ++g) {
            // padding segments: zero masks, a valid address
            const size_t si = s0 + g < segs.size() ? s0 + g : s0;
            const int cc = segs[si].first, o = segs[si].second;
            // window byte o (a multiple of 8) of the interleaved copies is at region + 2 o
            const int32_t ad = region[cc] + 2 * o;
            std::memcpy(rec.data() + kRecBase + 4 * g, &ad, 4);
            if (s0 + g >= segs.size()) continue;
            const int oa = wlo[cc] + o;   // absolute delay of the segment's first byte
            for (int m = 0; m < TPW; ++m) {
              const int d = out.perm[(size_t)tw * DT + TPW * w + m];
              if (d < 0) continue;
              const int st = p->start[(size_t)d * C + cc], nt = p->ntap[(size_t)d * C + cc];
              // bit j: delay oa - 8 + j is in the run (row (m, u) takes byte i when delay
              // oa + i - u is, i.e. bit i + 8 - u)
              uint32_t bits = 0;
              for (int j = 0; j < 32; ++j)
                if (oa - 8 + j >= st && oa - 8 + j < st + nt) bits |= 1u << j;
              std::memcpy(rec.data() + 4 * (4 * g + m), &bits, 4);
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

// Host-only consistency check of shape k's tables (test support): the staging units
// (register staging) and the copy blocks (direct staging) fill the same LDS pieces of each
// group with the same window bytes; every K-block segment's lanes read inside its channel's
// staged region (window bytes o + 8 n + 256 q' .. + 15 for column n < 32 and product q' of
// the tile, so o + TW <= the region's bytes per copy); window origins are multiples of 8;
// and the converted rows reach every copy block.  *pieces: LDS pieces compared.
dedisp_status mfma_check_tables(const dedisp_plan_s *p, int k, int64_t *pieces) {
  if (k < 0 || k >= kNumMfmaCfgs) return fail(DEDISP_ERR_INVALID_ARG, "shape out of range");
  MfmaCfgTables c;
  if (!build_mfma_cfg(p, k, c)) return fail(DEDISP_ERR_UNSUPPORTED, "plan does not fit the shape");
  const int TW = c.tw;
  auto bad = [](const std::string &m) { return fail(DEDISP_ERR_UNSUPPORTED, "table check: " + m); };
  int64_t n = 0;
  for (size_t g = 0; g < c.groups.size(); ++g) {
    const MGroup &G = c.groups[g];
    // LDS piece offset -> (channel, window sample of its first byte), from both stagings
    std::vector<std::pair<int32_t, std::pair<int32_t, int32_t>>> from_units, from_blocks;
    for (int u = G.unit_begin; u < G.unit_begin + G.nunits; ++u)
      for (int h = 0; h < kCopies; ++h)
        from_units.push_back({c.units[u].dst + 16 * h, {c.units[u].c, c.units[u].src + 8 * h}});
    for (int b = G.block_begin; b < G.block_begin + G.nblocks; ++b) {
      const MBlock &B = c.blocks[b];
      if (B.nl < 1 || B.nl > 64 || B.src % 8) return bad("copy block shape");
      if ((int64_t)B.src + 8 * (B.nl - 1) + 16 > c.xspan) return bad("converted row too short");
      for (int l = 0; l < B.nl; ++l) from_blocks.push_back({B.dst + 16 * l, {B.c, B.src + 8 * l}});
    }
    std::sort(from_units.begin(), from_units.end());
    std::sort(from_blocks.begin(), from_blocks.end());
    if (from_units != from_blocks) return bad("units and copy blocks differ in group " + std::to_string(g));
    n += (int64_t)from_units.size();
    if (from_units.empty()) continue;
    // the group's window area [0, rec_off): per channel region [first piece, last piece + 16)
    std::vector<int32_t> lo(p->nchan, INT32_MAX), hi(p->nchan, INT32_MIN), org(p->nchan, 0);
    for (auto &e : from_units) {
      const int ch = e.second.first;
      if (e.first < lo[ch]) {
        lo[ch] = e.first;
        org[ch] = e.second.second;   // window sample of the region's first byte
      }
      hi[ch] = std::max(hi[ch], e.first + 16);
      if (e.first + 16 > G.rec_off) return bad("window piece over the records");
    }
    for (int ch = 0; ch < p->nchan; ++ch)
      if (lo[ch] != INT32_MAX && (org[ch] % 8)) return bad("window origin not a multiple of 8");
    // every segment of the group's K blocks
    for (int kb = G.kb_first; kb < G.kb_first + G.nkb; ++kb)
      for (int sg = 0; sg < 2; ++sg) {
        int32_t ad = 0;
        std::memcpy(&ad, c.recs.data() + (size_t)kb * kRecBytes + kRecBase + 4 * sg, 4);
        if (ad % 16) return bad("segment base not 16-byte aligned");
        int ch = -1;
        for (int cc = 0; cc < p->nchan; ++cc)
          if (lo[cc] != INT32_MAX && ad >= lo[cc] && ad < hi[cc]) ch = cc;
        if (ch < 0) return bad("segment base outside every staged region");
        const int64_t o = (ad - lo[ch]) / 2;              // window byte of the segment
        if (2 * (o + TW) > (int64_t)(hi[ch] - lo[ch])) return bad("segment reads past its region");
      }
  }
  if (pieces) *pieces = n;
  return DEDISP_OK;
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

template <int NWD, int NWT, int NP, int WG>
static hipError_t launch_mfma_cfg(const MfmaArgs &a, int nbatch, hipStream_t s) {
  static bool done[64] = {};
  static std::mutex mu;
  hipError_t e = allow_lds_mfma((const void *)k_dedisp_mfma<NWD, NWT, NP, WG>, done, &mu,
                                2 * (kMfmaBufBytes / WG) + kLutBytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_dedisp_mfma<NWD, NWT, NP, WG>), dim3(a.ntw * a.ntt, nbatch),
                     dim3(64 * NWD * NWT), 2 * a.bufbytes + kLutBytes, s, a);
  return hipGetLastError();
}

static hipError_t launch_mfma(int ci, const MfmaArgs &a, int nbatch, hipStream_t s) {
  switch (ci) {
#define DD_MFMA_CASE(i, x, y, n, g) \
  case i: return launch_mfma_cfg<x, y, n, g>(a, nbatch, s);
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
      DD_HIP(upload(&c.d_blocks, c.blocks));
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
  a.blocks = c.d_blocks;
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
  int64_t xs_stride = 0;          // converted row length (0: staging through registers)
  size_t off_part = 0, off_xs = 0, total = 0;
};

// Workspace of shape k: noise tables, per-(trial, time tile) candidates and, for the
// direct staging (xspan > 0: the shape's reach past a tile's first output), the
// converted block [nchan][xs_stride].
static MfmaSearchLayout search_layout(const dedisp_plan_s *p, int k, int32_t nw, int64_t nout,
                                      int64_t xspan) {
  const MfmaCfg cf = kMfmaCfgs[k];
  const int tw = cf.nwt * kOutsPerProduct * cf.np, tstep = search_step(tw / 64);
  MfmaSearchLayout L;
  L.ntt = (nout + tstep - 1) / tstep;
  L.off_part = (2 * sizeof(double) * (size_t)p->ndm * nw + 255) & ~(size_t)255;
  L.off_xs = L.off_part + ((sizeof(CandRec) * (size_t)p->ndm * L.ntt + 255) & ~(size_t)255);
  L.total = L.off_xs;
  if (xspan > 0) {
    L.xs_stride = ((L.ntt - 1) * tstep + xspan + 255) & ~(int64_t)255;
    L.total += (size_t)p->nchan * (size_t)L.xs_stride;
  }
  return L;
}

// The most any shape's search can take: the converted block's rows reach at most
// max_span + 16 bytes plus a tile's outputs past a tile's first output.
static int64_t xspan_bound(const dedisp_plan_s *p, int k) {
  const MfmaCfg cf = kMfmaCfgs[k];
  return (int64_t)p->max_span + kPhases + 16 + 16 + cf.nwt * kOutsPerProduct * cf.np;
}

size_t mfma_search_work_bytes(const dedisp_plan_s *p, int32_t nw, int64_t nout) {
  size_t b = 0;
  for (int k = 0; k < kNumMfmaCfgs; ++k)
    b = std::max(b, search_layout(p, k, nw, nout, xspan_bound(p, k)).total);
  return b;
}

int mfma_search_count() { return kNumMfmaCfgs; }

template <int NWD, int NWT, int NP, int WG, bool DMA>
static hipError_t launch_search_cfg(const MfmaSearchArgs &sa, hipStream_t s) {
  static bool done[64] = {};
  static std::mutex mu;
  hipError_t e = allow_lds_mfma((const void *)k_search_mfma<NWD, NWT, NP, WG, DMA>, done, &mu,
                                2 * (kMfmaBufBytes / WG) + kLutBytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_search_mfma<NWD, NWT, NP, WG, DMA>), dim3(sa.m.ntw * sa.m.ntt),
                     dim3(64 * NWD * NWT), 2 * sa.m.bufbytes + kLutBytes, s, sa);
  return hipGetLastError();
}

static hipError_t launch_search_mfma(int k, bool dma, const MfmaSearchArgs &sa, hipStream_t s) {
  switch (k) {
#define DD_MFMA_SEARCH_CASE(i, x, y, n, g) \
  case i: return dma ? launch_search_cfg<x, y, n, g, true>(sa, s) \
                     : launch_search_cfg<x, y, n, g, false>(sa, s);
    DD_MFMA_CONFIGS(DD_MFMA_SEARCH_CASE)
#undef DD_MFMA_SEARCH_CASE
    default: return hipErrorInvalidValue;
  }
}

dedisp_status run_search_mfma(dedisp_plan p, int k, const uint8_t *x, int64_t nsamp,
                              int64_t in_stride, int64_t nout, const WidthList &wl,
                              const double *mu, const double *sigma, double *snr, int32_t *t,
                              int32_t *w, void *work, hipStream_t s, bool dma) {
  if (k < 0 || k >= kNumMfmaCfgs || p->wmode != DEDISP_W_UNIT || wl.w[wl.n - 1] > 32)
    return DEDISP_ERR_UNSUPPORTED;
  MfmaCfgTables *cfg = nullptr;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    dedisp_status st = ensure_mfma(p, k, &cfg);
    if (st != DEDISP_OK) return st;
  }
  if (!cfg) return DEDISP_ERR_UNSUPPORTED;
  // the direct staging needs its converted block within the workspace the caller sized
  // with dedisp_work_bytes, and 32-bit buffer offsets
  if (dma && cfg->xspan > xspan_bound(p, k)) dma = false;
  MfmaSearchLayout L = search_layout(p, k, wl.n, nout, dma ? cfg->xspan : 0);
  if (dma && L.xs_stride > INT32_MAX) {
    dma = false;
    L = search_layout(p, k, wl.n, nout, 0);
  }
  if (L.ntt * cfg->ntw > INT32_MAX / 2) return DEDISP_ERR_UNSUPPORTED;
  MfmaSearchArgs sa{};
  fill_args(p, *cfg, x, nsamp, in_stride, nout, sa.m);
  sa.m.ntt = (int32_t)L.ntt;
  if (dma) {
    sa.m.xs = (const uint8_t *)work + L.off_xs;
    sa.m.xs_stride = L.xs_stride;
  }
  double *M = (double *)work;
  sa.M = M;
  sa.S = M + (size_t)p->ndm * wl.n;
  sa.nw = wl.n;
  sa.wmask = 0;
  for (int i = 0; i < wl.n; ++i) sa.wmask |= 1u << (wl.w[i] - 1);
  sa.part = (CandRec *)((char *)work + L.off_part);
  // the noise tables, and the converted block of the direct staging in the same launch
  ConvertJob cv{x, in_stride, nsamp, (uint8_t *)sa.m.xs, L.xs_stride, p->nchan};
  DD_HIP(launch_norm(p, wl, mu, sigma, M, (double *)sa.S, s, dma ? &cv : nullptr));
  KernelTimer kt(p, s);
  DD_HIP(kt.begin());
  DD_HIP(launch_search_mfma(k, dma, sa, s));
  DD_HIP(kt.end());
  DD_HIP(launch_reduce(p->ndm, (int32_t)L.ntt, sa.part, snr, t, w, s));
  return DEDISP_OK;
}

// ---- allocation-free fused search -------------------------------------------------
// The workspace of the fused search (noise tables and per-(trial, time tile)
// candidates) in a file-scope device array, for callers that cannot allocate.  Host
// code never passes the array's name to a kernel (a host-side stand-in, not a device
// address): its device address is taken once per device with hipGetSymbolAddress
// and kept.  Every call on a device shares that device's array; each call overwrites
// every byte it reads (k_norm writes the whole noise table, the search kernel a
// candidate for every trial and time tile), so nothing needs clearing, and calls
// that overlap on one device race.
constexpr size_t kNoAllocScratchBytes = (size_t)DEDISP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static void *g_scratch_ptr[64] = {};
static std::mutex g_scratch_mu;

static dedisp_status scratch_of_current_device(void **out) {
  int dev = 0;
  DD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(DEDISP_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(DEDISP_ERR_DEVICE, "hipGetSymbolAddress(scratch) gave no address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return DEDISP_OK;
}

dedisp_status run_search_noalloc(dedisp_plan p, const uint8_t *x, int64_t nsamp,
                                 int64_t in_stride, int64_t nout, const WidthList &wl,
                                 const double *mu, const double *sigma, double *snr, int32_t *t,
                                 int32_t *w, hipStream_t s) {
  if (p->wmode != DEDISP_W_UNIT || wl.w[wl.n - 1] > 32)
    return fail(DEDISP_ERR_UNSUPPORTED,
                "the allocation-free search takes unit weights and widths up to 32");
  // the plan's matrix-core shape: the forced or tuned one, else the first of the untuned
  // search's order (two workgroups per CU, then one) whose tables the plan has
  const bool chosen = p->tile_choice >= 8 && p->tile_choice < 8 + kNumMfmaCfgs;
  int k = chosen ? p->tile_choice - 8 : 1;
  int dev = 0;
  DD_HIP(hipGetDevice(&dev));
  {
    // the plan's device tables must exist already: building them would allocate
    std::lock_guard<std::mutex> lk(p->mu);
    if (!chosen && p->mfma && !(p->mfma->tried[1] && p->mfma->cfg[1].ok) && p->mfma->tried[0])
      k = 0;
    if (!p->uploaded || p->device != dev || !p->mfma || !p->mfma->tried[k])
      return fail(DEDISP_ERR_INVALID_ARG,
                  "plan tables are not on this device yet: run dedisp_search (or "
                  "dedisp_autotune) with this plan once before the allocation-free search");
    if (!p->mfma->cfg[k].ok)
      return fail(DEDISP_ERR_UNSUPPORTED, "the plan does not fit the matrix-core search");
  }
  const MfmaSearchLayout L = search_layout(p, k, wl.n, nout, 0);
  if (L.total > kNoAllocScratchBytes)
    return fail(DEDISP_ERR_INVALID_ARG,
                "workspace of " + std::to_string(L.total) + " bytes exceeds the " +
                    std::to_string(kNoAllocScratchBytes) +
                    "-byte scratch array of the allocation-free search");
  void *work = nullptr;
  dedisp_status st = scratch_of_current_device(&work);
  if (st != DEDISP_OK) return st;
  st = run_search_mfma(p, k, x, nsamp, in_stride, nout, wl, mu, sigma, snr, t, w, work, s, false);
  if (st == DEDISP_OK) p->last_search_tile = 8 + k;
  return st;
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
  std::vector<int32_t> tbase;               // first trial of each beam, then the total
  int32_t *d_tbase = nullptr;
  MfmaSearchArgs *d_args_graph = nullptr;   // argument table of the captured graph
  std::vector<MfmaSearchArgs> args;         // argument table of the last enqueue
  ArgStage stage;                           // pinned staging of the eager table
  // persistent launch: work items (beam, tile) in beam order, their counter, grid size
  bool persistent = false;
  int2 *d_items = nullptr;
  int32_t nitems = 0, pgrid = 0;
  int32_t *d_counter = nullptr;
};

void mfma_batch_free(MfmaBatch *B) {
  if (!B) return;
  B->stage.release();
  (void)hipFree(B->d_base);
  (void)hipFree(B->d_tbase);
  (void)hipFree(B->d_args_graph);
  (void)hipFree(B->d_items);
  (void)hipFree(B->d_counter);
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
    const MfmaSearchLayout L = search_layout(p, chosen, wl.n, no, 0);
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
  int64_t trials = 0;
  for (int b = 0; b < B->nbeam; ++b) {
    B->tbase.push_back((int32_t)trials);
    trials += plans[b]->ndm;
  }
  B->tbase.push_back((int32_t)trials);
  if (trials > INT32_MAX / 2) {
    mfma_batch_free(B);
    return DEDISP_OK;   // too many trials for one launch: not this path
  }
  // the persistent launch (the default; DEDISP_BATCH_LAUNCH=grid selects one workgroup
  // per tile instead): every (beam, tile) as a work item, beam by beam, each beam's
  // tiles in the one-plan kernel's order (time tiles in groups of kTimeGroup, DM tile
  // by DM tile within a group; 0.5-1 % faster than time-major order on 36 beams)
  const char *lm = getenv("DEDISP_BATCH_LAUNCH");
  B->persistent = !(lm && std::string(lm) == "grid");
  std::vector<int2> items;
  if (B->persistent) {
    for (int b = 0; b < B->nbeam; ++b) {
      const int64_t ntw = plans[b]->mfma->cfg[chosen].ntw, ntt = B->lay[b].ntt;
      for (int64_t g0 = 0; g0 < ntt; g0 += kTimeGroup)
        for (int64_t tw = 0; tw < ntw; ++tw)
          for (int64_t tt = g0; tt < std::min(ntt, g0 + kTimeGroup); ++tt)
            items.push_back(make_int2(b, (int)(tt * ntw + tw)));
    }
    B->nitems = (int32_t)items.size();
  }
  B->args_off = off;
  B->work_bytes = off + sizeof(MfmaSearchArgs) * B->nbeam;
  hipError_t e = upload(&B->d_base, B->base);
  if (e == hipSuccess) e = upload(&B->d_tbase, B->tbase);
  if (e == hipSuccess)
    e = dev_malloc((void **)&B->d_args_graph, sizeof(MfmaSearchArgs) * B->nbeam);
  if (e == hipSuccess && B->persistent) {
    e = upload(&B->d_items, items);
    if (e == hipSuccess) e = dev_malloc((void **)&B->d_counter, sizeof(int32_t));
    int dev = 0, ncu = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    B->pgrid = ncu * kMfmaCfgs[chosen].wg;   // one wave of resident workgroups
  }
  if (e != hipSuccess) {
    mfma_batch_free(B);
    return hip_fail(e, "batch setup");
  }
  *out = B;
  return DEDISP_OK;
}

template <int NWD, int NWT, int NP, int WG>
static hipError_t launch_batch_mfma_cfg(const MfmaBatch *B, const MfmaSearchArgs *table,
                                        hipStream_t s) {
  if (B->persistent) {
    static bool pdone[64] = {};
    static std::mutex pmu;
    hipError_t e = allow_lds_mfma((const void *)k_search_mfma_persist<NWD, NWT, NP, WG>, pdone,
                                  &pmu, 2 * (kMfmaBufBytes / WG) + kLutBytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, B->d_counter);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_search_mfma_persist<NWD, NWT, NP, WG>), dim3(B->pgrid),
                       dim3(64 * NWD * NWT), 2 * (kMfmaBufBytes / WG) + kLutBytes, s, table, B->d_items,
                       B->nitems, B->d_counter);
    return hipGetLastError();
  }
  static bool done[64] = {};
  static std::mutex mu;
  hipError_t e = allow_lds_mfma((const void *)k_search_mfma_batch<NWD, NWT, NP, WG>, done, &mu,
                                2 * (kMfmaBufBytes / WG) + kLutBytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_search_mfma_batch<NWD, NWT, NP, WG>), dim3(B->base.back()),
                     dim3(64 * NWD * NWT), 2 * (kMfmaBufBytes / WG) + kLutBytes, s, table, B->d_base,
                     B->nbeam);
  return hipGetLastError();
}

static hipError_t launch_batch_mfma(const MfmaBatch *B, const MfmaSearchArgs *table,
                                    hipStream_t s) {
  switch (B->k) {
#define DD_MFMA_BATCH_CASE(i, x, y, n, g) \
  case i: return launch_batch_mfma_cfg<x, y, n, g>(B, table, s);
    DD_MFMA_CONFIGS(DD_MFMA_BATCH_CASE)
#undef DD_MFMA_BATCH_CASE
    default: return hipErrorInvalidValue;
  }
}

// The argument table, the noise tables of every beam in one launch, one launch over every
// beam's tiles, the per-trial reductions of every beam in one launch.  Outputs of beam b
// start at out_off[b], its first trial in the list.  Eager calls
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
    sa.ntap = p->dev.ntap;
    sa.nchan = p->nchan;
    sa.ndm = p->ndm;
    if (out_off[b] != B->tbase[b]) return fail(DEDISP_ERR_INVALID_ARG, "beam output offsets");
  }
  MfmaSearchArgs *table = B->d_args_graph;
  if (!for_graph) {
    table = (MfmaSearchArgs *)((char *)work + B->args_off);
    DD_HIP(B->stage.copy(table, B->args.data(), sizeof(MfmaSearchArgs) * B->nbeam, s));
  }
  const unsigned ntrial = (unsigned)B->tbase.back();
  hipLaunchKernelGGL(k_norm_beams, dim3(ntrial), dim3(64 * kBucketWaves), 0, s, table, B->d_tbase,
                     B->nbeam, B->wl, mu, sigma);
  DD_HIP(hipGetLastError());
  if (kt) DD_HIP(kt->begin());
  DD_HIP(launch_batch_mfma(B, table, s));
  if (kt) DD_HIP(kt->end());
  hipLaunchKernelGGL(k_reduce_beams, dim3(ntrial), dim3(kReduceThreads), 0, s, table, B->d_tbase,
                     B->nbeam, snr, t, w);
  DD_HIP(hipGetLastError());
  return DEDISP_OK;
}

dedisp_status mfma_batch_upload(MfmaBatch *B) {
  DD_HIP(hipMemcpy(B->d_args_graph, B->args.data(), sizeof(MfmaSearchArgs) * B->nbeam,
                   hipMemcpyHostToDevice));
  return DEDISP_OK;
}

}  // namespace dd
