// Tiled fused search for uint8 data with unit weights: the dedispersion sum of
// eq. p_dedisp followed by the boxcar S/N search, without writing the
// dedispersed series to HBM.
//
// Data flow of one search call:
//   1. k_window_rows: for every channel c and every tap count n the plan uses in
//      that channel, the windowed sums U_{c,n}[tau] = sum_{k<n} x[c][tau+k] as
//      uint16 (exact: n * 255 < 65536 is required), zero past the block end.
//   2. k_search<DPW, R2>: one workgroup per (DM tile, time tile).  For a group of
//      channels it copies the needed U windows into LDS, twice (the second copy
//      shifted by one sample) so that every lane reads an aligned dword holding
//      two consecutive outputs; lanes of a wave read 64 consecutive dwords, so the
//      reads are free of bank conflicts.  Sums of two outputs are kept in packed
//      uint16 lanes and flushed into int32 before they can wrap (the host plans the
//      flush points from the tap counts).  After the last channel group each wave
//      runs the boxcar search on its trials: a register prefix of the tile's series,
//      all widths 1..32, a transpose-reduce of the per-width maxima across lanes,
//      fp64 S/N at the per-width maxima, and the earliest start of the winner.
//   3. k_reduce (kernels_basic.hip): best candidate per trial over time tiles.
// Workgroups are mapped to tiles so that each XCD (blocks are dealt to the 8 XCDs
// round-robin) walks whole time tiles across all DM tiles, keeping a time tile's
// U windows in that XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <vector>

#include "boxcar_row.h"
#include "internal.h"

namespace dd {

// ------------------------------------------------------------------------------
// Tile configurations (candidates for the autotuner)
// ------------------------------------------------------------------------------
// (trials per wave, packed output pairs per lane per row, waves per workgroup):
// a tile covers NW * DPW trials and 128 * R2 outputs; the NW waves share the
// staged windows, so more waves stage fewer bytes per sum.
#define DD_TILE_CONFIGS(X) \
  X(0, 4, 6, 4)            \
  X(1, 4, 8, 4)            \
  X(2, 6, 4, 4)            \
  X(3, 4, 4, 8)            \
  X(4, 4, 6, 8)            \
  X(5, 4, 8, 8)            \
  X(6, 4, 4, 16)           \
  X(7, 4, 6, 16)
struct TileCfg {
  int dpw;   // trials per wave
  int r2;    // packed output pairs per lane per row: outputs per tile row = 128 * r2
  int nw;    // waves per workgroup
};
#define DD_CFG_ENTRY(i, d, r, w) {d, r, w},
static const TileCfg kCfgs[] = {DD_TILE_CONFIGS(DD_CFG_ENTRY)};
#undef DD_CFG_ENTRY
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);
constexpr int kDefaultCfg = 0;
// Time-tile step: TY minus a halo of at least 31 outputs, rounded so that every
// lane (SP = 2 * r2 consecutive starts) owns either all or none of its starts.
constexpr int tile_step(int r2) { return 128 * r2 - ((32 + 2 * r2 - 1) / (2 * r2)) * (2 * r2); }
// LDS bytes for one channel group's windows per 4 waves, smallest first: two such
// buffers per workgroup (double buffering) let 16, 12 or 8 waves share a CU's
// 160 KiB.  A plan takes the smallest budget that holds every channel's windows.
constexpr int kStageBudgets[3] = {19968, 26624, 39936};
constexpr int kMaxLds = 160 * 1024;
// Window-row bytes per chunk of a multi-beam search: rows written just before the
// chunk's search should still sit in the 256 MiB last-level cache when read.
constexpr size_t kBatchChunkRows = 192u << 20;

struct GroupInfo {
  int32_t job_begin, njobs, lw, c_begin;   // lw: window length in samples (multiple of 8)
  int32_t c_count, flush, inv_nchunk, pad1;   // inv_nchunk: bits of (float)(1 / (lw / 8))
};

struct TiledCfgTables {
  bool ok = false;
  int dt = 0, ty = 0, tt = 0, ntd = 0, ngroups = 0, lds_bytes = 0, bufbytes = 0;
  std::vector<int32_t> offs;          // [ntd*dt][nchan] LDS byte offsets
  std::vector<GroupInfo> groups;      // flat
  std::vector<int32_t> group_begin;   // [ntd+1]
  std::vector<int2> jobs;             // {window row of (c, n), channel base start}
  std::vector<int32_t> perm;          // [ntd*dt] trial index or -1
  // device copies
  int32_t *d_offs = nullptr, *d_group_begin = nullptr, *d_perm = nullptr;
  GroupInfo *d_groups = nullptr;
  int2 *d_jobs = nullptr;
};

struct TiledTables {
  // Window rows: per channel, rows for n in [nmin_c, nmax_c].
  std::vector<int32_t> nmin, nmax;
  std::vector<int64_t> rowidx;        // first row index of channel c
  int64_t nrows = 0;
  int32_t *d_nmin = nullptr, *d_nmax = nullptr;
  int64_t *d_rowidx = nullptr;
  int32_t nmax_all = 0;
  TiledCfgTables cfg[kNumCfgs];
};

static void free_cfg(TiledCfgTables &c) {
  (void)hipFree(c.d_offs);
  (void)hipFree(c.d_group_begin);
  (void)hipFree(c.d_perm);
  (void)hipFree(c.d_groups);
  (void)hipFree(c.d_jobs);
}

void free_tiled(TiledTables *t) {
  if (!t) return;
  (void)hipFree(t->d_nmin);
  (void)hipFree(t->d_nmax);
  (void)hipFree(t->d_rowidx);
  for (auto &c : t->cfg) free_cfg(c);
  delete t;
}

// ------------------------------------------------------------------------------
// Kernels
// ------------------------------------------------------------------------------
namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_add_u16(uint32_t a, uint32_t b) {
  u16x2 va = __builtin_bit_cast(u16x2, a), vb = __builtin_bit_cast(u16x2, b);
  return __builtin_bit_cast(uint32_t, va + vb);
}

// U_{c,n}[tau] for tau in [0, tpad), n in [nmin_c, nmax_c], and the same rows one
// sample later, U1_{c,n}[tau] = U_{c,n}[tau + 1], so that a window starting at
// either parity can be copied to LDS from a dword-aligned source.  Each thread
// makes 8 consecutive tau of every row of its channel from bytes staged in LDS.
constexpr int kRowThreads = 256;
constexpr int kRowSpan = kRowThreads * 8;   // tau per block
__global__ void __launch_bounds__(kRowThreads)
k_window_rows(const uint8_t *__restrict__ x, int64_t in_stride, int64_t nsamp, int64_t tpad,
              const int32_t *__restrict__ nmin, const int32_t *__restrict__ nmaxv,
              const int64_t *__restrict__ rowidx, uint16_t *__restrict__ U,
              uint16_t *__restrict__ U1) {
  extern __shared__ unsigned char sx[];
  const int c = blockIdx.y, tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blockIdx.x * kRowSpan;
  const int n0 = nmin[c], n1 = nmaxv[c];
  const uint8_t *row = x + (int64_t)c * in_stride;
  const int nbytes = kRowSpan + 1 + n1;
  for (int i = tid; i < nbytes; i += kRowThreads) {
    const int64_t g = blk0 + i;
    sx[i] = g < nsamp ? row[g] : 0;
  }
  __syncthreads();
  const int64_t tau0 = blk0 + tid * 8;
  if (tau0 >= tpad) return;
  uint32_t s[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) s[i] = 0;
  const unsigned char *b = sx + tid * 8;
  for (int n = 1; n <= n1; ++n) {
#pragma unroll
    for (int i = 0; i < 9; ++i) s[i] += b[i + n - 1];
    if (n >= n0) {
      // windows running past the end of the block are zero
      uint32_t v[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) v[i] = (tau0 + i + n <= nsamp) ? s[i] : 0u;
      const int64_t r = (rowidx[c] + (n - n0)) * tpad + tau0;
      *(uint4 *)(U + r) = make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16),
                                     v[4] | (v[5] << 16), v[6] | (v[7] << 16));
      *(uint4 *)(U1 + r) = make_uint4(v[1] | (v[2] << 16), v[3] | (v[4] << 16),
                                      v[5] | (v[6] << 16), v[7] | (v[8] << 16));
    }
  }
  if (n0 == 0) {
    const int64_t r = rowidx[c] * tpad + tau0;
    *(uint4 *)(U + r) = make_uint4(0, 0, 0, 0);
    *(uint4 *)(U1 + r) = make_uint4(0, 0, 0, 0);
  }
}

struct SearchArgs {
  const uint16_t *U, *U1;   // window rows and the same rows one sample later
  int64_t tpad;
  int32_t bufbytes;         // LDS bytes of one of the two window buffers
  const int32_t *offs;
  const GroupInfo *groups;
  const int32_t *group_begin;
  const int2 *jobs;
  const int32_t *perm;
  int32_t ntd, ntt, nchan;
  int64_t nout;
  const double *M, *S;
  int32_t nw;
  uint32_t wmask;           // bit W-1 set for every searched width W <= 32
  int8_t widx[33];          // W -> index into the width list, -1 if absent
  void *part;               // Cand[ndm][ntt]
};

typedef __attribute__((address_space(3))) void lds_void;

// s_waitcnt immediate (gfx9 layout: vmcnt in bits 3:0 and 15:14, expcnt in 6:4,
// lgkmcnt in 11:8) waiting for all vector memory operations, the direct-to-LDS
// copies included.  Issued through the builtin, not inline asm, so that the
// compiler's own wait insertion knows the counter is zero afterwards.
constexpr unsigned kWaitVm0 = 0x0f70;

// Read-only tables read through the constant address space: their fields become
// scalar loads, which do not share the vector memory counter with the direct
// global-to-LDS copies (the compiler cannot prove on its own that those copies
// leave the tables untouched).
__device__ __forceinline__ int32_t ldc(const int32_t *p, int64_t i) {
  return ((const __attribute__((address_space(4))) int32_t *)p)[i];
}

// The descriptor is read with one scalar load, so that using any field waits for
// all of them (a field read later would otherwise leave a scalar load in flight,
// forcing every LDS wait in between to wait for all outstanding reads).
__device__ __forceinline__ GroupInfo load_group(const GroupInfo *groups, int g) {
  static_assert(sizeof(GroupInfo) == 8 * sizeof(int32_t), "GroupInfo layout");
  typedef int32_t i32x8 __attribute__((ext_vector_type(8)));
  const i32x8 v = *(const __attribute__((address_space(4))) i32x8 *)(groups + g);
  GroupInfo gi;
  gi.job_begin = v[0];
  gi.njobs = v[1];
  gi.lw = v[2];
  gi.c_begin = v[3];
  gi.c_count = v[4];
  gi.flush = v[5];
  gi.inv_nchunk = v[6];
  gi.pad1 = 0;
  return gi;
}

// Buffer descriptor word 3 for raw (unformatted, unswizzled) 32-bit buffers.
constexpr int kBufWord3 = 0x00020000;

// Starts the copy of group gi's windows into one LDS buffer: copy A of a window
// (aligned to its first sample) and copy B (one sample later), each from the row
// parity whose start is dword-aligned.  Whole windows go to waves; lanes move
// 16-byte chunks with direct buffer-to-LDS loads, which complete asynchronously
// (the caller waits on the vector memory counter before its barrier).  Each
// window copy gets its own buffer descriptor covering exactly that copy, so a
// read past it returns zeros instead of touching other memory.
template <int NW, typename Args>
__device__ __forceinline__ void stage_group(Args &a, const GroupInfo &gi, int64_t t0, int wave,
                                            int lane, unsigned char *buf) {
  const int nchunk = gi.lw >> 3;
  for (int j = wave; j < gi.njobs; j += NW) {
    const int32_t *jp = (const int32_t *)(a.jobs + gi.job_begin + j);
    const int jrow = ldc(jp, 0), jstart = ldc(jp, 1);
    const int64_t e0 = (int64_t)jstart + t0;
    const int64_t base = (int64_t)jrow * a.tpad + (e0 & ~(int64_t)1);
    const bool odd = (e0 & 1) != 0;
    const uint16_t *srcA = (odd ? a.U1 : a.U) + base;        // U[e0 ...]
    const uint16_t *srcB = odd ? a.U + base + 2 : a.U1 + base;  // U[e0 + 1 ...]
    const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc((void *)srcA, (short)0, 2 * gi.lw, kBufWord3);
    const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc((void *)srcB, (short)0, 2 * gi.lw, kBufWord3);
    unsigned char *rowA = buf + j * 4 * gi.lw;
    unsigned char *rowB = rowA + 2 * gi.lw;
    for (int k = 0; 64 * k < nchunk; ++k) {
      const int ch = lane + 64 * k;
      if (ch < nchunk) {
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rA, (lds_void *)(rowA + 1024 * k), 16, 16 * ch, 0, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rB, (lds_void *)(rowB + 1024 * k), 16, 16 * ch, 0, 0, 0);
      }
    }
  }
}

// LDS read offset of (trial trial0 + lane / cc, channel c_begin + lane % cc) for the
// first DPW * cc lanes; broadcast later with v_readlane.
template <int DPW, typename Args>
__device__ __forceinline__ int group_offsets(Args &a, const GroupInfo &gi, int trial0, int lane) {
  const int cc = gi.c_count;
  int o = 0;
  if (lane < DPW * cc) {
    const int jj = lane / cc, c = lane - jj * cc;
    o = a.offs[(int64_t)(trial0 + jj) * a.nchan + gi.c_begin + c];
  }
  return o;
}

// One (DM tile, time tile) of the fused search: channel-group loop, then the
// boxcar stage.  Shared by the one-plan kernel and the multi-beam kernel.
template <int DPW, int R2, int NW, typename Args>
__device__ __forceinline__ void search_tile(Args &a, const int tt, const int td,
                                            unsigned char *lds) {
  constexpr int TY = 128 * R2, TT = tile_step(R2), DT = NW * DPW, SP = TY / 64;
  constexpr int YROW = TY + kHalo + 4;   // ints per wave for the boxcar stage
  static_assert(TT % SP == 0 && TY - TT >= 31, "tile step");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t t0 = (int64_t)tt * TT;

  int acc[DPW][2 * R2];
  uint32_t a16[DPW][R2];
#pragma unroll
  for (int j = 0; j < DPW; ++j) {
#pragma unroll
    for (int r = 0; r < 2 * R2; ++r) acc[j][r] = 0;
#pragma unroll
    for (int r = 0; r < R2; ++r) a16[j][r] = 0;
  }

  const int gb = ldc(a.group_begin, td), ge = ldc(a.group_begin, td + 1);
  const int trial0 = td * DT + wave * DPW;
  // Software pipeline over channel groups: while the waves accumulate group g from
  // one LDS buffer, the windows of group g + 1 stream into the other.
  int myoff;
  {
    const GroupInfo g0 = load_group(a.groups, gb);
    myoff = group_offsets<DPW>(a, g0, trial0, lane);
    stage_group<NW>(a, g0, t0, wave, lane, lds);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
  }
  for (int g = gb; g < ge; ++g) {
    const GroupInfo gi = load_group(a.groups, g);
    const int cc = gi.c_count;
    const int par = (g - gb) & 1;
    int nextoff = 0;
    if (g + 1 < ge) {
      const GroupInfo gn = load_group(a.groups, g + 1);
      nextoff = group_offsets<DPW>(a, gn, trial0, lane);
      stage_group<NW>(a, gn, t0, wave, lane, lds + (par ^ 1) * a.bufbytes);
    }
    // ---- accumulate: per trial, per channel, R2 aligned dword reads (pairs of
    // them 256 bytes apart are merged into one two-address read, so one LDS
    // instruction moves 512 bytes per wave).  Channels go in chunks of CH, so that
    // a chunk keeps 12 reads in flight: the LDS counter holds at most 15, and the
    // adds can then wait for the reads one at a time.
    constexpr int CH = 24 / R2;
    static_assert(CH * R2 == 24, "chunk of 12 two-address reads");
    const unsigned char *lbase = lds + par * a.bufbytes + lane * 4;
#pragma unroll
    for (int j = 0; j < DPW; ++j) {
      int c = 0;
      const int jb = j * cc;
      for (; c + CH <= cc; c += CH) {
        const unsigned char *pc[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) pc[q] = lbase + __builtin_amdgcn_readlane(myoff, jb + c + q);
#pragma unroll
        for (int q = 0; q < CH; ++q)
#pragma unroll
          for (int r = 0; r < R2; ++r)
            a16[j][r] = pk_add_u16(a16[j][r], *(const uint32_t *)(pc[q] + 256 * r));
      }
      for (; c < cc; ++c) {
        const unsigned char *pp = lbase + __builtin_amdgcn_readlane(myoff, jb + c);
#pragma unroll
        for (int r = 0; r < R2; ++r) a16[j][r] = pk_add_u16(a16[j][r], *(const uint32_t *)(pp + 256 * r));
      }
    }
    if (gi.flush) {
#pragma unroll
      for (int j = 0; j < DPW; ++j) {
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          acc[j][2 * r] += (int)(a16[j][r] & 0xffffu);
          acc[j][2 * r + 1] += (int)(a16[j][r] >> 16);
          a16[j][r] = 0;
        }
      }
    }
    // the next group's windows and offsets have landed; this group's reads are done
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
    myoff = nextoff;
  }

  // ---- boxcar search, one trial of each wave at a time.  Each lane owns SP
  // consecutive starts of the tile.  Every wave transposes its series through its
  // own LDS rows, so no workgroup barrier is needed until the stage ends (the
  // group loop ended with one, so the window buffers are free).
  int *Yw = (int *)lds + wave * (YROW + 32);
  CandRec *part = (CandRec *)a.part;
#pragma unroll
  for (int j = 0; j < DPW; ++j) {
    const int dg = a.perm[td * DT + wave * DPW + j];
#pragma unroll
    for (int r = 0; r < R2; ++r)
      *(int2 *)(Yw + 2 * lane + 128 * r) = make_int2(acc[j][2 * r], acc[j][2 * r + 1]);
    const CandRec rec = boxcar_row<SP>(Yw, lane, t0, TT, a.nout, dg, a.wmask, a.nw, a.M, a.S);
    if (dg >= 0 && lane == 0) part[(int64_t)dg * a.ntt + tt] = rec;
  }
  __syncthreads();   // LDS may be reused by whatever runs next in this workgroup
}

template <int DPW, int R2, int NW>
__global__ void __launch_bounds__(64 * NW)
k_search(SearchArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  // XCD-aware tile order: blocks b = x (mod 8) all run on XCD x; give XCD x a
  // contiguous run of tiles in time-major order.
  const int nb = a.ntd * a.ntt;
  const int b = blockIdx.x;
  const int xcd = b & 7, k = b >> 3, q = nb >> 3, rem = nb & 7;
  const int L = xcd * q + min(xcd, rem) + k;
  const int tt = L / a.ntd, td = L - tt * a.ntd;
  search_tile<DPW, R2, NW>(a, tt, td, lds);
}

// Multi-beam search: one workgroup per (beam, tile).  Beam b owns the blocks
// [base[b], base[b] + nb_b rounded up to 8), base[b] a multiple of 8, so that
// block i of a beam runs on XCD i mod 8 (blocks are dealt to the 8 XCDs
// round-robin) and the beam's tiles take the single-plan kernel's XCD-aware order:
// all XCDs work through one beam at a time, each on a contiguous run of its time
// tiles.  Blocks past a beam's tile count exit at once.
template <int DPW, int R2, int NW>
__global__ void __launch_bounds__(64 * NW)
k_search_batch(const SearchArgs *__restrict__ beams, const int32_t *__restrict__ base,
               int32_t nbeam) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const int bi = blockIdx.x;
  int lo = 0, hi = nbeam - 1;   // last beam whose first block <= bi
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ldc(base, mid) <= bi) lo = mid; else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  // the argument table is read through the constant address space, so that its
  // fields are scalar loads
  typedef const __attribute__((address_space(4))) SearchArgs CArgs;
  CArgs &a = ((CArgs *)beams)[lo];
  const int nb = a.ntd * a.ntt;
  const int kl = bi - ldc(base, lo);
  const int xcd = kl & 7, k = kl >> 3, q = nb >> 3, rem = nb & 7;
  if (k >= q + (xcd < rem ? 1 : 0)) return;
  const int L = xcd * q + min(xcd, rem) + k;
  const int tt = L / a.ntd, td = L - tt * a.ntd;
  search_tile<DPW, R2, NW>(a, tt, td, lds);
}


}  // namespace

// ------------------------------------------------------------------------------
// Host: tables
// ------------------------------------------------------------------------------
static void build_rows(const dedisp_plan_s *p, TiledTables *T) {
  const int C = p->nchan, D = p->ndm;
  T->nmin.assign(C, INT32_MAX);
  T->nmax.assign(C, 0);
  for (int d = 0; d < D; ++d)
    for (int c = 0; c < C; ++c) {
      const int n = p->ntap[(size_t)d * C + c];
      T->nmin[c] = std::min(T->nmin[c], n);
      T->nmax[c] = std::max(T->nmax[c], n);
    }
  T->rowidx.assign(C, 0);
  int64_t r = 0;
  T->nmax_all = 0;
  for (int c = 0; c < C; ++c) {
    T->rowidx[c] = r;
    r += T->nmax[c] - T->nmin[c] + 1;
    T->nmax_all = std::max(T->nmax_all, T->nmax[c]);
  }
  T->nrows = r;
}

// Groups of channels per DM tile, their LDS window layout and the per-(trial,
// channel) LDS read offsets.  Returns false if some channel's windows alone exceed
// the LDS budget or a single run could wrap a uint16 lane.
static bool build_cfg_budget(const dedisp_plan_s *p, const TiledTables &T, int ci, int budget,
                             TiledCfgTables &out);

static bool build_cfg(const dedisp_plan_s *p, const TiledTables &T, int ci, TiledCfgTables &out) {
  for (int budget : kStageBudgets) {
    budget = budget * kCfgs[ci].nw / 4;
    if (2 * budget > kMaxLds) break;
    if (build_cfg_budget(p, T, ci, budget, out)) return true;
  }
  return false;
}

static bool build_cfg_budget(const dedisp_plan_s *p, const TiledTables &T, int ci, int budget,
                             TiledCfgTables &out) {
  const TileCfg cf = kCfgs[ci];
  const int C = p->nchan, D = p->ndm;
  const int DT = cf.nw * cf.dpw, TY = 128 * cf.r2;
  out = TiledCfgTables();
  out.dt = DT;
  out.ty = TY;
  out.tt = tile_step(cf.r2);
  std::vector<int32_t> order(D);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p->dm[a] < p->dm[b]; });
  const int ntd = (D + DT - 1) / DT;
  out.ntd = ntd;
  out.perm.assign((size_t)ntd * DT, -1);
  for (int i = 0; i < D; ++i) out.perm[i] = order[i];
  out.offs.assign((size_t)ntd * DT * C, 0);
  out.group_begin.assign(ntd + 1, 0);
  int lds_max = 0;
  std::vector<int> tr(DT);
  std::vector<int64_t> run(DT);
  for (int td = 0; td < ntd; ++td) {
    out.group_begin[td] = (int)out.groups.size();
    for (int j = 0; j < DT; ++j) {
      const int d = out.perm[(size_t)td * DT + j];
      tr[j] = d >= 0 ? d : out.perm[(size_t)td * DT];
    }
    std::fill(run.begin(), run.end(), 0);
    int c = 0;
    while (c < C) {
      GroupInfo gi{};
      gi.job_begin = (int)out.jobs.size();
      gi.c_begin = c;
      int span = 0, nrows_g = 0, ccount = 0;
      while (c < C) {
        int smin = INT32_MAX, smax = INT32_MIN;
        std::vector<int> ns;
        bool over = false;
        for (int j = 0; j < DT; ++j) {
          const int s = p->start[(size_t)tr[j] * C + c], n = p->ntap[(size_t)tr[j] * C + c];
          smin = std::min(smin, s);
          smax = std::max(smax, s);
          if (std::find(ns.begin(), ns.end(), n) == ns.end()) ns.push_back(n);
          if (run[j] + 255LL * n > 65535) over = true;
        }
        const int nspan = std::max(span, smax - smin);
        const int lw = ((TY + nspan + 2) + 7) & ~7;
        const int bytes = (nrows_g + (int)ns.size()) * 4 * lw;
        if (ccount == 0 && (bytes > budget || over)) return false;
        if (bytes > budget || over || ccount >= 64 / cf.dpw) break;
        span = nspan;
        nrows_g += (int)ns.size();
        for (int j = 0; j < DT; ++j) run[j] += 255LL * p->ntap[(size_t)tr[j] * C + c];
        ++ccount;
        ++c;
      }
      const int lw = ((TY + span + 2) + 7) & ~7;
      gi.lw = lw;
      {
        const float inv = 1.0f / (float)(lw / 8);
        std::memcpy(&gi.inv_nchunk, &inv, sizeof(float));
      }
      gi.c_count = ccount;
      bool flush = c >= C;
      if (!flush)
        for (int j = 0; j < DT; ++j)
          if (run[j] + 255LL * p->ntap[(size_t)tr[j] * C + c] > 65535) flush = true;
      gi.flush = flush ? 1 : 0;
      if (flush) std::fill(run.begin(), run.end(), 0);
      // rows of the group in channel order, each (c, n) once
      int ri = 0;
      for (int cc = gi.c_begin; cc < gi.c_begin + ccount; ++cc) {
        int smin = INT32_MAX;
        std::vector<int> ns;
        for (int j = 0; j < DT; ++j) {
          smin = std::min(smin, p->start[(size_t)tr[j] * C + cc]);
          const int n = p->ntap[(size_t)tr[j] * C + cc];
          if (std::find(ns.begin(), ns.end(), n) == ns.end()) ns.push_back(n);
        }
        for (size_t k = 0; k < ns.size(); ++k) {
          const int64_t row = T.rowidx[cc] + (ns[k] - T.nmin[cc]);
          out.jobs.push_back(make_int2((int)row, smin));
        }
        for (int j = 0; j < DT; ++j) {
          const int s = p->start[(size_t)tr[j] * C + cc], n = p->ntap[(size_t)tr[j] * C + cc];
          const int k = (int)(std::find(ns.begin(), ns.end(), n) - ns.begin());
          const int e = s - smin;
          const int odd = e & 1;
          out.offs[((size_t)td * DT + j) * C + cc] = (ri + k) * 4 * lw + (odd ? 2 * lw : 0) + 2 * (e - odd);
        }
        ri += (int)ns.size();
      }
      gi.njobs = ri;
      lds_max = std::max(lds_max, ri * 4 * lw);
      out.groups.push_back(gi);
    }
  }
  out.group_begin[ntd] = (int)out.groups.size();
  out.ngroups = (int)out.groups.size();
  out.bufbytes = (lds_max + 15) & ~15;
  out.lds_bytes = std::max(2 * out.bufbytes, cf.nw * (TY + kHalo + 4 + 32) * 4);
  out.ok = true;
  return true;
}

template <typename T>
static hipError_t upload(T **dst, const std::vector<T> &v) {
  hipError_t e = dev_malloc((void **)dst, std::max<size_t>(1, v.size()) * sizeof(T));
  if (e != hipSuccess) return e;
  if (v.empty()) return hipSuccess;
  return hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Search candidates: the kNumCfgs shapes of k_search, then the shapes of the
// matrix-core search (kernels_mfma.hip).  Without a choice the order of kUntunedOrder
// applies.
static int num_candidates() { return kNumCfgs + mfma_search_count(); }

static int cfg_index(const dedisp_plan_s *p) {
  return (p->tile_choice >= 0 && p->tile_choice < num_candidates()) ? p->tile_choice : kNumCfgs;
}

// The k_search shape of a choice (the multi-beam kernel has only those).
static int valu_index(const dedisp_plan_s *p) {
  const int ci = cfg_index(p);
  return ci < kNumCfgs ? ci : kDefaultCfg;
}

// Tables for configuration ci, built and uploaded on first use.  Caller holds p->mu.
static dedisp_status ensure_cfg(dedisp_plan p, int ci, TiledCfgTables **out) {
  if (!p->tiled) {
    p->tiled = new (std::nothrow) TiledTables;
    if (!p->tiled) return fail(DEDISP_ERR_OOM, "host allocation failed");
    build_rows(p, p->tiled);
    DD_HIP(upload(&p->tiled->d_nmin, p->tiled->nmin));
    DD_HIP(upload(&p->tiled->d_nmax, p->tiled->nmax));
    DD_HIP(upload(&p->tiled->d_rowidx, p->tiled->rowidx));
  }
  TiledCfgTables &c = p->tiled->cfg[ci];
  if (!c.ok && c.dt == 0) {
    if (!build_cfg(p, *p->tiled, ci, c)) {
      c.dt = -1;   // remember: not supported
    } else {
      DD_HIP(upload(&c.d_offs, c.offs));
      DD_HIP(upload(&c.d_groups, c.groups));
      DD_HIP(upload(&c.d_group_begin, c.group_begin));
      DD_HIP(upload(&c.d_jobs, c.jobs));
      DD_HIP(upload(&c.d_perm, c.perm));
    }
  }
  *out = c.ok ? &c : nullptr;
  return DEDISP_OK;
}

struct Layout {
  int64_t ntt, tpad, nrows;
  size_t off_part, off_u, total;
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static Layout layout(const dedisp_plan_s *p, int ci, int32_t nw, int64_t nout, int64_t nrows) {
  const TileCfg cf = kCfgs[ci];
  const int TY = 128 * cf.r2, TT = tile_step(cf.r2);
  Layout L;
  L.ntt = (nout + TT - 1) / TT;
  L.tpad = (((L.ntt - 1) * TT + TY + 2 * (int64_t)p->max_span + 32) + 7) & ~(int64_t)7;
  L.nrows = nrows;
  const size_t tables = align256(2 * sizeof(double) * (size_t)p->ndm * nw);
  L.off_part = tables;
  L.off_u = L.off_part + align256(sizeof(CandRec) * (size_t)p->ndm * L.ntt);
  L.total = L.off_u + align256(2 * sizeof(uint16_t) * (size_t)nrows * L.tpad);
  return L;
}

size_t search_work_bytes(const dedisp_plan_s *p, int32_t nw, int64_t nout) {
  if (p->wmode != DEDISP_W_UNIT) return 0;
  const int64_t nrows = p->window_rows;
  size_t best = mfma_search_work_bytes(p, nw, nout);
  for (int ci = 0; ci < kNumCfgs; ++ci) best = std::max(best, layout(p, ci, nw, nout, nrows).total);
  return best;
}

bool search_supported(const dedisp_plan_s *p, const WidthList &wl) {
  if (p->wmode != DEDISP_W_UNIT) return false;
  if (wl.w[wl.n - 1] > 32) return false;
  if (p->max_ntap > 257) return false;
  // the register prefix of the boxcar stage sums up to SP + 32 <= 48 outputs and
  // must stay below 2^30; invalid entries are placed near -2^29, so every
  // difference of two entries fits in int32
  const double ymax = 255.0 * (double)p->sum_max_ntap;
  if (ymax * 49.0 >= 1073741824.0) return false;
  return true;
}

// Workgroups may take more than the default 64 KiB of LDS: raise each kernel's
// limit once per device.
static hipError_t allow_lds(const void *fn, bool *done, std::mutex *mu) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= 64) return e;
  std::lock_guard<std::mutex> lk(*mu);
  if (!done[dev]) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    if (e == hipSuccess) done[dev] = true;
  }
  return e;
}

template <int DPW, int R2, int NW>
static hipError_t launch_cfg(const SearchArgs &a, int nblocks, int lds, hipStream_t s) {
  static bool done[64] = {};
  static std::mutex mu;
  hipError_t e = allow_lds((const void *)k_search<DPW, R2, NW>, done, &mu);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_search<DPW, R2, NW>), dim3(nblocks), dim3(64 * NW), lds, s, a);
  return hipGetLastError();
}

static hipError_t launch_search_kernel(int ci, const SearchArgs &a, int nblocks, int lds,
                                       hipStream_t s) {
  switch (ci) {
#define DD_CFG_CASE(i, d, r, w) \
  case i: return launch_cfg<d, r, w>(a, nblocks, lds, s);
    DD_TILE_CONFIGS(DD_CFG_CASE)
#undef DD_CFG_CASE
    default: return hipErrorInvalidValue;
  }
}

// The tile kernel's arguments for one plan and one block (pointers into `work`,
// or the window rows at u_rows when given), without launching anything.  Returns
// DEDISP_ERR_UNSUPPORTED when the tiled kernel cannot take this plan.
static dedisp_status describe_tiled(dedisp_plan p, int ci, int64_t nout, const WidthList &wl,
                                    void *work, uint16_t *u_rows, SearchArgs *out,
                                    TiledCfgTables **cfg_out = nullptr, Layout *lay_out = nullptr) {
  TiledCfgTables *cfg = nullptr;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    dedisp_status st = ensure_cfg(p, ci, &cfg);
    if (st != DEDISP_OK) return st;
  }
  if (!cfg) return DEDISP_ERR_UNSUPPORTED;
  const TiledTables &T = *p->tiled;
  const Layout L = layout(p, ci, wl.n, nout, T.nrows);
  if (L.ntt * (int64_t)cfg->ntd > INT32_MAX / 2) return DEDISP_ERR_UNSUPPORTED;
  double *M = (double *)work;
  uint16_t *U = u_rows ? u_rows : (uint16_t *)((char *)work + L.off_u);
  SearchArgs a{};
  a.U = U;
  a.U1 = U + (size_t)T.nrows * L.tpad;
  a.tpad = L.tpad;
  a.bufbytes = cfg->bufbytes;
  a.offs = cfg->d_offs;
  a.groups = cfg->d_groups;
  a.group_begin = cfg->d_group_begin;
  a.jobs = cfg->d_jobs;
  a.perm = cfg->d_perm;
  a.ntd = cfg->ntd;
  a.ntt = (int32_t)L.ntt;
  a.nchan = p->nchan;
  a.nout = nout;
  a.M = M;
  a.S = M + (size_t)p->ndm * wl.n;
  a.nw = wl.n;
  a.wmask = 0;
  for (int i = 0; i <= 32; ++i) a.widx[i] = -1;
  for (int i = 0; i < wl.n; ++i) {
    a.wmask |= 1u << (wl.w[i] - 1);
    a.widx[wl.w[i]] = (int8_t)i;
  }
  a.part = (char *)work + L.off_part;
  *out = a;
  if (cfg_out) *cfg_out = cfg;
  if (lay_out) *lay_out = L;
  return DEDISP_OK;
}

// Launches the per-block preparation of one plan (noise tables, window rows) into
// `work` (rows at u_rows when given) and fills the tile kernel's arguments.
// Returns DEDISP_ERR_UNSUPPORTED (without launching anything) when the tiled
// kernel cannot take this plan.
static dedisp_status prepare_tiled(dedisp_plan p, int ci, const uint8_t *x, int64_t nsamp,
                                   int64_t in_stride, int64_t nout, const WidthList &wl,
                                   const double *mu, const double *sigma, void *work,
                                   hipStream_t s, SearchArgs *out, TiledCfgTables **cfg_out,
                                   Layout *lay_out, uint16_t *u_rows = nullptr) {
  SearchArgs a;
  TiledCfgTables *cfg = nullptr;
  Layout L;
  dedisp_status st = describe_tiled(p, ci, nout, wl, work, u_rows, &a, &cfg, &L);
  if (st != DEDISP_OK) return st;
  const TiledTables &T = *p->tiled;
  DD_HIP(launch_norm(p, wl, mu, sigma, (double *)a.M, (double *)a.S, s));
  {
    const dim3 g((unsigned)((L.tpad + kRowSpan - 1) / kRowSpan), (unsigned)p->nchan);
    const int shm = kRowSpan + T.nmax_all + 16;
    hipLaunchKernelGGL(k_window_rows, g, dim3(kRowThreads), shm, s, x, in_stride, nsamp, L.tpad,
                       T.d_nmin, T.d_nmax, T.d_rowidx, (uint16_t *)a.U, (uint16_t *)a.U1);
    DD_HIP(hipGetLastError());
  }
  *out = a;
  *cfg_out = cfg;
  *lay_out = L;
  return DEDISP_OK;
}

static dedisp_status search_ci(dedisp_plan p, int ci, const uint8_t *x, int64_t nsamp,
                               int64_t in_stride, int64_t nout, const WidthList &wl,
                               const double *mu, const double *sigma, double *snr, int32_t *t,
                               int32_t *w, void *work, hipStream_t s) {
  if (ci >= kNumCfgs) {
    const dedisp_status st = run_search_mfma(p, ci - kNumCfgs, x, nsamp, in_stride, nout, wl, mu,
                                             sigma, snr, t, w, work, s);
    if (st == DEDISP_OK) p->last_search_tile = ci;
    return st;
  }
  SearchArgs a;
  TiledCfgTables *cfg = nullptr;
  Layout L;
  dedisp_status st = prepare_tiled(p, ci, x, nsamp, in_stride, nout, wl, mu, sigma, work, s, &a,
                                   &cfg, &L);
  if (st != DEDISP_OK) return st;
  KernelTimer kt(p, s);
  DD_HIP(kt.begin());
  DD_HIP(launch_search_kernel(ci, a, cfg->ntd * (int)L.ntt, cfg->lds_bytes, s));
  DD_HIP(kt.end());
  DD_HIP(launch_reduce(p->ndm, (int32_t)L.ntt, a.part, snr, t, w, s));
  p->last_search_tile = ci;
  return DEDISP_OK;
}

// Without a tuned or forced shape: the matrix-core shape of two workgroups per CU (32
// trials x 1024 outputs each, the faster one with the direct staging), else the one of one
// workgroup per CU, else the packed-add default.
static const int kUntunedOrder[] = {kNumCfgs + 1, kNumCfgs, kDefaultCfg};

dedisp_status run_search_tiled(dedisp_plan p, const uint8_t *x, int64_t nsamp, int64_t in_stride,
                               int64_t nout, const WidthList &wl, const double *mu,
                               const double *sigma, double *snr, int32_t *t, int32_t *w,
                               void *work, hipStream_t s) {
  if (p->tile_choice >= 0 && p->tile_choice < num_candidates())
    return search_ci(p, p->tile_choice, x, nsamp, in_stride, nout, wl, mu, sigma, snr, t, w,
                     work, s);
  dedisp_status st = DEDISP_ERR_UNSUPPORTED;
  for (const int ci : kUntunedOrder) {
    if (ci >= num_candidates()) continue;
    st = search_ci(p, ci, x, nsamp, in_stride, nout, wl, mu, sigma, snr, t, w, work, s);
    if (st != DEDISP_ERR_UNSUPPORTED) break;
  }
  return st;
}


}  // namespace dd

extern "C" {

dedisp_status dedisp_set_tile(dedisp_plan p, int32_t tile) {
  if (!p) return dd::fail(DEDISP_ERR_INVALID_ARG, "null plan");
  if (tile < -2 || tile >= dd::num_candidates())
    return dd::fail(DEDISP_ERR_INVALID_ARG, "tile index out of range");
  p->tile_choice = tile;
  return DEDISP_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------
// Batched search over many beams: one launch over every beam's tiles, optionally
// replayed from a captured HIP graph.
// ------------------------------------------------------------------------------
struct dedisp_batch_s {
  int32_t nbeam = 0, nchan = 0, ci = 0;
  dd::MfmaBatch *mb = nullptr;      // the matrix-core path, when it takes every beam
  std::vector<dedisp_plan> plans;
  std::vector<int64_t> nsamp, nout;
  dd::WidthList wl{};
  std::vector<size_t> off;          // workspace offset of each beam
  std::vector<int64_t> out_off;     // first output row of each beam
  size_t work_bytes = 0;
  int64_t total_trials = 0, total_sums = 0;
  // Beams are searched in chunks whose window rows fit kBatchChunkRows bytes (so
  // that rows written by the preparation are still cached when the search reads
  // them); chunk k covers beams [chunk_beam[k], chunk_beam[k + 1]), its block
  // bases start at tile_begin[chunk_tb[k]] = 0, and all chunks share one rows
  // region at u_off of the workspace.
  std::vector<int32_t> tile_begin, chunk_beam, chunk_tb, chunk_grid, chunk_lds;
  std::vector<size_t> u_rel;          // rows offset of each beam inside the shared region
  size_t u_off = 0;
  int32_t *d_tile_begin = nullptr;
  dd::SearchArgs *d_args_graph = nullptr;   // argument table of the captured graph
  size_t args_off = 0;                      // workspace offset of the eager argument table
  dd::ArgStage stage;                       // pinned staging of the eager table
  // captured graph and the pointers it was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<const void *> key;
  hipStream_t cap = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

namespace dd {

template <int DPW, int R2, int NW>
static hipError_t launch_batch_cfg(const dedisp_batch_s *B, int k, const SearchArgs *table,
                                   hipStream_t s) {
  static bool done[64] = {};
  static std::mutex mu;
  hipError_t e = allow_lds((const void *)k_search_batch<DPW, R2, NW>, done, &mu);
  if (e != hipSuccess) return e;
  const int b0 = B->chunk_beam[k], b1 = B->chunk_beam[k + 1];
  hipLaunchKernelGGL((k_search_batch<DPW, R2, NW>), dim3(B->chunk_grid[k]), dim3(64 * NW),
                     B->chunk_lds[k], s, table + b0, B->d_tile_begin + B->chunk_tb[k], b1 - b0);
  return hipGetLastError();
}

static hipError_t launch_batch_kernel(const dedisp_batch_s *B, int k, const SearchArgs *table,
                                      hipStream_t s) {
  switch (B->ci) {
#define DD_CFG_CASE(i, d, r, w) \
  case i: return launch_batch_cfg<d, r, w>(B, k, table, s);
    DD_TILE_CONFIGS(DD_CFG_CASE)
#undef DD_CFG_CASE
    default: return hipErrorInvalidValue;
  }
}

// The whole per-call launch sequence: per-beam tables and window rows, the
// multi-beam search and the per-beam reductions.
// Eager calls (for_graph false) copy the argument table into the caller's workspace
// through the pinned staging buffer; a captured sequence (for_graph true) reads the
// batch's own graph table, uploaded outside the capture (it depends only on the
// pointers the graph is keyed on).  The two tables are distinct, so an eager call
// never changes what a graph replays.
static dedisp_status batch_enqueue(dedisp_batch_s *B, const void *const *in, const int64_t *stride,
                                   const double *mu, const double *sigma, double *snr, int32_t *t,
                                   int32_t *w, void *work, hipStream_t s, bool for_graph,
                                   std::vector<SearchArgs> &args) {
  if (B->mb) {
    KernelTimer kt(B->plans[0], s);
    return mfma_batch_enqueue(B->mb, in, stride, mu, sigma, snr, t, w, B->out_off, work, s,
                              for_graph, &kt);
  }
  args.assign(B->nbeam, SearchArgs{});
  uint16_t *urows = (uint16_t *)((char *)work + B->u_off);
  for (int b = 0; b < B->nbeam; ++b) {
    dedisp_status st = describe_tiled(B->plans[b], B->ci, B->nout[b], B->wl,
                                      (char *)work + B->off[b],
                                      (uint16_t *)((char *)urows + B->u_rel[b]), &args[b]);
    if (st != DEDISP_OK) return st == DEDISP_ERR_UNSUPPORTED
                                    ? fail(st, "a beam's plan cannot use the tiled search")
                                    : st;
  }
  SearchArgs *table = B->d_args_graph;
  if (!for_graph) {
    table = (SearchArgs *)((char *)work + B->args_off);
    DD_HIP(B->stage.copy(table, args.data(), sizeof(SearchArgs) * B->nbeam, s));
  }
  // chunk by chunk: the beams' noise tables and window rows (the rows region is
  // shared by all chunks: stream order keeps a chunk's search ahead of the next
  // chunk's rows), then one search launch over the chunk's tiles
  const int nchunk = (int)B->chunk_beam.size() - 1;
  KernelTimer kt(B->plans[0], s);
  for (int k = 0; k < nchunk; ++k) {
    for (int b = B->chunk_beam[k]; b < B->chunk_beam[k + 1]; ++b) {
      TiledCfgTables *cfg = nullptr;
      Layout L;
      SearchArgs a;
      dedisp_status st = prepare_tiled(B->plans[b], B->ci, (const uint8_t *)in[b], B->nsamp[b],
                                       stride[b], B->nout[b], B->wl, mu, sigma,
                                       (char *)work + B->off[b], s, &a, &cfg, &L,
                                       (uint16_t *)((char *)urows + B->u_rel[b]));
      if (st != DEDISP_OK) return st;
    }
    if (k == 0) DD_HIP(kt.begin());
    DD_HIP(launch_batch_kernel(B, k, table, s));
  }
  DD_HIP(kt.end());
  for (int b = 0; b < B->nbeam; ++b) {
    const int64_t o = B->out_off[b];
    DD_HIP(launch_reduce(B->plans[b]->ndm, args[b].ntt, args[b].part, snr + o, t + o, w + o, s));
  }
  return DEDISP_OK;
}

}  // namespace dd

extern "C" {

dedisp_status dedisp_batch_create(dedisp_batch *out, int32_t nbeam, const dedisp_plan *plans,
                                  const int64_t *nsamp, const int32_t *widths, int32_t nw) {
  using namespace dd;
  if (!out || nbeam < 1 || !plans || !nsamp || !widths) return fail(DEDISP_ERR_INVALID_ARG, "bad batch arguments");
  *out = nullptr;
  for (int b = 0; b < nbeam; ++b) {
    if (!plans[b]) return fail(DEDISP_ERR_INVALID_ARG, "null plan in batch");
    if (plans[b]->nchan != plans[0]->nchan) return fail(DEDISP_ERR_INVALID_ARG, "beams must share the channel count");
    if (plans[b]->wmode != DEDISP_W_UNIT) return fail(DEDISP_ERR_UNSUPPORTED, "batched search needs unit weights");
    if (nsamp[b] < plans[b]->max_span) return fail(DEDISP_ERR_SHAPE, "a beam is shorter than its longest run");
  }
  if (nw < 1 || nw > kMaxWidths) return fail(DEDISP_ERR_INVALID_ARG, "need 1..64 widths");
  std::vector<int32_t> wv(widths, widths + nw);
  std::sort(wv.begin(), wv.end());
  wv.erase(std::unique(wv.begin(), wv.end()), wv.end());
  if (wv.front() < 1 || wv.back() > 32) return fail(DEDISP_ERR_UNSUPPORTED, "batched search takes widths 1..32");
  dedisp_batch_s *B = new (std::nothrow) dedisp_batch_s;
  if (!B) return fail(DEDISP_ERR_OOM, "host allocation failed");
  B->nbeam = nbeam;
  B->nchan = plans[0]->nchan;
  B->plans.assign(plans, plans + nbeam);
  B->nsamp.assign(nsamp, nsamp + nbeam);
  B->wl.n = (int32_t)wv.size();
  for (int i = 0; i < B->wl.n; ++i) B->wl.w[i] = wv[i];
  B->ci = valu_index(plans[0]);
  dedisp_status st = DEDISP_OK;
  // The matrix-core kernel unless the first plan forces the packed-add kernel or the
  // general path, or no matrix-core shape takes every beam.
  const int tc = plans[0]->tile_choice;
  if (tc != -2 && (tc < 0 || tc >= kNumCfgs)) {
    for (int b = 0; b < nbeam && st == DEDISP_OK; ++b) {
      if (!search_supported(plans[b], B->wl))
        st = fail(DEDISP_ERR_UNSUPPORTED, "a beam's plan cannot use the tiled search");
      else
        st = ensure_device(plans[b]);
    }
    if (st == DEDISP_OK)
      st = mfma_batch_create(B->plans, B->nsamp, B->wl, tc >= kNumCfgs ? tc - kNumCfgs : 0, &B->mb);
    if (st != DEDISP_OK) {
      dedisp_batch_destroy(B);
      return st;
    }
    if (B->mb) {
      for (int b = 0; b < nbeam; ++b) {
        const int64_t no = nsamp[b] - plans[b]->max_span + 1;
        B->nout.push_back(no);
        B->out_off.push_back(B->total_trials);
        B->total_trials += plans[b]->ndm;
        B->total_sums += (int64_t)plans[b]->ndm * plans[b]->nchan * no;
      }
      B->work_bytes = mfma_batch_work_bytes(B->mb);
      *out = B;
      return DEDISP_OK;
    }
  }
  size_t off = 0;
  std::vector<size_t> rows;      // window-row bytes of each beam
  std::vector<int64_t> blocks;   // workgroups of each beam (a multiple of 8)
  std::vector<int> lds;          // LDS bytes per workgroup of each beam
  for (int b = 0; b < nbeam && st == DEDISP_OK; ++b) {
    dedisp_plan p = plans[b];
    const int64_t no = nsamp[b] - p->max_span + 1;
    B->nout.push_back(no);
    if (!search_supported(p, B->wl)) {
      st = fail(DEDISP_ERR_UNSUPPORTED, "a beam's plan cannot use the tiled search");
      break;
    }
    if ((st = ensure_device(p)) != DEDISP_OK) break;
    TiledCfgTables *cfg = nullptr;
    {
      std::lock_guard<std::mutex> lk(p->mu);
      st = ensure_cfg(p, B->ci, &cfg);
    }
    if (st != DEDISP_OK) break;
    if (!cfg) {
      st = fail(DEDISP_ERR_UNSUPPORTED, "a beam's plan cannot use the tiled search");
      break;
    }
    const Layout L = layout(p, B->ci, B->wl.n, no, p->tiled->nrows);
    B->off.push_back(off);
    off += (L.off_u + 255) & ~(size_t)255;   // noise tables and partial results
    rows.push_back((L.total - L.off_u + 255) & ~(size_t)255);
    B->out_off.push_back(B->total_trials);
    B->total_trials += p->ndm;
    B->total_sums += (int64_t)p->ndm * p->nchan * no;
    const int64_t nit = ((int64_t)cfg->ntd * L.ntt + 7) & ~(int64_t)7;   // blocks of this beam
    if (nit > INT32_MAX / 2) {
      st = fail(DEDISP_ERR_UNSUPPORTED, "too many tiles in one beam");
      break;
    }
    blocks.push_back(nit);
    lds.push_back(cfg->lds_bytes);
  }
  if (st == DEDISP_OK) {
    // chunks of consecutive beams whose rows fit kBatchChunkRows (at least one beam)
    size_t rows_max = 0, rows_in = 0;
    int64_t items = 0;
    int lds_in = 0;
    B->chunk_beam.push_back(0);
    B->chunk_tb.push_back(0);
    B->tile_begin.push_back(0);
    for (int b = 0; b < nbeam; ++b) {
      if (b > B->chunk_beam.back() &&
          (rows_in + rows[b] > kBatchChunkRows || items + blocks[b] > INT32_MAX / 2)) {
        B->chunk_grid.push_back((int32_t)items);
        B->chunk_lds.push_back(lds_in);
        B->chunk_beam.push_back(b);
        B->chunk_tb.push_back((int32_t)B->tile_begin.size());
        B->tile_begin.push_back(0);
        rows_in = 0;
        items = 0;
        lds_in = 0;
      }
      lds_in = std::max(lds_in, lds[b]);
      B->u_rel.push_back(rows_in);
      rows_in += rows[b];
      rows_max = std::max(rows_max, rows_in);
      items += blocks[b];
      B->tile_begin.push_back((int32_t)items);
    }
    B->chunk_grid.push_back((int32_t)items);
    B->chunk_lds.push_back(lds_in);
    B->chunk_beam.push_back(nbeam);
    B->u_off = off;
    off += rows_max;
  }
  B->args_off = (off + 255) & ~(size_t)255;
  B->work_bytes = B->args_off + sizeof(SearchArgs) * nbeam;
  if (st == DEDISP_OK) {
    hipError_t e = upload(&B->d_tile_begin, B->tile_begin);
    if (e == hipSuccess) e = dev_malloc((void **)&B->d_args_graph, sizeof(SearchArgs) * nbeam);
    if (e != hipSuccess) st = hip_fail(e, "batch setup");
  }
  if (st != DEDISP_OK) {
    dedisp_batch_destroy(B);
    return st;
  }
  *out = B;
  return DEDISP_OK;
}

dedisp_status dedisp_batch_destroy(dedisp_batch B) {
  if (!B) return dd::fail(DEDISP_ERR_INVALID_ARG, "null batch");
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  if (B->ev_in) (void)hipEventDestroy(B->ev_in);
  if (B->ev_out) (void)hipEventDestroy(B->ev_out);
  B->stage.release();
  (void)hipFree(B->d_tile_begin);
  (void)hipFree(B->d_args_graph);
  dd::mfma_batch_free(B->mb);
  delete B;
  return DEDISP_OK;
}

dedisp_status dedisp_batch_work_bytes(dedisp_batch B, size_t *bytes) {
  if (!B || !bytes) return dd::fail(DEDISP_ERR_INVALID_ARG, "null argument");
  *bytes = B->work_bytes;
  return DEDISP_OK;
}

dedisp_status dedisp_batch_info(dedisp_batch B, int64_t *total_trials, int64_t *total_sums) {
  if (!B) return dd::fail(DEDISP_ERR_INVALID_ARG, "null batch");
  if (total_trials) *total_trials = B->total_trials;
  if (total_sums) *total_sums = B->total_sums;
  return DEDISP_OK;
}

dedisp_status dedisp_batch_run(dedisp_batch B, const void *const *d_in, const int64_t *in_stride,
                               const double *d_chan_mean, const double *d_chan_sigma,
                               double *d_snr, int32_t *d_t, int32_t *d_w, void *d_work,
                               size_t work_bytes, int32_t use_graph, void *stream) {
  using namespace dd;
  if (!B || !d_in || !in_stride || !d_chan_mean || !d_chan_sigma || !d_snr || !d_t || !d_w || !d_work)
    return fail(DEDISP_ERR_INVALID_ARG, "null argument");
  if (work_bytes < B->work_bytes) return fail(DEDISP_ERR_INVALID_ARG, "workspace too small");
  for (int b = 0; b < B->nbeam; ++b)
    if (!d_in[b] || in_stride[b] < B->nsamp[b]) return fail(DEDISP_ERR_INVALID_ARG, "bad beam input");
  hipStream_t s = (hipStream_t)stream;
  std::vector<SearchArgs> args;
  if (!use_graph)
    return batch_enqueue(B, d_in, in_stride, d_chan_mean, d_chan_sigma, d_snr, d_t, d_w, d_work, s,
                         false, args);
  // Graph path: capture once per set of pointers on a private stream, then replay.
  std::vector<const void *> key(d_in, d_in + B->nbeam);
  for (int b = 0; b < B->nbeam; ++b) key.push_back((const void *)(intptr_t)in_stride[b]);
  key.insert(key.end(), {d_chan_mean, d_chan_sigma, d_snr, d_t, d_w, d_work});
  if (!B->cap) {
    DD_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    DD_HIP(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
    DD_HIP(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
  }
  if (!B->gexec || key != B->key) {
    if (B->gexec) {
      (void)hipGraphExecDestroy(B->gexec);
      B->gexec = nullptr;
    }
    if (B->graph) {
      (void)hipGraphDestroy(B->graph);
      B->graph = nullptr;
    }
    // Anything still running from an earlier replay must not see a new table.
    DD_HIP(hipStreamSynchronize(B->cap));
    DD_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    // from here on the capture is ended on every path; instrumentation events
    // are not captured
    std::vector<hipEvent_t> e0, e1;
    e0.swap(B->plans[0]->ev_start);
    e1.swap(B->plans[0]->ev_stop);
    dedisp_status st = batch_enqueue(B, d_in, in_stride, d_chan_mean, d_chan_sigma, d_snr, d_t, d_w,
                                     d_work, B->cap, true, args);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(B->cap, &g);
    e0.swap(B->plans[0]->ev_start);
    e1.swap(B->plans[0]->ev_stop);
    if (st != DEDISP_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
    B->graph = g;
    DD_HIP(hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0));
    if (B->mb) {
      const dedisp_status su = mfma_batch_upload(B->mb);
      if (su != DEDISP_OK) return su;
    } else {
      DD_HIP(hipMemcpy(B->d_args_graph, args.data(), sizeof(SearchArgs) * B->nbeam,
                       hipMemcpyHostToDevice));
    }
    B->key = key;
  }
  DD_HIP(hipEventRecord(B->ev_in, s));
  DD_HIP(hipStreamWaitEvent(B->cap, B->ev_in, 0));
  DD_HIP(hipGraphLaunch(B->gexec, B->cap));
  DD_HIP(hipEventRecord(B->ev_out, B->cap));
  DD_HIP(hipStreamWaitEvent(s, B->ev_out, 0));
  return DEDISP_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------
// Autotuner: time every tile shape of the fused search on the caller's block and
// keep the fastest.  Results are cached per (device architecture, plan shape,
// table hash, block length, widths) in the text file named by DEDISP_TUNE_CACHE.
// ------------------------------------------------------------------------------
namespace dd {

static std::string tune_key(const dedisp_plan_s *p, int64_t nsamp, const WidthList &wl) {
  uint64_t h = 1469598103934665603ull;   // FNV-1a over the tables and widths
  auto mix = [&](const void *data, size_t n) {
    const unsigned char *c = (const unsigned char *)data;
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  };
  mix(p->start.data(), p->start.size() * sizeof(int32_t));
  mix(p->ntap.data(), p->ntap.size() * sizeof(int32_t));
  mix(wl.w, sizeof(int32_t) * wl.n);
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  for (char &ch : arch)
    if (ch == ' ') ch = '_';
  char buf[256];
  snprintf(buf, sizeof(buf), "%s:%d:%d:%d:%lld:%016llx", arch.c_str(), p->nchan, p->ndm,
           p->max_span, (long long)nsamp, (unsigned long long)h);
  return buf;
}

static int tune_cache_lookup(const std::string &key) {
  const char *path = getenv("DEDISP_TUNE_CACHE");
  if (!path) return -1;
  FILE *f = fopen(path, "r");
  if (!f) return -1;
  char k[256];
  int ci = -1, found = -1;
  double ms;
  while (fscanf(f, "%255s %d %lf", k, &ci, &ms) == 3)
    if (key == k && ci >= 0 && ci < num_candidates()) found = ci;
  fclose(f);
  return found;
}

static void tune_cache_store(const std::string &key, int ci, double ms) {
  const char *path = getenv("DEDISP_TUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %.6f\n", key.c_str(), ci, ms);
  fclose(f);
}

}  // namespace dd

extern "C" dedisp_status dedisp_autotune(dedisp_plan p, const void *d_in, int64_t nsamp,
                                         int64_t in_stride, const int32_t *widths, int32_t nw,
                                         const double *d_chan_mean, const double *d_chan_sigma,
                                         void *d_work, size_t work_bytes, void *stream,
                                         int32_t *chosen) {
  using namespace dd;
  if (!p || !d_in || !widths || !d_chan_mean || !d_chan_sigma || !d_work || !chosen)
    return fail(DEDISP_ERR_INVALID_ARG, "null argument");
  if (p->wmode != DEDISP_W_UNIT) return fail(DEDISP_ERR_UNSUPPORTED, "the tuned kernel takes unit weights");
  if (nsamp < p->max_span || in_stride < nsamp) return fail(DEDISP_ERR_SHAPE, "bad block length");
  const int64_t nout = nsamp - p->max_span + 1;
  if (nw < 1 || nw > kMaxWidths) return fail(DEDISP_ERR_INVALID_ARG, "need 1..64 widths");
  std::vector<int32_t> wv(widths, widths + nw);
  std::sort(wv.begin(), wv.end());
  wv.erase(std::unique(wv.begin(), wv.end()), wv.end());
  WidthList wl;
  wl.n = (int32_t)wv.size();
  for (int i = 0; i < wl.n; ++i) wl.w[i] = wv[i];
  if (wv.front() < 1 || wv.back() > nout) return fail(DEDISP_ERR_INVALID_ARG, "bad widths");
  if (!search_supported(p, wl)) return fail(DEDISP_ERR_UNSUPPORTED, "plan cannot use the tiled search");
  if (work_bytes < search_work_bytes(p, wl.n, nout)) return fail(DEDISP_ERR_INVALID_ARG, "workspace too small");
  dedisp_status st = ensure_device(p);
  if (st != DEDISP_OK) return st;
  const std::string key = tune_key(p, nsamp, wl);
  const int cached = tune_cache_lookup(key);
  if (cached >= 0) {
    p->tile_choice = cached;
    *chosen = cached;
    return DEDISP_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  // scratch outputs and timing events, released on every return path
  struct Scratch {
    double *snr = nullptr;
    int32_t *tt = nullptr, *ww = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Scratch() {
      (void)hipFree(snr);
      (void)hipFree(tt);
      (void)hipFree(ww);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } sc;
  DD_HIP(dev_malloc((void **)&sc.snr, sizeof(double) * p->ndm));
  DD_HIP(dev_malloc((void **)&sc.tt, sizeof(int32_t) * p->ndm));
  DD_HIP(dev_malloc((void **)&sc.ww, sizeof(int32_t) * p->ndm));
  DD_HIP(hipEventCreate(&sc.e0));
  DD_HIP(hipEventCreate(&sc.e1));
  double *snr = sc.snr;
  int32_t *tt = sc.tt, *ww = sc.ww;
  hipEvent_t e0 = sc.e0, e1 = sc.e1;
  int best = -1;
  double best_ms = 1e30;
  // the timed calls must not advance the instrumentation slots
  std::vector<hipEvent_t> es, et;
  es.swap(p->ev_start);
  et.swap(p->ev_stop);
  // milliseconds of 3 searches in shape ci (after one untimed call when warm is set)
  auto time3 = [&](int ci, bool warm, float *ms) -> dedisp_status {
    dedisp_status r = DEDISP_OK;
    if (warm) {
      r = search_ci(p, ci, (const uint8_t *)d_in, nsamp, in_stride, nout, wl, d_chan_mean,
                    d_chan_sigma, snr, tt, ww, d_work, s);
      if (r != DEDISP_OK) return r;
    }
    hipError_t e = hipEventRecord(e0, s);
    for (int k = 0; k < 3 && e == hipSuccess && r == DEDISP_OK; ++k)
      r = search_ci(p, ci, (const uint8_t *)d_in, nsamp, in_stride, nout, wl, d_chan_mean,
                    d_chan_sigma, snr, tt, ww, d_work, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e != hipSuccess && r == DEDISP_OK) r = hip_fail(e, "autotune timing");
    return r;
  };
  std::vector<double> first(num_candidates(), -1.0);
  for (int ci = 0; ci < num_candidates() && st == DEDISP_OK; ++ci) {
    float ms = 0;
    st = time3(ci, true, &ms);
    if (st == DEDISP_ERR_UNSUPPORTED) {
      st = DEDISP_OK;
      continue;
    }
    if (st != DEDISP_OK) break;
    first[ci] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = ci;
    }
  }
  // the shapes within 3 % of the fastest are timed again, interleaved, twice more (so
  // that a drift of the clocks during the first pass does not decide between them)
  std::vector<int> close;
  for (int ci = 0; ci < num_candidates() && st == DEDISP_OK; ++ci)
    if (first[ci] >= 0 && first[ci] <= 1.03 * best_ms) close.push_back(ci);
  if (st == DEDISP_OK && close.size() > 1) {
    std::vector<double> tot(close.size(), 0.0);
    for (int round = 0; round < 2 && st == DEDISP_OK; ++round)
      for (size_t i = 0; i < close.size() && st == DEDISP_OK; ++i) {
        float ms = 0;
        st = time3(close[i], false, &ms);
        tot[i] += ms;
      }
    if (st == DEDISP_OK) {
      size_t bi = 0;
      for (size_t i = 1; i < close.size(); ++i)
        if (tot[i] < tot[bi]) bi = i;
      best = close[bi];
      best_ms = tot[bi] / 2.0;
    }
  }
  es.swap(p->ev_start);
  et.swap(p->ev_stop);
  // the scratch outputs are freed on return; the timed searches must have finished
  if (st == DEDISP_OK) DD_HIP(hipStreamSynchronize(s));
  if (st != DEDISP_OK) return st;
  if (best < 0) return fail(DEDISP_ERR_UNSUPPORTED, "no tile shape fits this plan");
  p->tile_choice = best;
  tune_cache_store(key, best, best_ms / 3.0);
  *chosen = best;
  return DEDISP_OK;
}
