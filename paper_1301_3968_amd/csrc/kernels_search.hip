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

#include "internal.h"

namespace dd {

// ------------------------------------------------------------------------------
// Tile configurations (candidates for the autotuner)
// ------------------------------------------------------------------------------
struct TileCfg {
  int dpw;   // trials per wave (4 waves per workgroup)
  int r2;    // packed output pairs per lane per row: outputs per tile row = 128 * r2
};
static const TileCfg kCfgs[] = {{4, 8}, {8, 4}, {2, 8}, {4, 4}};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);
constexpr int kDefaultCfg = 0;
constexpr int kHalo = 32;                 // boxcar widths up to 32
constexpr int kStageBudget = 48 * 1024;   // LDS bytes for one channel group's windows

struct GroupInfo {
  int32_t job_begin, njobs, lw, c_begin;   // lw: window length in samples (multiple of 8)
  int32_t c_count, flush, pad0, pad1;
};

struct TiledCfgTables {
  bool ok = false;
  int dt = 0, ty = 0, tt = 0, ntd = 0, ngroups = 0, lds_bytes = 0;
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

// U_{c,n}[tau] for tau in [0, tpad), n in [nmin_c, nmax_c]; each thread makes 8
// consecutive tau of every row of its channel from bytes staged in LDS.
constexpr int kRowThreads = 256;
constexpr int kRowSpan = kRowThreads * 8;   // tau per block
__global__ void __launch_bounds__(kRowThreads)
k_window_rows(const uint8_t *__restrict__ x, int64_t in_stride, int64_t nsamp, int64_t tpad,
              const int32_t *__restrict__ nmin, const int32_t *__restrict__ nmaxv,
              const int64_t *__restrict__ rowidx, uint16_t *__restrict__ U) {
  extern __shared__ unsigned char sx[];
  const int c = blockIdx.y, tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blockIdx.x * kRowSpan;
  const int n0 = nmin[c], n1 = nmaxv[c];
  const uint8_t *row = x + (int64_t)c * in_stride;
  const int nbytes = kRowSpan + n1;
  for (int i = tid; i < nbytes; i += kRowThreads) {
    const int64_t g = blk0 + i;
    sx[i] = g < nsamp ? row[g] : 0;
  }
  __syncthreads();
  const int64_t tau0 = blk0 + tid * 8;
  if (tau0 >= tpad) return;
  uint32_t s[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) s[i] = 0;
  const unsigned char *b = sx + tid * 8;
  for (int n = 1; n <= n1; ++n) {
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] += b[i + n - 1];
    if (n >= n0) {
      uint16_t *dst = U + (rowidx[c] + (n - n0)) * tpad + tau0;
      uint32_t w[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // windows running past the end of the block are zero
        const uint32_t lo = (tau0 + 2 * i + n <= nsamp) ? s[2 * i] : 0u;
        const uint32_t hi = (tau0 + 2 * i + 1 + n <= nsamp) ? s[2 * i + 1] : 0u;
        w[i] = lo | (hi << 16);
      }
      *(uint4 *)dst = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
  if (n0 == 0) {
    uint16_t *dst = U + rowidx[c] * tpad + tau0;
    *(uint4 *)dst = make_uint4(0, 0, 0, 0);
  }
}

struct SearchArgs {
  const uint16_t *U;
  int64_t tpad;
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

struct CandRec {
  double snr;
  int32_t t;
  int32_t w;
};

__device__ __forceinline__ int bitrev5(int v) {
  return ((v & 1) << 4) | ((v & 2) << 2) | (v & 4) | ((v & 8) >> 2) | ((v & 16) >> 4);
}

template <int DPW, int R2>
__global__ void __launch_bounds__(256)
k_search(SearchArgs a) {
  constexpr int TY = 128 * R2, TT = TY - kHalo, DT = 4 * DPW, SP = TY / 64;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

  // XCD-aware tile order: blocks b = x (mod 8) all run on XCD x; give XCD x a
  // contiguous run of tiles in time-major order.
  const int nb = a.ntd * a.ntt;
  const int b = blockIdx.x;
  const int xcd = b & 7, k = b >> 3, q = nb >> 3, rem = nb & 7;
  const int L = xcd * q + min(xcd, rem) + k;
  const int tt = L / a.ntd, td = L - tt * a.ntd;
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

  const int gb = a.group_begin[td], ge = a.group_begin[td + 1];
  const int trial0 = td * DT + wave * DPW;
  for (int g = gb; g < ge; ++g) {
    const GroupInfo gi = a.groups[g];
    // LDS read offsets of this wave's (trial, channel) pairs, one per lane;
    // broadcast later with v_readlane (no memory latency in the inner loop).
    const int cc = gi.c_count;
    int myoff = 0;
    if (lane < DPW * cc) {
      const int jj = lane / cc, c = lane - jj * cc;
      myoff = a.offs[(int64_t)(trial0 + jj) * a.nchan + gi.c_begin + c];
    }
    __syncthreads();
    // ---- stage the group's U windows: copy A (aligned) and copy B (shifted by one)
    {
      const int nchunk = gi.lw >> 3;
      for (int j = 0; j < gi.njobs; ++j) {
        const int2 jb = a.jobs[gi.job_begin + j];
        const int64_t e0 = (int64_t)jb.x * a.tpad + jb.y + t0;
        const uint32_t *src = (const uint32_t *)(a.U + (e0 & ~(int64_t)1));
        unsigned char *rowA = lds + j * 4 * gi.lw;
        unsigned char *rowB = rowA + 2 * gi.lw;
        if (e0 & 1) {
          for (int ch = tid; ch < nchunk; ch += 256) {
            const uint32_t *q = src + 4 * ch;
            const uint32_t w0 = q[0], w1 = q[1], w2 = q[2], w3 = q[3], w4 = q[4];
            *(uint4 *)(rowA + ch * 16) = make_uint4(__builtin_amdgcn_alignbyte(w1, w0, 2),
                                                    __builtin_amdgcn_alignbyte(w2, w1, 2),
                                                    __builtin_amdgcn_alignbyte(w3, w2, 2),
                                                    __builtin_amdgcn_alignbyte(w4, w3, 2));
            *(uint4 *)(rowB + ch * 16) = make_uint4(w1, w2, w3, w4);
          }
        } else {
          for (int ch = tid; ch < nchunk; ch += 256) {
            const uint32_t *q = src + 4 * ch;
            const uint32_t w0 = q[0], w1 = q[1], w2 = q[2], w3 = q[3], w4 = q[4];
            *(uint4 *)(rowA + ch * 16) = make_uint4(w0, w1, w2, w3);
            *(uint4 *)(rowB + ch * 16) = make_uint4(__builtin_amdgcn_alignbyte(w1, w0, 2),
                                                    __builtin_amdgcn_alignbyte(w2, w1, 2),
                                                    __builtin_amdgcn_alignbyte(w3, w2, 2),
                                                    __builtin_amdgcn_alignbyte(w4, w3, 2));
          }
        }
      }
    }
    __syncthreads();
    // ---- accumulate: per trial, per channel, R2 aligned dword reads
    const unsigned char *lbase = lds + lane * 4;
#pragma unroll
    for (int j = 0; j < DPW; ++j) {
      int c = 0;
      for (; c + 4 <= cc; c += 4) {
        int o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) o[u] = __builtin_amdgcn_readlane(myoff, j * cc + c + u);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const unsigned char *pp = lbase + o[u];
#pragma unroll
          for (int r = 0; r < R2; ++r) a16[j][r] = pk_add_u16(a16[j][r], *(const uint32_t *)(pp + 256 * r));
        }
      }
      for (; c < cc; ++c) {
        const unsigned char *pp = lbase + __builtin_amdgcn_readlane(myoff, j * cc + c);
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
  }

  // ---- boxcar search, one trial of each wave at a time
  __syncthreads();
  int *Yw = (int *)lds + wave * (TY + kHalo + 4);
  CandRec *part = (CandRec *)a.part;
#pragma unroll
  for (int j = 0; j < DPW; ++j) {
    const int dg = a.perm[td * DT + wave * DPW + j];
#pragma unroll
    for (int r = 0; r < R2; ++r)
      *(int2 *)(Yw + 2 * lane + 128 * r) = make_int2(acc[j][2 * r], acc[j][2 * r + 1]);
    if (lane < kHalo) Yw[TY + lane] = 0;
    __syncthreads();
    // register prefix over this lane's starts and their windows
    int qv[SP + kHalo + 1];
    qv[0] = 0;
#pragma unroll
    for (int i = 0; i < SP + kHalo; ++i) qv[i + 1] = qv[i] + Yw[lane * SP + i];
    const int64_t ts = t0 + lane * SP;          // first start of this lane
    const bool owned = lane * SP < TT;
    const bool full = owned && (ts + SP - 1 + kHalo <= a.nout);
    int mx[32];
#pragma unroll
    for (int w = 0; w < 32; ++w) mx[w] = INT_MIN;
    if (full) {
#pragma unroll
      for (int w = 1; w <= 32; ++w) {
        if ((a.wmask >> (w - 1)) & 1u) {
          int m = INT_MIN;
#pragma unroll
          for (int i = 0; i < SP; ++i) m = max(m, qv[i + w] - qv[i]);
          mx[w - 1] = m;
        }
      }
    } else if (owned) {
#pragma unroll
      for (int w = 1; w <= 32; ++w) {
        if ((a.wmask >> (w - 1)) & 1u) {
          int m = INT_MIN;
#pragma unroll
          for (int i = 0; i < SP; ++i)
            if (ts + i + w <= a.nout) m = max(m, qv[i + w] - qv[i]);
          mx[w - 1] = m;
        }
      }
    }
    // transpose-reduce: lane l ends with the max over all lanes for W = bitrev5(l&31)+1
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      const int half = 16 >> s;
      const bool hi = (lane >> s) & 1;
#pragma unroll
      for (int i = 0; i < half; ++i) {
        const int send = hi ? mx[i] : mx[i + half];
        const int keep = hi ? mx[i + half] : mx[i];
        const int got = __shfl_xor(send, 1 << s, 64);
        mx[i] = max(keep, got);
      }
    }
    int bmax = max(mx[0], __shfl_xor(mx[0], 32, 64));
    const int wl = bitrev5(lane & 31) + 1;
    const int ji = a.widx[wl];
    double snr = -INFINITY;
    if (ji >= 0 && bmax != INT_MIN && dg >= 0)
      snr = ((double)bmax - a.M[(int64_t)dg * a.nw + ji]) / a.S[(int64_t)dg * a.nw + ji];
    // wave argmax over (snr desc, W asc)
    int bw = wl, bb = bmax;
#pragma unroll
    for (int s = 1; s < 32; s <<= 1) {
      const double os = __shfl_xor(snr, s, 64);
      const int ow = __shfl_xor(bw, s, 64), ob = __shfl_xor(bb, s, 64);
      if (os > snr || (os == snr && ow < bw)) {
        snr = os;
        bw = ow;
        bb = ob;
      }
    }
    snr = __shfl(snr, 0, 64);
    bw = __shfl(bw, 0, 64);
    bb = __shfl(bb, 0, 64);
    // earliest start of the winning width in this tile
    int first = -1;
    if (owned && snr != -INFINITY) {
#pragma unroll
      for (int w = 1; w <= 32; ++w) {
        if (w == bw) {
#pragma unroll
          for (int i = SP - 1; i >= 0; --i)
            if (ts + i + w <= a.nout && qv[i + w] - qv[i] == bb) first = i;
        }
      }
    }
    const unsigned long long hit = __ballot(first >= 0);
    int tbest = -1;
    if (hit != 0ull) {
      const int fl = __builtin_ctzll(hit);
      const int fi = __shfl(first, fl, 64);
      tbest = (int)(t0 + fl * SP + fi);
    }
    if (dg >= 0 && lane == 0) {
      CandRec rec;
      rec.snr = (hit != 0ull) ? snr : -INFINITY;
      rec.t = (hit != 0ull) ? tbest : -1;
      rec.w = (hit != 0ull) ? bw : 0;
      part[(int64_t)dg * a.ntt + tt] = rec;
    }
    __syncthreads();
  }
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
static bool build_cfg(const dedisp_plan_s *p, const TiledTables &T, int ci, TiledCfgTables &out) {
  const TileCfg cf = kCfgs[ci];
  const int C = p->nchan, D = p->ndm;
  const int DT = 4 * cf.dpw, TY = 128 * cf.r2;
  out = TiledCfgTables();
  out.dt = DT;
  out.ty = TY;
  out.tt = TY - kHalo;
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
        if (ccount == 0 && (bytes > kStageBudget || over)) return false;
        if (bytes > kStageBudget || over || ccount >= 64 / cf.dpw) break;
        span = nspan;
        nrows_g += (int)ns.size();
        for (int j = 0; j < DT; ++j) run[j] += 255LL * p->ntap[(size_t)tr[j] * C + c];
        ++ccount;
        ++c;
      }
      const int lw = ((TY + span + 2) + 7) & ~7;
      gi.lw = lw;
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
  out.lds_bytes = std::max(lds_max, 4 * (TY + kHalo + 4) * 4);
  out.ok = true;
  return true;
}

template <typename T>
static hipError_t upload(T **dst, const std::vector<T> &v) {
  hipError_t e = hipMalloc((void **)dst, std::max<size_t>(1, v.size()) * sizeof(T));
  if (e != hipSuccess) return e;
  if (v.empty()) return hipSuccess;
  return hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

static int cfg_index(const dedisp_plan_s *p) {
  return (p->tile_choice >= 0 && p->tile_choice < kNumCfgs) ? p->tile_choice : kDefaultCfg;
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
  const int TY = 128 * cf.r2, TT = TY - kHalo;
  Layout L;
  L.ntt = (nout + TT - 1) / TT;
  L.tpad = (((L.ntt - 1) * TT + TY + 2 * (int64_t)p->max_span + 32) + 7) & ~(int64_t)7;
  L.nrows = nrows;
  const size_t tables = align256(2 * sizeof(double) * (size_t)p->ndm * nw);
  L.off_part = tables;
  L.off_u = L.off_part + align256(sizeof(CandRec) * (size_t)p->ndm * L.ntt);
  L.total = L.off_u + align256(sizeof(uint16_t) * (size_t)nrows * L.tpad);
  return L;
}

static int64_t count_rows(const dedisp_plan_s *p) {
  const int C = p->nchan, D = p->ndm;
  int64_t r = 0;
  for (int c = 0; c < C; ++c) {
    int lo = INT32_MAX, hi = 0;
    for (int d = 0; d < D; ++d) {
      lo = std::min(lo, p->ntap[(size_t)d * C + c]);
      hi = std::max(hi, p->ntap[(size_t)d * C + c]);
    }
    r += hi - lo + 1;
  }
  return r;
}

size_t search_work_bytes(const dedisp_plan_s *p, int32_t nw, int64_t nout) {
  if (p->wmode != DEDISP_W_UNIT) return 0;
  const int64_t nrows = count_rows(p);
  size_t best = 0;
  for (int ci = 0; ci < kNumCfgs; ++ci) best = std::max(best, layout(p, ci, nw, nout, nrows).total);
  return best;
}

bool search_supported(const dedisp_plan_s *p, const WidthList &wl) {
  if (p->wmode != DEDISP_W_UNIT) return false;
  if (wl.w[wl.n - 1] > 32) return false;
  if (p->max_ntap > 257) return false;
  // the register prefix of the boxcar stage sums up to SP + 32 int32 outputs
  const double ymax = 255.0 * (double)p->sum_max_ntap;
  if (ymax * (16 + 32 + 1) >= 2147483647.0) return false;
  return true;
}

template <int DPW, int R2>
static hipError_t launch_cfg(const SearchArgs &a, int nblocks, int lds, hipStream_t s) {
  hipLaunchKernelGGL((k_search<DPW, R2>), dim3(nblocks), dim3(256), lds, s, a);
  return hipGetLastError();
}

static hipError_t launch_search_kernel(int ci, const SearchArgs &a, int nblocks, int lds,
                                       hipStream_t s) {
  switch (ci) {
    case 0: return launch_cfg<4, 8>(a, nblocks, lds, s);
    case 1: return launch_cfg<8, 4>(a, nblocks, lds, s);
    case 2: return launch_cfg<2, 8>(a, nblocks, lds, s);
    default: return launch_cfg<4, 4>(a, nblocks, lds, s);
  }
}

dedisp_status run_search_tiled(dedisp_plan p, const uint8_t *x, int64_t nsamp, int64_t in_stride,
                               int64_t nout, const WidthList &wl, const double *mu,
                               const double *sigma, double *snr, int32_t *t, int32_t *w,
                               void *work, hipStream_t s) {
  const int ci = cfg_index(p);
  TiledCfgTables *cfg = nullptr;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    dedisp_status st = ensure_cfg(p, ci, &cfg);
    if (st != DEDISP_OK) return st;
  }
  if (!cfg) return DEDISP_ERR_UNSUPPORTED;   // caller falls back to the general path
  const TiledTables &T = *p->tiled;
  const Layout L = layout(p, ci, wl.n, nout, T.nrows);
  if (L.ntt * (int64_t)cfg->ntd > INT32_MAX / 2) return DEDISP_ERR_UNSUPPORTED;
  double *M = (double *)work;
  double *S = M + (size_t)p->ndm * wl.n;
  void *part = (char *)work + L.off_part;
  uint16_t *U = (uint16_t *)((char *)work + L.off_u);
  DD_HIP(launch_norm(p, wl, mu, sigma, M, S, s));
  {
    const dim3 g((unsigned)((L.tpad + kRowSpan - 1) / kRowSpan), (unsigned)p->nchan);
    const int shm = kRowSpan + T.nmax_all + 16;
    hipLaunchKernelGGL(k_window_rows, g, dim3(kRowThreads), shm, s, x, in_stride, nsamp, L.tpad,
                       T.d_nmin, T.d_nmax, T.d_rowidx, U);
    DD_HIP(hipGetLastError());
  }
  SearchArgs a{};
  a.U = U;
  a.tpad = L.tpad;
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
  a.S = S;
  a.nw = wl.n;
  a.wmask = 0;
  for (int i = 0; i <= 32; ++i) a.widx[i] = -1;
  for (int i = 0; i < wl.n; ++i) {
    a.wmask |= 1u << (wl.w[i] - 1);
    a.widx[wl.w[i]] = (int8_t)i;
  }
  a.part = part;
  KernelTimer kt(p, s);
  DD_HIP(kt.begin());
  DD_HIP(launch_search_kernel(ci, a, cfg->ntd * (int)L.ntt, cfg->lds_bytes, s));
  DD_HIP(kt.end());
  DD_HIP(launch_reduce(p->ndm, (int32_t)L.ntt, part, snr, t, w, s));
  p->last_search_tile = ci;
  return DEDISP_OK;
}

int search_config_count() { return kNumCfgs; }

}  // namespace dd

extern "C" {

dedisp_status dedisp_set_tile(dedisp_plan p, int32_t tile) {
  if (!p) return dd::fail(DEDISP_ERR_INVALID_ARG, "null plan");
  if (tile < -2 || tile >= dd::kNumCfgs) return dd::fail(DEDISP_ERR_INVALID_ARG, "tile index out of range");
  p->tile_choice = tile;
  return DEDISP_OK;
}

}  // extern "C"
