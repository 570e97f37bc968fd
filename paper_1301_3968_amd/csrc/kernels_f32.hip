// Tiled fp32 dedispersion (eq. p_dedisp) for weighted profiles: per-channel weights
// w_c, per-tap weights w_{c,k}, or unit weights with fp32 output; uint8 or fp32
// input.
//
//   1. k_rows_f32: for every channel c and every tap count n the plan uses there,
//      the weighted window row R_{c,n}[tau] = sum_{k<n} omega_{c,k} x[c][tau + k]
//      (omega = 1, w_c or w_{c,k}), fp32, zero past the block end.  A trial's sum
//      over channel c is then one sample of one row: y[d,t] = sum_c R_{c,n[d,c]}[t +
//      start[d,c]].
//   2. k_dedisp_f32<R, DPW, NW>: one workgroup per (DM tile, time tile, batch
//      element).  Trials are sorted by DM and taken NW * DPW at a time, so their
//      delays in a channel span few samples; for a group of channels the rows they
//      need are copied into LDS (direct buffer-to-LDS loads, double-buffered so the
//      next group streams in while the current one is summed).  Lane l adds, per
//      (trial, channel), the R samples l, l + 64, .. of the trial's window (fp32
//      rows need no second copy: any sample offset is dword-aligned).  Sums over a
//      group (at most 32 channels) run in fp32; group sums are added in fp64, so the
//      result is within a few fp32 roundings of the exact sum.  The transposed use
//      below instead adds every term in fp64 and writes fp64 (A64).
// Long blocks are processed in time segments so that the rows stay within 4 GiB.
//
// The same two kernels compute the transpose of the one-sample-per-channel sum (the
// adjoint needed for per-tap weights): with trials as row channels, channels as
// outputs and the trial gradients as rows, it is again a sum of shifted rows.  Its
// terms have mixed signs and the weight gradient formed from it cancels heavily, so
// there each term is added in fp64 (exact conversion of the fp32 row sample) and the
// fp64 sum is written out: the transposed sum is then exact to fp64 rounding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <numeric>
#include <type_traits>
#include <vector>

#include "internal.h"

namespace dd {

// Tile shapes: R outputs per lane (TY = 64 R outputs per tile), DPW trials per
// wave, NW waves per workgroup.
#define DD_F32_CONFIGS(X) \
  X(0, 8, 2, 16)          \
  X(1, 8, 2, 8)
struct F32Cfg {
  int r, dpw, nw;
};
#define DD_F32_ENTRY(i, r, d, w) {r, d, w},
static const F32Cfg kF32Cfgs[] = {DD_F32_CONFIGS(DD_F32_ENTRY)};
#undef DD_F32_ENTRY
constexpr int kNumF32Cfgs = sizeof(kF32Cfgs) / sizeof(kF32Cfgs[0]);
constexpr int kF32MaxLds = 160 * 1024;
constexpr size_t kF32RowBytesMax = (size_t)4 << 30;   // rows per time segment
constexpr int kF32MaxTaps = 4096;                     // longest window row built

struct F32Group {
  int32_t job_begin, njobs, lw, c_begin;   // lw: window length in samples (multiple of 4)
  int32_t c_count, pad0, pad1, pad2;
};

struct F32CfgTables {
  bool ok = false;
  int dt = 0, ty = 0, ntd = 0, bufbytes = 0, lds_bytes = 0;
  std::vector<int32_t> offs, group_begin, perm;
  std::vector<F32Group> groups;
  std::vector<int32_t> jobs;   // pairs {row, base start}
  int32_t *d_offs = nullptr, *d_group_begin = nullptr, *d_perm = nullptr, *d_jobs = nullptr;
  F32Group *d_groups = nullptr;
};

struct F32Tables {
  std::vector<int32_t> nmin, nmax;
  std::vector<int64_t> rowidx;
  int64_t nrows = 0;
  int32_t nmax_all = 0;
  int32_t *d_nmin = nullptr, *d_nmax = nullptr;
  int64_t *d_rowidx = nullptr;
  int32_t lead = 0;            // zeros in front of each row (transposed gathers)
  F32CfgTables cfg[kNumF32Cfgs];
  bool tried[kNumF32Cfgs] = {};
};

void free_f32(F32Tables *t) {
  if (!t) return;
  (void)hipFree(t->d_nmin);
  (void)hipFree(t->d_nmax);
  (void)hipFree(t->d_rowidx);
  for (auto &c : t->cfg) {
    (void)hipFree(c.d_offs);
    (void)hipFree(c.d_group_begin);
    (void)hipFree(c.d_perm);
    (void)hipFree(c.d_jobs);
    (void)hipFree(c.d_groups);
  }
  delete t;
}

namespace {

typedef __attribute__((address_space(3))) void lds_void;
constexpr unsigned kWaitVm0 = 0x0f70;      // s_waitcnt vmcnt(0) (gfx9 encoding)
constexpr int kBufWord3 = 0x00020000;      // raw 32-bit buffer descriptor word 3

__device__ __forceinline__ int32_t ldc(const int32_t *p, int64_t i) {
  return ((const __attribute__((address_space(4))) int32_t *)p)[i];
}

// ---- rows ----------------------------------------------------------------------
// Each thread builds 4 consecutive tau in each of kRowHalves runs of 4 * kRowThreads.
constexpr int kRowThreads = 256, kRowHalves = 2, kRowTau = 4 * kRowThreads * kRowHalves;
constexpr int kRowLoads = kRowTau / kRowThreads;   // block samples loaded per thread

template <typename XT>
__global__ void __launch_bounds__(kRowThreads)
k_rows_f32(const XT *__restrict__ x, int64_t in_stride, int64_t in_bstride, int64_t nsamp,
           int64_t lead, int64_t seg0, int64_t tpad, const int32_t *__restrict__ nmin,
           const int32_t *__restrict__ nmaxv, const int64_t *__restrict__ rowidx, int64_t nrows,
           int32_t wmode, int32_t K, const float *__restrict__ w, float *__restrict__ R) {
  extern __shared__ float sxf[];
  const int c = blockIdx.y, b = blockIdx.z, tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blockIdx.x * kRowTau;
  const int n0 = nmin[c], n1 = nmaxv[c];
  const XT *row = x + (int64_t)b * in_bstride + (int64_t)c * in_stride;
  // input samples blk0 .. blk0 + kRowTau + n1 of the row (rows start `lead` zeros
  // before the input); the fixed part is loaded with every load in flight at once
  const int64_t g0 = seg0 + blk0 - lead;
  float v0[kRowLoads];
#pragma unroll
  for (int j = 0; j < kRowLoads; ++j) {
    const int64_t g = g0 + tid + kRowThreads * j;
    v0[j] = (g >= 0 && g < nsamp) ? (float)row[g] : 0.0f;
  }
#pragma unroll
  for (int j = 0; j < kRowLoads; ++j) sxf[tid + kRowThreads * j] = v0[j];
  for (int i = kRowTau + tid; i < kRowTau + n1; i += kRowThreads) {
    const int64_t g = g0 + i;
    sxf[i] = (g >= 0 && g < nsamp) ? (float)row[g] : 0.0f;
  }
  __syncthreads();
  const float wc = wmode == DEDISP_W_CHANNEL ? w[c] : 1.0f;
  float *rbase = R + ((int64_t)b * nrows + rowidx[c]) * tpad;
  float s[kRowHalves][4] = {};
  bool live[kRowHalves];
  int64_t tau0[kRowHalves];
#pragma unroll
  for (int h = 0; h < kRowHalves; ++h) {
    tau0[h] = blk0 + 4 * tid + 4 * kRowThreads * h;
    live[h] = tau0[h] < tpad;   // tpad is a multiple of 4
    if (live[h] && n0 == 0) *(float4 *)(rbase + tau0[h]) = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  for (int n = 1; n <= n1; ++n) {
    const float wk = wmode == DEDISP_W_TAP ? w[(int64_t)c * K + (n - 1)] : 1.0f;
#pragma unroll
    for (int h = 0; h < kRowHalves; ++h) {
      const float *xl = sxf + 4 * tid + 4 * kRowThreads * h + (n - 1);
#pragma unroll
      for (int i = 0; i < 4; ++i) s[h][i] += wk * xl[i];
    }
    if (n >= n0) {
#pragma unroll
      for (int h = 0; h < kRowHalves; ++h) {
        if (!live[h]) continue;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)   // windows running past the end of the block are zero
          v[i] = (seg0 + tau0[h] + i + n <= nsamp + lead) ? s[h][i] * wc : 0.0f;
        *(float4 *)(rbase + (int64_t)(n - n0) * tpad + tau0[h]) = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  }
}

// ---- tile kernel ---------------------------------------------------------------
struct F32Args {
  const float *R;          // rows of batch element 0; element b at + b * rbstride
  int64_t rbstride, tpad;
  int32_t bufbytes, ntd, ntt, nchan;
  const int32_t *offs;
  const F32Group *groups;
  const int32_t *group_begin, *jobs, *perm;
  int64_t nout;            // outputs of this segment
  void *out;               // y of batch element 0 at this segment's first output
  int64_t out_stride, out_bstride;
};

__device__ __forceinline__ F32Group load_group(const F32Group *groups, int g) {
  typedef int32_t i32x8 __attribute__((ext_vector_type(8)));
  const i32x8 v = *(const __attribute__((address_space(4))) i32x8 *)(groups + g);
  F32Group gi;
  gi.job_begin = v[0];
  gi.njobs = v[1];
  gi.lw = v[2];
  gi.c_begin = v[3];
  gi.c_count = v[4];
  gi.pad0 = gi.pad1 = gi.pad2 = 0;
  return gi;
}

// Starts the copy of group gi's rows (one window of lw samples per job) into an
// LDS buffer; each copy has its own buffer descriptor covering exactly that window.
template <int NW>
__device__ __forceinline__ void stage_group(const F32Args &a, const F32Group &gi, const float *R,
                                            int64_t t0, int wave, int lane, unsigned char *buf) {
  const int nchunk = gi.lw >> 2;   // 16-byte chunks
  for (int j = wave; j < gi.njobs; j += NW) {
    const int32_t *jp = a.jobs + 2 * (gi.job_begin + j);
    const int jrow = ldc(jp, 0), jstart = ldc(jp, 1);
    const float *src = R + (int64_t)jrow * a.tpad + jstart + t0;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)src, (short)0, 4 * gi.lw, kBufWord3);
    unsigned char *dst = buf + j * 4 * gi.lw;
    for (int k = 0; 64 * k < nchunk; ++k) {
      const int ch = lane + 64 * k;
      if (ch < nchunk)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void *)(dst + 1024 * k), 16, 16 * ch, 0, 0, 0);
    }
  }
}

template <int DPW>
__device__ __forceinline__ int group_offsets(const F32Args &a, const F32Group &gi, int trial0,
                                             int lane) {
  const int cc = gi.c_count;
  int o = 0;
  if (lane < DPW * cc) {
    const int jj = lane / cc, c = lane - jj * cc;
    o = a.offs[(int64_t)(trial0 + jj) * a.nchan + gi.c_begin + c];
  }
  return o;
}

// A64 false: fp32 group sums added into fp64, fp32 output.  A64 true: every term
// added in fp64, fp64 output.
template <int R, int DPW, int NW, bool A64>
__global__ void __launch_bounds__(64 * NW)
k_dedisp_f32(F32Args a) {
  typedef typename std::conditional<A64, double, float>::type PT;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  constexpr int TY = 64 * R, DT = NW * DPW;
  constexpr int CH = 24 / R;   // channels per chunk: 12 two-address reads in flight
  static_assert(CH * R == 24, "chunk of 12 two-address reads");
  // XCD-aware tile order (blocks b = x mod 8 run on XCD x): contiguous runs of tiles
  const int nb = a.ntd * a.ntt;
  const int bi = blockIdx.x;
  const int xcd = bi & 7, kk = bi >> 3, q = nb >> 3, rem = nb & 7;
  const int L = xcd * q + min(xcd, rem) + kk;
  const int tt = L / a.ntd, td = L - tt * a.ntd;
  const int bb = blockIdx.y;
  const float *Rb = a.R + (int64_t)bb * a.rbstride;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t t0 = (int64_t)tt * TY;
  const int trial0 = td * DT + wave * DPW;

  double acc[DPW][R];
#pragma unroll
  for (int j = 0; j < DPW; ++j)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[j][r] = 0.0;

  const int gb = ldc(a.group_begin, td), ge = ldc(a.group_begin, td + 1);
  int myoff;
  {
    const F32Group g0 = load_group(a.groups, gb);
    myoff = group_offsets<DPW>(a, g0, trial0, lane);
    stage_group<NW>(a, g0, Rb, t0, wave, lane, lds);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
  }
  for (int g = gb; g < ge; ++g) {
    const F32Group gi = load_group(a.groups, g);
    const int cc = gi.c_count;
    const int par = (g - gb) & 1;
    int nextoff = 0;
    if (g + 1 < ge) {
      const F32Group gn = load_group(a.groups, g + 1);
      nextoff = group_offsets<DPW>(a, gn, trial0, lane);
      stage_group<NW>(a, gn, Rb, t0, wave, lane, lds + (par ^ 1) * a.bufbytes);
    }
    const unsigned char *lbase = lds + par * a.bufbytes + lane * 4;
#pragma unroll
    for (int j = 0; j < DPW; ++j) {
      PT part[R];
#pragma unroll
      for (int r = 0; r < R; ++r) part[r] = (PT)0;
      const int jb = j * cc;
      int c = 0;
      for (; c + CH <= cc; c += CH) {
        const unsigned char *pc[CH];
#pragma unroll
        for (int qq = 0; qq < CH; ++qq) pc[qq] = lbase + __builtin_amdgcn_readlane(myoff, jb + c + qq);
#pragma unroll
        for (int qq = 0; qq < CH; ++qq)
#pragma unroll
          for (int r = 0; r < R; ++r) part[r] += (PT)*(const float *)(pc[qq] + 256 * r);
      }
      for (; c < cc; ++c) {
        const unsigned char *pp = lbase + __builtin_amdgcn_readlane(myoff, jb + c);
#pragma unroll
        for (int r = 0; r < R; ++r) part[r] += (PT)*(const float *)(pp + 256 * r);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) acc[j][r] += (double)part[r];
    }
    // the next group's windows and offsets have landed; this group's reads are done
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
    myoff = nextoff;
  }
  typedef typename std::conditional<A64, double, float>::type OT;
  OT *ob = (OT *)a.out + (int64_t)bb * a.out_bstride;
#pragma unroll
  for (int j = 0; j < DPW; ++j) {
    const int d = a.perm[td * DT + wave * DPW + j];
    if (d < 0) continue;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t t = t0 + lane + 64 * r;
      if (t < a.nout) ob[(int64_t)d * a.out_stride + t] = (OT)acc[j][r];
    }
  }
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

// What the tiled kernel sums: out[o][t] = sum_r row_{r, ntap[o][r]}[t + start[o][r]]
// for `nout_rows` outputs o (the forward's trials) over `nrow_ch` row channels r (the
// forward's channels); outputs are tiled in the order of `key`.
struct GatherSpec {
  int32_t nout_rows = 0, nrow_ch = 0;
  const int32_t *start = nullptr, *ntap = nullptr;   // [nout_rows][nrow_ch], host
  const double *key = nullptr;                       // [nout_rows]
};

static void build_rows_f32(const GatherSpec &gs, F32Tables *T) {
  const int C = gs.nrow_ch, D = gs.nout_rows;
  T->nmin.assign(C, INT32_MAX);
  T->nmax.assign(C, 0);
  for (int d = 0; d < D; ++d)
    for (int c = 0; c < C; ++c) {
      const int n = gs.ntap[(size_t)d * C + c];
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

// Row-channel groups per output tile (LDS budget per buffer), window jobs and the
// per-(output, row channel) LDS byte offsets.  Returns false if one row channel alone
// does not fit.
static bool build_f32_cfg(const GatherSpec &gs, const F32Tables &T, int ci, int budget,
                          F32CfgTables &out) {
  const F32Cfg cf = kF32Cfgs[ci];
  const int C = gs.nrow_ch, D = gs.nout_rows;
  const int DT = cf.nw * cf.dpw, TY = 64 * cf.r;
  out = F32CfgTables();
  out.dt = DT;
  out.ty = TY;
  std::vector<int32_t> order(D);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return gs.key[a] < gs.key[b]; });
  const int ntd = (D + DT - 1) / DT;
  out.ntd = ntd;
  out.perm.assign((size_t)ntd * DT, -1);
  for (int i = 0; i < D; ++i) out.perm[i] = order[i];
  out.offs.assign((size_t)ntd * DT * C, 0);
  out.group_begin.assign(ntd + 1, 0);
  int lds_max = 0;
  std::vector<int> tr(DT);
  for (int td = 0; td < ntd; ++td) {
    out.group_begin[td] = (int)out.groups.size();
    for (int j = 0; j < DT; ++j) {
      const int d = out.perm[(size_t)td * DT + j];
      tr[j] = d >= 0 ? d : out.perm[(size_t)td * DT];
    }
    int c = 0;
    while (c < C) {
      F32Group gi{};
      gi.job_begin = (int)out.jobs.size() / 2;
      gi.c_begin = c;
      int span = 0, nrows_g = 0, ccount = 0;
      while (c < C) {
        int smin = INT32_MAX, smax = INT32_MIN;
        std::vector<int> ns;
        for (int j = 0; j < DT; ++j) {
          const int s = gs.start[(size_t)tr[j] * C + c], n = gs.ntap[(size_t)tr[j] * C + c];
          smin = std::min(smin, s);
          smax = std::max(smax, s);
          if (std::find(ns.begin(), ns.end(), n) == ns.end()) ns.push_back(n);
        }
        const int nspan = std::max(span, smax - smin);
        const int lw = (TY + nspan + 3) & ~3;
        const int64_t bytes = (int64_t)(nrows_g + (int)ns.size()) * 4 * lw;
        if (ccount == 0 && bytes > budget) return false;
        if (bytes > budget || ccount >= 64 / cf.dpw) break;
        span = nspan;
        nrows_g += (int)ns.size();
        ++ccount;
        ++c;
      }
      const int lw = (TY + span + 3) & ~3;
      gi.lw = lw;
      gi.c_count = ccount;
      int ri = 0;
      for (int cc = gi.c_begin; cc < gi.c_begin + ccount; ++cc) {
        int smin = INT32_MAX;
        std::vector<int> ns;
        for (int j = 0; j < DT; ++j) {
          smin = std::min(smin, gs.start[(size_t)tr[j] * C + cc]);
          const int n = gs.ntap[(size_t)tr[j] * C + cc];
          if (std::find(ns.begin(), ns.end(), n) == ns.end()) ns.push_back(n);
        }
        for (size_t k = 0; k < ns.size(); ++k) {
          out.jobs.push_back((int32_t)(T.rowidx[cc] + (ns[k] - T.nmin[cc])));
          out.jobs.push_back(smin);
        }
        for (int j = 0; j < DT; ++j) {
          const int s = gs.start[(size_t)tr[j] * C + cc], n = gs.ntap[(size_t)tr[j] * C + cc];
          const int k = (int)(std::find(ns.begin(), ns.end(), n) - ns.begin());
          out.offs[((size_t)td * DT + j) * C + cc] = (ri + k) * 4 * lw + 4 * (s - smin);
        }
        ri += (int)ns.size();
      }
      gi.njobs = ri;
      lds_max = std::max(lds_max, ri * 4 * lw);
      out.groups.push_back(gi);
    }
  }
  out.group_begin[ntd] = (int)out.groups.size();
  out.bufbytes = (lds_max + 15) & ~15;
  out.lds_bytes = 2 * out.bufbytes;
  out.ok = true;
  return true;
}

// Builds (once) the row tables in *slot and the tables of configuration ci.  Caller
// holds the plan's mutex.
static dedisp_status ensure_gather(const GatherSpec &gs, F32Tables **slot, int ci,
                                   F32CfgTables **out) {
  *out = nullptr;
  if (!*slot) {
    *slot = new (std::nothrow) F32Tables;
    if (!*slot) return fail(DEDISP_ERR_OOM, "host allocation failed");
    build_rows_f32(gs, *slot);
    DD_HIP(upload(&(*slot)->d_nmin, (*slot)->nmin));
    DD_HIP(upload(&(*slot)->d_nmax, (*slot)->nmax));
    DD_HIP(upload(&(*slot)->d_rowidx, (*slot)->rowidx));
  }
  F32Tables &T = **slot;
  F32CfgTables &c = T.cfg[ci];
  if (!T.tried[ci]) {
    T.tried[ci] = true;
    // two buffers per workgroup, 16 waves per CU, a little LDS left over
    const int budget = 79872 * kF32Cfgs[ci].nw / 16;
    if (build_f32_cfg(gs, T, ci, budget, c)) {
      DD_HIP(upload(&c.d_offs, c.offs));
      DD_HIP(upload(&c.d_groups, c.groups));
      DD_HIP(upload(&c.d_group_begin, c.group_begin));
      DD_HIP(upload(&c.d_jobs, c.jobs));
      DD_HIP(upload(&c.d_perm, c.perm));
    }
  }
  if (c.ok) *out = &c;
  return DEDISP_OK;
}

static hipError_t allow_lds(const void *fn, bool *done, std::mutex *mu) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= 64) return e;
  std::lock_guard<std::mutex> lk(*mu);
  if (!done[dev]) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kF32MaxLds);
    if (e == hipSuccess) done[dev] = true;
  }
  return e;
}

template <int R, int DPW, int NW, bool A64>
static hipError_t launch_f32_cfg(const F32Args &a, int nbatch, int lds, hipStream_t s) {
  static bool done[64] = {};
  static std::mutex mu;
  hipError_t e = allow_lds((const void *)k_dedisp_f32<R, DPW, NW, A64>, done, &mu);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_dedisp_f32<R, DPW, NW, A64>), dim3(a.ntd * a.ntt, nbatch), dim3(64 * NW),
                     lds, s, a);
  return hipGetLastError();
}

static hipError_t launch_f32(int ci, bool a64, const F32Args &a, int nbatch, int lds,
                             hipStream_t s) {
  switch (ci) {
#define DD_F32_CASE(i, r, d, w)                                               \
  case i:                                                                     \
    return a64 ? launch_f32_cfg<r, d, w, true>(a, nbatch, lds, s)             \
               : launch_f32_cfg<r, d, w, false>(a, nbatch, lds, s);
    DD_F32_CONFIGS(DD_F32_CASE)
#undef DD_F32_CASE
    default: return hipErrorInvalidValue;
  }
}

// Rows from the input (`lead` zeros in front of it and zeros past its nsamp
// samples), then the tiled sum into `nout` outputs per output row, segment by segment.
// out is fp32, or fp64 with every term added in fp64 when a64.
static dedisp_status run_gather_f32(const F32Tables &T, const F32CfgTables &cfg, int ci,
                                    const void *in, int32_t in_dtype, int64_t nsamp,
                                    int64_t in_stride, int64_t in_bstride, int32_t nbatch,
                                    int32_t nrow_ch, int32_t wmode, int32_t K, const float *w,
                                    int32_t max_span, void *out, bool a64, int64_t out_stride,
                                    int64_t out_bstride, int64_t nout, hipStream_t s,
                                    KernelTimer *kt) {
  const int TY = cfg.ty;
  const int64_t halo = 2 * (int64_t)max_span + 32;
  // time segment: as many tiles as keep the rows of all batch elements within
  // kF32RowBytesMax (at least one tile)
  const double row_bytes = 4.0 * (double)T.nrows * nbatch;
  int64_t seg = (int64_t)((double)kF32RowBytesMax / row_bytes) - halo;
  seg = std::max<int64_t>(TY, seg / TY * TY);
  seg = std::min<int64_t>(seg, (nout + TY - 1) / TY * TY);
  const int64_t ntt = seg / TY;
  if (ntt * (int64_t)cfg.ntd > INT32_MAX / 2) return DEDISP_ERR_UNSUPPORTED;
  const int64_t tpad = (seg + halo + 3) & ~(int64_t)3;
  float *Rrows = nullptr;
  DD_HIP(dev_malloc_async((void **)&Rrows, sizeof(float) * (size_t)T.nrows * tpad * nbatch, s));
  hipError_t e = hipSuccess;
  for (int64_t o0 = 0; o0 < nout && e == hipSuccess; o0 += seg) {
    const int64_t nseg = std::min(seg, nout - o0);
    const dim3 g((unsigned)((tpad + kRowTau - 1) / kRowTau), (unsigned)nrow_ch, (unsigned)nbatch);
    const int shm = (kRowTau + T.nmax_all + 4) * (int)sizeof(float);
    if (in_dtype == DEDISP_U8)
      hipLaunchKernelGGL(k_rows_f32<uint8_t>, g, dim3(kRowThreads), shm, s, (const uint8_t *)in,
                         in_stride, in_bstride, nsamp, (int64_t)T.lead, o0, tpad, T.d_nmin,
                         T.d_nmax, T.d_rowidx, T.nrows, wmode, K, w, Rrows);
    else
      hipLaunchKernelGGL(k_rows_f32<float>, g, dim3(kRowThreads), shm, s, (const float *)in,
                         in_stride, in_bstride, nsamp, (int64_t)T.lead, o0, tpad, T.d_nmin,
                         T.d_nmax, T.d_rowidx, T.nrows, wmode, K, w, Rrows);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    F32Args a{};
    a.R = Rrows;
    a.rbstride = T.nrows * tpad;
    a.tpad = tpad;
    a.bufbytes = cfg.bufbytes;
    a.ntd = cfg.ntd;
    a.ntt = (int32_t)((nseg + TY - 1) / TY);
    a.nchan = nrow_ch;
    a.offs = cfg.d_offs;
    a.groups = cfg.d_groups;
    a.group_begin = cfg.d_group_begin;
    a.jobs = cfg.d_jobs;
    a.perm = cfg.d_perm;
    a.nout = nseg;
    a.out = (char *)out + (a64 ? sizeof(double) : sizeof(float)) * o0;
    a.out_stride = out_stride;
    a.out_bstride = out_bstride;
    if (kt && o0 == 0) e = kt->begin();
    if (e == hipSuccess) e = launch_f32(ci, a64, a, nbatch, cfg.lds_bytes, s);
    if (e == hipSuccess && kt && o0 + seg >= nout) e = kt->end();
  }
  hipError_t e2 = hipFreeAsync(Rrows, s);
  if (e != hipSuccess) return hip_fail(e, "tiled fp32 gather");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
  return DEDISP_OK;
}

dedisp_status run_dedisperse_f32_tiled(dedisp_plan p, const void *in, int32_t in_dtype,
                                       int64_t nsamp, int64_t in_stride, int64_t in_bstride,
                                       int32_t nbatch, float *out, int64_t out_stride,
                                       int64_t out_bstride, int64_t nout, hipStream_t s,
                                       KernelTimer *kt) {
  if (in_dtype != DEDISP_U8 && in_dtype != DEDISP_F32) return DEDISP_ERR_UNSUPPORTED;
  if (p->max_ntap > kF32MaxTaps) return DEDISP_ERR_UNSUPPORTED;
  const int ci = p->ndm >= 256 ? 0 : 1;
  F32CfgTables *cfg = nullptr;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    GatherSpec gs;
    gs.nout_rows = p->ndm;
    gs.nrow_ch = p->nchan;
    gs.start = p->start.data();
    gs.ntap = p->ntap.data();
    gs.key = p->dm.data();
    dedisp_status st = ensure_gather(gs, &p->f32, ci, &cfg);
    if (st != DEDISP_OK) return st;
  }
  if (!cfg) return DEDISP_ERR_UNSUPPORTED;
  return run_gather_f32(*p->f32, *cfg, ci, in, in_dtype, nsamp, in_stride, in_bstride, nbatch,
                        p->nchan, p->wmode, p->ktaps, weights_of(p), p->max_span, out, false,
                        out_stride, out_bstride, nout, s, kt);
}

// zbar[b][c][tau] = sum_d g[b][d][tau - start[d][c]] (terms with the index outside
// [0, nout) are zero) for tau in [0, nz): the transpose of the one-sample-per-channel
// sum, every term added in fp64, fp64 output.  It is the same tiled gather with the
// roles swapped: outputs are channels, row channels are trials, rows are g with
// smax = max start zeros in front, and the start of (c, d) is smax - start[d][c].
dedisp_status run_adjoint_z_tiled(dedisp_plan p, const float *g, int64_t nout, int64_t gstride,
                                  int64_t gbstride, int32_t nbatch, int64_t nz, double *z,
                                  hipStream_t s) {
  const int C = p->nchan, D = p->ndm;
  const int ci = C >= 256 ? 0 : 1;
  F32CfgTables *cfg = nullptr;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->f32_adj || !p->f32_adj->tried[ci]) {
      int32_t smax = 0;
      for (int32_t v : p->start) smax = std::max(smax, v);
      std::vector<int32_t> st((size_t)C * D), nt((size_t)C * D, 1);
      std::vector<double> key(C, 0.0);   // channels with similar delays share tiles
      for (int c = 0; c < C; ++c)
        for (int d = 0; d < D; ++d) {
          st[(size_t)c * D + d] = smax - p->start[(size_t)d * C + c];
          key[c] += (double)p->start[(size_t)d * C + c];
        }
      GatherSpec gs;
      gs.nout_rows = C;
      gs.nrow_ch = D;
      gs.start = st.data();
      gs.ntap = nt.data();
      gs.key = key.data();
      const bool fresh = !p->f32_adj;
      dedisp_status e = ensure_gather(gs, &p->f32_adj, ci, &cfg);
      if (fresh && p->f32_adj) p->f32_adj->lead = smax;
      if (e != DEDISP_OK) return e;
    } else {
      F32CfgTables &c = p->f32_adj->cfg[ci];
      cfg = c.ok ? &c : nullptr;
    }
  }
  if (!cfg) return DEDISP_ERR_UNSUPPORTED;
  const F32Tables &T = *p->f32_adj;
  return run_gather_f32(T, *cfg, ci, g, DEDISP_F32, nout, gstride, gbstride, nbatch, D,
                        DEDISP_W_UNIT, 1, nullptr, T.lead + 1, z, true, nz, (int64_t)C * nz, nz,
                        s, nullptr);
}

}  // namespace dd
