// LDS read rate of the lane address patterns the matrix-core search's operand reads can
// take: every lane reads 16 bytes (ds_read_b128) or 8 bytes (ds_read_b64, issued in pairs
// 4 KiB apart), 8 reads in flight per wave, 8 waves per workgroup, 2 workgroups per CU,
// all addresses inside a 64 KiB shared array.
// Prints one JSON line per pattern: bytes per clock per CU, taking the 2.4 GHz engine
// clock.  A measurement program (not part of the library): built beside it, run by the
// benchmark's "lds" workload.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

constexpr int kPatterns = 9;
// how a lane reads: one 16-byte read, or one 8-byte read
enum Width { kB128, kB64 };
const Width kWidth[kPatterns] = {kB128, kB128, kB128, kB128, kB128, kB128, kB64, kB128, kB128};
const char *const kPatternText[kPatterns] = {
    "1 KiB contiguous (lane l at 16 l)",
    "two 512-byte halves 16 bytes out of step (lane 32 g + n at 16 n + 1040 g)",
    "two 512-byte halves in step (lane 32 g + n at 16 n + 1024 g)",
    "four 256-byte quarters at different 16-byte phases (lane 16 g + n at 16 n + 1024 g + "
    "16 ((5 g + 3) mod 16))",
    "four 256-byte quarters in step (lane 16 g + n at 16 n + 1024 g)",
    "64-byte lane stride (lane l at 64 l)",
    "8-byte reads, 512 bytes contiguous (lane l at 8 l)",
    "two halves of 16-byte reads at 8-byte steps (lane 32 g + n at 8 n + 1024 g)",
    "1 KiB contiguous, 8 bytes off 16-byte alignment (lane l at 16 l + 8)",
};

__device__ __forceinline__ int lane_offset(int pat, int lane) {
  const int n16 = lane & 15, g4 = lane >> 4, n32 = lane & 31, g2 = lane >> 5;
  switch (pat) {
    case 0: return 16 * lane;
    case 1: return 16 * n32 + 1040 * g2;
    case 2: return 16 * n32 + 1024 * g2;
    case 3: return 16 * n16 + 1024 * g4 + 16 * ((5 * g4 + 3) & 15);
    case 4: return 16 * n16 + 1024 * g4;
    case 5: return 64 * lane;
    case 6: return 8 * lane;
    case 8: return 16 * lane + 8;
    default: return 8 * n32 + 1024 * g2;   // pattern 7
  }
}

// Largest lane offset is 4032 (pattern 5); with the wave's 8 KiB half, the 16 KiB base
// and the 8 reads 4 KiB apart, the last byte read is below 57344 < 64 KiB.  Unaligned
// reads (patterns 7 and 8) stay 8-byte aligned.
__global__ void __launch_bounds__(512) k_lds_rate(int pat, int width, int iters, int *sink) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[65536];
  for (int i = threadIdx.x; i < 65536 / 4; i += 512) ((int *)lds)[i] = i;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int a = lane_offset(pat, lane) + 8192 * ((threadIdx.x >> 6) & 1) + 16384;
  v4i acc = {0, 0, 0, 0};
  if (width == kB64) {
    v2i acc2 = {0, 0};
    for (int it = 0; it < iters; ++it) {
      int ai = a;
      asm volatile("" : "+v"(ai));
      v2i v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = *(const v2i *)(lds + ai + 4096 * j);
#pragma unroll
      for (int j = 0; j < 8; ++j) acc2 += v[j];
    }
    acc[0] = acc2[0];
    acc[1] = acc2[1];
  } else {
    for (int it = 0; it < iters; ++it) {
      int ai = a;
      asm volatile("" : "+v"(ai));   // the address is opaque, so every iteration reads
      v4i v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = *(const v4i *)(lds + ai + 4096 * j);
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += v[j];
    }
  }
  if (acc[0] == 12345 && acc[1] == 678) sink[threadIdx.x] = acc[2];   // keeps the reads
}

}  // namespace

int main() {
  int *sink = nullptr;
  if (hipMalloc(&sink, 512 * sizeof(int)) != hipSuccess) return 1;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, 0) != hipSuccess) return 1;
  const int cus = prop.multiProcessorCount, blocks = 2 * cus, iters = 4000;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  for (int pat = 0; pat < kPatterns; ++pat) {
    hipLaunchKernelGGL(k_lds_rate, dim3(blocks), dim3(512), 0, 0, pat, (int)kWidth[pat], 50, sink);
    if (hipEventRecord(e0) != hipSuccess) return 1;
    hipLaunchKernelGGL(k_lds_rate, dim3(blocks), dim3(512), 0, 0, pat, (int)kWidth[pat], iters, sink);
    if (hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
    const double bytes = (double)blocks * 512 * (kWidth[pat] == kB64 ? 8 : 16) * 8 * iters;
    printf("{\"pattern\": %d, \"lanes\": \"%s\", \"ms\": %.4f, \"bytes_per_clk_per_cu\": %.1f}\n",
           pat, kPatternText[pat], ms, bytes / (ms * 1e-3) / cus / 2.4e9);
  }
  (void)hipFree(sink);
  return 0;
}
