#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
// LDS read bandwidth per CU for four read forms (a measurement program, not
// part of the library): the peak that the benchmark reports the scoring
// kernel's LDS traffic against.  Each workgroup of four waves fills 16 KB of
// LDS and reads it in a loop, eight independent reads per iteration; every
// index is masked into the buffer, the eight reads of an iteration touch
// distinct words (their results are combined by xor, so equal reads would
// cancel and could be removed), and the per-iteration base is made opaque
// with an empty asm so that no read is hoisted out of the loop.  32
// workgroups per CU.
//
// Built by paper_2502_01286_amd/build.py as paper_2502_01286_amd/lds_probe:
//   hipcc -O3 -std=c++17 -x hip --offload-arch=gfx950 (packed FP32 off) lds_probe.hip
constexpr int WORDS = 4096, MASK = WORDS - 1;
template <int MODE>
__global__ __launch_bounds__(256) void lds_bw(uint32_t *out, int iters) {
  __shared__ __align__(16) uint32_t buf[WORDS];
  for (int i = threadIdx.x; i < WORDS; i += 256) buf[i] = i * 2654435761u;
  __syncthreads();
  uint32_t acc = 0;
  int base = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
    asm volatile("" : "+v"(base));
    if (MODE == 0) {  // ds_read_b32, 8 per iteration
#pragma unroll
      for (int k = 0; k < 8; ++k) acc ^= buf[(base + k * 256) & MASK];
    } else if (MODE == 1) {  // pairs 64 words apart (ds_read2st64_b32), 8 pairs
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int a = (base + k * 512) & (MASK & ~127);
        const int l = threadIdx.x & 63;
        acc ^= buf[a + l] + buf[a + l + 64];
      }
    } else if (MODE == 2) {  // ds_read_b64, 8 per iteration
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int a = ((base + k * 256) * 2) & (MASK & ~1);
        const uint2 v = *reinterpret_cast<const uint2 *>(&buf[a]);
        acc ^= v.x + v.y;
      }
    } else {  // ds_read_b128, 8 per iteration
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int a = (base * 4 + k * 256) & (MASK & ~3);
        const uint4 v = *reinterpret_cast<const uint4 *>(&buf[a]);
        acc ^= v.x + v.y + v.z + v.w;
      }
    }
    base += 64;
  }
  out[blockIdx.x * 256 + threadIdx.x] = acc;
}
template <int MODE>
double run(uint32_t *d, int grid, int iters) {
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  hipLaunchKernelGGL(lds_bw<MODE>, dim3(grid), dim3(256), 0, 0, d, 16);
  hipEventRecord(a);
  hipLaunchKernelGGL(lds_bw<MODE>, dim3(grid), dim3(256), 0, 0, d, iters);
  hipEventRecord(b);
  hipEventSynchronize(b);
  float ms = 0;
  hipEventElapsedTime(&ms, a, b);
  return ms;
}
int main() {
  int dev = 0, cus = 0, clk = 0;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  hipDeviceGetAttribute(&clk, hipDeviceAttributeClockRate, dev);  // kHz
  const int grid = cus * 32, iters = 2048;  // 16 KB each: up to ten per CU at once
  uint32_t *d;
  if (hipMalloc(&d, (size_t)grid * 256 * 4)) return 1;
  const double bytes_per_iter[4] = {8 * 256.0, 8 * 512.0, 8 * 512.0, 8 * 1024.0};
  const char *names[4] = {"ds_read_b32", "ds_read2st64_b32 (pairs)", "ds_read_b64", "ds_read_b128"};
  printf("CUs %d, max clock %d MHz\n", cus, clk / 1000);
  for (int m = 0; m < 4; ++m) {
    double ms = m == 0 ? run<0>(d, grid, iters) : m == 1 ? run<1>(d, grid, iters)
              : m == 2 ? run<2>(d, grid, iters) : run<3>(d, grid, iters);
    const double bytes = (double)grid * 4 /*waves*/ * iters * bytes_per_iter[m];
    const double per_clk = bytes / (ms * 1e-3) / (clk * 1e3) / cus;
    printf("%-28s %8.3f ms  %8.1f TB/s  %7.1f B/clk/CU at %d MHz\n", names[m], ms,
           bytes / (ms * 1e-3) / 1e12, per_clk, clk / 1000);
  }
  return hipDeviceSynchronize() == hipSuccess ? 0 : 2;
}
