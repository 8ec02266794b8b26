// Tile-local sum tables (Eqs. (10), (14)) fused into the scoring of one
// frame by one template (Eqs. (11)-(18)).
//
// One workgroup of four waves per tile of 64 x 16 offsets.  The tile's image
// region (16 + H rows, 64 + W columns, pixels outside the frame counted as 0)
// is read straight from the frame and its sum table is built in LDS twice:
// first of f^2, from which every offset's window sum of f^2 is taken, then of
// f, which serves the window sums of f and every segment's box sum.  Entry
// [r][c] holds the sum over the region's rows 0 .. r-1 and columns 0 .. c-1,
// modulo 2^32: a box sum is the same integer from any table origin, so the
// four-corner differences equal those of the frame's own tables.  No table of
// the frame is written to or read from HBM; the frame is read once per
// overlapping tile region, from L2 mostly.
//
// Arithmetic per offset is the batched kernel's: window sums of f and f^2,
// integer bias b = rint(sum f / n), exact energy V = n sum f^2 - (sum f)^2,
// per segment G_i = F_i - A_i b in integers and G_i c_i accumulated in FP32,
// four products per compensated (Kahan) step; rho = num / sqrt(V q_k / n).
#include <hip/hip_runtime.h>

#include "device_util.hpp"

namespace sncc {

// Four pixels x .. x + 3 of frame row y, 0 outside the frame.
__device__ __forceinline__ uint32_t fused_px4(const uint8_t *__restrict__ f, int M, int N,
                                              int f_pitch, bool dword_rows, int x, int y,
                                              uint32_t (&v)[4]) {
  if (y >= N || x >= M) {
    v[0] = v[1] = v[2] = v[3] = 0;
    return 0;
  }
  const uint8_t *row = f + (size_t)y * f_pitch;
  if (dword_rows && x + 3 < M) {
    const uint32_t w = *reinterpret_cast<const uint32_t *>(row + x);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (w >> (8 * q)) & 0xffu;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = x + q < M ? (uint32_t)row[x + q] : 0u;
  }
  return 0;
}

// The region's sum table of f (SQ false) or f^2 (SQ true) in LDS, rows
// 0 .. R, columns 0 .. C, row pitch LP words.  Row pass: each wave takes
// table rows 1 + wave, 1 + wave + NW, ...; a lane holds four pixels of each
// 256-column block, their prefix plus the wave's exclusive scan of the
// lanes' totals gives the row's running sums.  Column pass: a thread per
// column adds the rows down.
template <int LP, bool SQ>
__device__ __forceinline__ void fused_table(const uint8_t *__restrict__ f, int M, int N,
                                            int f_pitch, bool dword_rows, int x0, int y0, int R,
                                            int C, uint32_t *lds, int wave, int lane) {
  constexpr int NB = (LP + 255) / 256;  // 256-column blocks a row can span
  const int t = wave * 64 + lane;
  for (int c = t; c <= C; c += 64 * kFusedNW) lds[c] = 0;  // row 0
  for (int r = 1 + wave; r <= R; r += kFusedNW) {
    uint32_t *row = lds + r * LP;
    if (lane == 0) row[0] = 0;
    uint32_t carry = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int x = 256 * b + 4 * lane;  // region column of the lane's first pixel
      if (256 * b >= C) break;           // uniform
      uint32_t v[4];
      fused_px4(f, M, N, f_pitch, dword_rows, x0 + x, y0 + r - 1, v);
      uint32_t p[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t e = x + q < C ? (SQ ? v[q] * v[q] : v[q]) : 0u;
        p[q] = (q ? p[q - 1] : 0u) + e;
      }
      const uint32_t inc = wave_incl_scan(p[3]);
      const uint32_t base = carry + inc - p[3];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (x + q < C) row[1 + x + q] = base + p[q];
      carry += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
    }
  }
  __syncthreads();
  for (int c = 1 + t; c <= C; c += 64 * kFusedNW) {
    uint32_t acc = 0;
    int r = 1;
    for (; r + 8 <= R + 1; r += 8) {
      uint32_t e[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) e[j] = lds[(r + j) * LP + c];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        acc += e[j];
        lds[(r + j) * LP + c] = acc;
      }
    }
    for (; r <= R; ++r) {
      acc += lds[r * LP + c];
      lds[r * LP + c] = acc;
    }
  }
  __syncthreads();
}

template <int LP>
__global__ __launch_bounds__(64 * kFusedNW) void fused_kernel(
    const uint8_t *__restrict__ f, int M, int N, int f_pitch, int W, int H, int K, int nu,
    int nv, int ntu, const int4 *__restrict__ geom, const int *__restrict__ area,
    const float *__restrict__ c32, double q_k, float *__restrict__ rho, int rho_pitch,
    uint8_t *__restrict__ degen, long long *__restrict__ energy) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int tv = blockIdx.x / ntu, tu = blockIdx.x - tv * ntu;
  const int u0 = tu * kFusedBU, v0 = tv * kFusedBV;
  const int R = kFusedBV + H, C = kFusedBU + W;
  const bool dword_rows = (f_pitch & 3) == 0;
  const int n = W * H;
  // the lane's offsets: column `lane`, rows wave * RV + dv of the tile
  const uint32_t *mine = lds + (wave * kFusedRV) * LP + lane;
  constexpr int RV = kFusedRV;
  const int oW = W, oH = H * LP;

  uint32_t sf2[RV], sf[RV];
  fused_table<LP, true>(f, M, N, f_pitch, dword_rows, u0, v0, R, C, lds, wave, lane);
#pragma unroll
  for (int dv = 0; dv < RV; ++dv) {
    const uint32_t *a = mine + dv * LP;
    sf2[dv] = (a[oH + oW] - a[oH]) - (a[oW] - a[0]);  // Eq. (15)
  }
  __syncthreads();
  fused_table<LP, false>(f, M, N, f_pitch, dword_rows, u0, v0, R, C, lds, wave, lane);

  int nb[RV];
  float scale[RV], acc[RV], cmp[RV];
  long long V[RV];
  const float inv_n = 1.0f / (float)n;
  const double qnd = q_k / (double)n;
#pragma unroll
  for (int dv = 0; dv < RV; ++dv) {
    const uint32_t *a = mine + dv * LP;
    sf[dv] = (a[oH + oW] - a[oH]) - (a[oW] - a[0]);  // Eq. (13)
    nb[dv] = -(int)__builtin_rintf((float)sf[dv] * inv_n);
    // n * sum f^2 - (sum f)^2 as one FP64 fma of integers below 2^53: exact
    const double fs = (double)sf[dv];
    const double Vd = __builtin_fma((double)n, (double)sf2[dv], -(fs * fs));
    V[dv] = (long long)Vd;
    scale[dv] = Vd == 0.0 ? 0.f : __builtin_amdgcn_rsqf((float)(Vd * qnd));
    acc[dv] = 0.f;
    cmp[dv] = 0.f;
  }

  // per-segment terms (Eqs. (11), (12)): four corners from LDS per offset
  for (int i = 0; i < K; i += 4) {
    float y[RV];
#pragma unroll
    for (int dv = 0; dv < RV; ++dv) y[dv] = -cmp[dv];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (i + q < K) {  // uniform
        const int4 g = geom[i + q];  // x, y, width, height
        const int A = area[i + q];
        const float c = c32[i + q];
        const uint32_t *t0 = mine + g.y * LP + g.x;
        const uint32_t *t1 = t0 + g.w * LP;
#pragma unroll
        for (int dv = 0; dv < RV; ++dv) {
          const int o = dv * LP;
          const uint32_t F = (t1[o + g.z] - t1[o]) - (t0[o + g.z] - t0[o]);  // Eq. (11)
          const int G = (int)F + __mul24(A, nb[dv]);
          y[dv] = __builtin_fmaf((float)G, c, y[dv]);
        }
      }
    }
#pragma unroll
    for (int dv = 0; dv < RV; ++dv) {
      const float s = acc[dv] + y[dv];
      cmp[dv] = (s - acc[dv]) - y[dv];
      acc[dv] = s;
    }
  }

  // epilogue: rho = num / sqrt(V q_k / n) (Eqs. (17), (18))
  const int u = u0 + lane;
#pragma unroll
  for (int dv = 0; dv < RV; ++dv) {
    const int v = v0 + wave * RV + dv;
    if (u < nu && v < nv) {
      const long long o = (long long)v * rho_pitch + u;
      rho[o] = (acc[dv] - cmp[dv]) * scale[dv];
      if (degen) degen[o] = scale[dv] == 0.f ? 1 : 0;
      if (energy) energy[o] = V[dv];
    }
  }
}

int launch_fused(const FusedArgs &a, hipStream_t st) {
  const int LP = fused_lp(a.W);
  const size_t lds = fused_lds_bytes(a.W, a.H);
  if (!LP || lds > (size_t)kFusedMaxLds) return -1;
  const int ntu = (a.nu + kFusedBU - 1) / kFusedBU, ntv = (a.nv + kFusedBV - 1) / kFusedBV;
  const dim3 grid((unsigned)(ntu * ntv)), block(64 * kFusedNW);
#define SNCC_FUSED(LPV)                                                                        \
  case LPV: {                                                                                  \
    static bool attr = false;                                                                  \
    if (!attr) {                                                                               \
      if (hipFuncSetAttribute((const void *)fused_kernel<LPV>,                                 \
                              hipFuncAttributeMaxDynamicSharedMemorySize,                      \
                              kFusedMaxLds) != hipSuccess)                                     \
        return -1;                                                                             \
      attr = true;                                                                             \
    }                                                                                          \
    hipLaunchKernelGGL(fused_kernel<LPV>, grid, block, lds, st, a.f, a.M, a.N, a.f_pitch, a.W, \
                       a.H, a.K, a.nu, a.nv, ntu, a.geom, a.area, a.c32, a.q_k, a.rho,         \
                       a.rho_pitch, a.degen, a.energy);                                        \
    break;                                                                                     \
  }
  switch (LP) {
    SNCC_FUSED(128)
    SNCC_FUSED(160)
    SNCC_FUSED(192)
    SNCC_FUSED(224)
    SNCC_FUSED(256)
    SNCC_FUSED(288)
    SNCC_FUSED(320)
    SNCC_FUSED(384)
    SNCC_FUSED(448)
    SNCC_FUSED(512)
    SNCC_FUSED(576)
    default:
      return -1;
  }
#undef SNCC_FUSED
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sncc
