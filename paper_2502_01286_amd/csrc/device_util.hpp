// Device helpers shared by the HIP kernels: wavefront scans and maxima over
// DPP, 64-bit lane reads, the order-preserving float code and selection key,
// the register-resident per-wave top-k list, and raw buffer access.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sncc_internal.hpp"

namespace sncc {

typedef unsigned long long u64;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  // Hillis-Steele within rows of 16 lanes, then row broadcasts (GFX9 DPP).
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
  return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), 63);
}

__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
  // running maximum over lanes (same DPP pattern as the scan)
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
  return v;
}

// Value of lane `src` (wave-uniform) of a 64-bit register.
__device__ __forceinline__ u64 lane_u64(u64 x, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), src);
  return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ u64 shfl_up_u64(u64 x, int d) {
  unsigned lo = (unsigned)__shfl_up((int)(unsigned)x, d);
  unsigned hi = (unsigned)__shfl_up((int)(unsigned)(x >> 32), d);
  return ((u64)hi << 32) | lo;
}

// Maximum of a 64-bit key over the wave: the high words first, then the
// low words among the lanes holding the highest high word.
__device__ __forceinline__ u64 wave_max_u64(u64 x) {
  const uint32_t hi = (uint32_t)(x >> 32);
  const uint32_t mh = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(hi), 63);
  const uint32_t lo = hi == mh ? (uint32_t)x : 0u;
  const uint32_t ml = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(lo), 63);
  return ((u64)mh << 32) | ml;
}

// Order-preserving map of a float to uint32 (larger float -> larger code).
__device__ __forceinline__ uint32_t float_order(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float float_unorder(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  return __uint_as_float(u);
}

// Selection key: higher rho first, then smaller row-major offset index.
__device__ __forceinline__ u64 make_key(float rho, int idx) {
  return ((u64)float_order(rho) << 32) | (u64)(0xffffffffu - (uint32_t)idx);
}

// Per-wave top-k list: lane j < k holds the j-th best key (0 = empty).
// Inserts a wave-uniform key that beats the current k-th entry.
__device__ __forceinline__ void topk_insert(u64 &lkey, u64 key, int k, int lane) {
  const bool better = lane < k && lkey > key;
  const int pos = __popcll(__ballot(better));
  const u64 up = shfl_up_u64(lkey, 1);
  if (lane == pos)
    lkey = key;
  else if (lane > pos && lane < k)
    lkey = up;
}

// Offers R candidate keys per lane (0 = none) to the wave's list.  Keys not
// above `floor` (a key known to have k better keys elsewhere) are dropped.
template <int R>
__device__ __forceinline__ void topk_offer(u64 &lkey, u64 (&cand)[R], int k, int lane,
                                           u64 floor = 0) {
  u64 thr = lane_u64(lkey, k - 1);
  thr = thr > floor ? thr : floor;
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (cand[r] <= thr) cand[r] = 0;
  for (;;) {
    u64 best = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) best = cand[r] > best ? cand[r] : best;
    if (__ballot(best != 0) == 0) break;
    best = wave_max_u64(best);
    topk_insert(lkey, best, k, lane);
    thr = lane_u64(lkey, k - 1);
    thr = thr > floor ? thr : floor;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (cand[r] == best || cand[r] <= thr) cand[r] = 0;
  }
}

// Value of lane l ^ m of a 64-bit register.
__device__ __forceinline__ u64 shfl_xor_u64(u64 x, int m) {
  const unsigned lo = (unsigned)__shfl_xor((int)(unsigned)x, m);
  const unsigned hi = (unsigned)__shfl_xor((int)(unsigned)(x >> 32), m);
  return ((u64)hi << 32) | lo;
}

// Bitonic sort of one 64-bit key per lane across the wave: afterwards lane j
// holds the j-th largest key.
__device__ __forceinline__ u64 wave_sort_desc_u64(u64 key, int lane) {
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1)
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const u64 other = shfl_xor_u64(key, stride);
      // pairs (l, l ^ stride) inside blocks of `size` lanes: descending
      // blocks where bit `size` of l is 0, ascending otherwise
      const bool desc = (lane & size) == 0 || size == 64;
      const bool lower = (lane & stride) == 0;
      const u64 hi = key > other ? key : other, lo = key > other ? other : key;
      key = (lower == desc) ? hi : lo;
    }
  return key;
}

// Merges a wave-sorted list of keys (`sorted`, lane j the j-th largest) into
// the top-k list `lkey` (lane j < k the j-th best): the k best of both.  The
// lane-wise maxima of one list and the other reversed form a bitonic
// sequence holding the 64 largest keys of the union, which six
// compare-exchange steps put in descending order.
__device__ __forceinline__ void topk_merge_sorted(u64 &lkey, u64 sorted, int k, int lane) {
  const unsigned rlo = (unsigned)__shfl((int)(unsigned)sorted, 63 - lane);
  const unsigned rhi = (unsigned)__shfl((int)(unsigned)(sorted >> 32), 63 - lane);
  const u64 rev = ((u64)rhi << 32) | rlo;
  const u64 mine = lane < k ? lkey : 0;
  u64 c = mine > rev ? mine : rev;
#pragma unroll
  for (int stride = 32; stride > 0; stride >>= 1) {
    const u64 other = shfl_xor_u64(c, stride);
    const bool lower = (lane & stride) == 0;
    const u64 hi = c > other ? c : other, lo = c > other ? other : c;
    c = lower ? hi : lo;
  }
  lkey = lane < k ? c : 0;
}

// Batched offers to a wave's top-k list, for a batch of many keys.  Keys
// above the list's k-th key (and above `floor`) are appended to a 64-entry
// buffer in LDS (low words at lo[j], high words at hi[j], j < 64, stored
// as float bit patterns; the wave's own memory); a full buffer, and finally the remainder, is sorted
// across the lanes and merged into the list.  The k-th key that filters is
// that of the last merge, never above the current one, so no key of the
// final top k is dropped.
__device__ __forceinline__ void topk_flush(u64 &lkey, float *lo, float *hi, int &cnt, int k,
                                           int lane) {
  const u64 b = lane < cnt ? ((u64)__float_as_uint(hi[lane]) << 32) | __float_as_uint(lo[lane])
                           : 0;
  topk_merge_sorted(lkey, wave_sort_desc_u64(b, lane), k, lane);
  cnt = 0;
}

template <int R>
__device__ __forceinline__ void topk_offer_batched(u64 &lkey, const u64 (&cand)[R], int k,
                                                   int lane, u64 floor, float *lo, float *hi) {
  int cnt = 0;
  u64 thr = lane_u64(lkey, k - 1);
  thr = thr > floor ? thr : floor;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    bool take = cand[r] > thr;
    u64 m = __ballot(take);
    if (m == 0) continue;
    if (cnt + __popcll(m) > 64) {
      topk_flush(lkey, lo, hi, cnt, k, lane);
      thr = lane_u64(lkey, k - 1);
      thr = thr > floor ? thr : floor;
      take = cand[r] > thr;
      m = __ballot(take);
      if (m == 0) continue;
    }
    const int j = cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (take) {
      lo[j] = __uint_as_float((uint32_t)cand[r]);
      hi[j] = __uint_as_float((uint32_t)(cand[r] >> 32));
    }
    cnt += __popcll(m);
  }
  if (cnt > 0) topk_flush(lkey, lo, hi, cnt, k, lane);
}

// Exact selection keys for FP64 values: the order-preserving 64-bit code of
// the double (larger value -> larger code) and a 32-bit word that breaks ties
// by the smaller index (its complement).  (0, 0) is the empty key.
__device__ __forceinline__ u64 double_order(double d) {
  const u64 u = (u64)__double_as_longlong(d);
  return (u >> 63) ? ~u : (u | (1ull << 63));
}
__device__ __forceinline__ double double_unorder(u64 o) {
  return __longlong_as_double((long long)((o >> 63) ? (o & ~(1ull << 63)) : ~o));
}
__device__ __forceinline__ bool key96_gt(u64 ah, uint32_t al, u64 bh, uint32_t bl) {
  return ah > bh || (ah == bh && al > bl);
}

// Per-wave top-k list of 96-bit keys: lane j < k holds the j-th best.
__device__ __forceinline__ void topk96_insert(u64 &lh, uint32_t &ll, u64 kh, uint32_t kl, int k,
                                              int lane) {
  const bool better = lane < k && key96_gt(lh, ll, kh, kl);
  const int pos = __popcll(__ballot(better));
  const u64 uh = shfl_up_u64(lh, 1);
  const uint32_t ul = (uint32_t)__shfl_up((int)ll, 1);
  if (lane == pos) {
    lh = kh;
    ll = kl;
  } else if (lane > pos && lane < k) {
    lh = uh;
    ll = ul;
  }
}

// Largest 96-bit key over the wave (high parts first, then the low words of
// the lanes holding the largest high part).
__device__ __forceinline__ void wave_max96(u64 h, uint32_t l, u64 &mh, uint32_t &ml) {
  mh = wave_max_u64(h);
  const uint32_t lo = h == mh ? l : 0u;
  ml = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(lo), 63);
}

// Buffer resource over `bytes` bytes at `p` (GFX9 raw buffer: loads at or
// beyond `bytes` return zero).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                           0x00020000);
}

// Four-corner box sum of a window (Eqs. (13), (15)) through a buffer
// resource: corners at byte offsets 0, cW, cH, cH + cW from voff + so.
__device__ __forceinline__ uint32_t window_box(__amdgpu_buffer_rsrc_t r, int voff, int so, int cW,
                                               int cH) {
  const uint32_t a00 = __builtin_amdgcn_raw_buffer_load_b32(r, voff, so, 0);
  const uint32_t a01 = __builtin_amdgcn_raw_buffer_load_b32(r, voff, so + cW, 0);
  const uint32_t a10 = __builtin_amdgcn_raw_buffer_load_b32(r, voff, so + cH, 0);
  const uint32_t a11 = __builtin_amdgcn_raw_buffer_load_b32(r, voff, so + cH + cW, 0);
  return (a11 - a10) - (a01 - a00);
}

// The four corner entries of a window through a buffer resource (top-left,
// top-right, bottom-left, bottom-right at byte offsets voff + so, + cW, + cH,
// + cH + cW; so is wave-uniform); its box sum is (c[3] - c[2]) - (c[1] - c[0]).
__device__ __forceinline__ void window_corners(__amdgpu_buffer_rsrc_t r, int voff, int so, int cW,
                                               int cH, uint32_t (&c)[4]) {
  c[0] = __builtin_amdgcn_raw_buffer_load_b32(r, voff, so, 0);
  c[1] = __builtin_amdgcn_raw_buffer_load_b32(r, voff, so + cW, 0);
  c[2] = __builtin_amdgcn_raw_buffer_load_b32(r, voff, so + cH, 0);
  c[3] = __builtin_amdgcn_raw_buffer_load_b32(r, voff, so + cH + cW, 0);
}

// Sum of f^2 over a W x H window (Eq. (15)) as an exact 64-bit value.  Each
// box of at most kMaxSqBoxArea pixels is exact as a difference of four
// entries of the modulo-2^32 table, so the window is taken in bands of
// `band` rows (band * W <= kMaxSqBoxArea) and the band sums are added in
// 64 bits.  Buffer form: corners at voff + so (+ cW for the right column),
// `rowb` bytes per table row.
__device__ __forceinline__ u64 window_sq(__amdgpu_buffer_rsrc_t r, int voff, int so, int cW,
                                         int rowb, int H, int band) {
  if (band >= H) return window_box(r, voff, so, cW, H * rowb);
  u64 acc = 0;
  for (int y = 0; y < H; y += band) {
    const int h = min(band, H - y);
    acc += window_box(r, voff, so + y * rowb, cW, h * rowb);
  }
  return acc;
}

// Pointer form: a0 is the window's top-left table entry, P the row pitch.
__device__ __forceinline__ u64 window_sq(const uint32_t *__restrict__ a0, int W, int H, int P,
                                         int band) {
  u64 acc = 0;
  for (int y = 0; y < H; y += band) {
    const int h = min(band, H - y);
    const uint32_t *t0 = a0 + (long long)y * P, *t1 = t0 + (long long)h * P;
    acc += (uint32_t)((t1[W] - t1[0]) - (t0[W] - t0[0]));
  }
  return acc;
}

}  // namespace sncc
