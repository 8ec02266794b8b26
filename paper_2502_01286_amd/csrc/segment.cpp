// Host-side segmented template approximation (split-and-merge).
//
// precompute_template_approximation, split_segment and
// merge_redundant_segments of Section 5 (same results, computed with a work
// list and a corner grid); the deviation test is Eq. (2).
// Sums over a rectangle come from an int64 summed-area table of the template,
// so every split decision costs O(1).  The test "population standard
// deviation < sigma_max" is decided exactly: with S = sum t, S2 = sum t^2 and
// area A, it is A*S2 - S^2 < sigma_max^2 * A^2, where sigma_max = m * 2^e is
// the exact binary value of the double; both sides are compared as 256-bit
// integers.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "sncc_internal.hpp"

namespace sncc {

namespace {

typedef unsigned __int128 u128;

// 256-bit unsigned integer, little-endian 64-bit limbs.
struct U256 {
  uint64_t w[4];
};

U256 mul128(u128 a, u128 b) {
  uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64);
  uint64_t b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
  u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0,
       p11 = (u128)a1 * b1;
  U256 r;
  r.w[0] = (uint64_t)p00;
  u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
  r.w[1] = (uint64_t)mid;
  u128 hi = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + (uint64_t)p11;
  r.w[2] = (uint64_t)hi;
  r.w[3] = (uint64_t)((hi >> 64) + (p11 >> 64));
  return r;
}

U256 shl(U256 x, int s) {  // 0 <= s < 256, caller ensures no overflow
  U256 r = {{0, 0, 0, 0}};
  int limb = s / 64, bit = s % 64;
  for (int i = 3; i >= 0; --i) {
    int src = i - limb;
    if (src < 0) continue;
    uint64_t v = x.w[src] << bit;
    if (bit && src > 0) v |= x.w[src - 1] >> (64 - bit);
    r.w[i] = v;
  }
  return r;
}

int bitlen(U256 x) {
  for (int i = 3; i >= 0; --i)
    if (x.w[i]) return 64 * i + 64 - __builtin_clzll(x.w[i]);
  return 0;
}

bool less(U256 a, U256 b) {
  for (int i = 3; i >= 0; --i)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i];
  return false;
}

U256 from128(u128 a) {
  U256 r = {{(uint64_t)a, (uint64_t)(a >> 64), 0, 0}};
  return r;
}

}  // namespace

// Eq. (2) with a strict '<', exactly: A*S2 - S^2 < sigma^2 * A^2.
bool std_below(int64_t S, int64_t S2, int64_t A, double sigma) {
  if (!(sigma > 0) || std::isinf(sigma) || std::isnan(sigma))
    return std::isinf(sigma) && sigma > 0;
  __int128 lhs_s = (__int128)A * S2 - (__int128)S * S;
  if (lhs_s < 0) lhs_s = 0;  // cannot happen for integer data
  u128 lhs = (u128)lhs_s;
  int e;
  double fr = std::frexp(sigma, &e);  // sigma = fr * 2^e, fr in [0.5, 1)
  uint64_t m = (uint64_t)std::ldexp(fr, 53);
  e -= 53;
  while (m && !(m & 1)) {  // make the mantissa odd
    m >>= 1;
    ++e;
  }
  u128 X = (u128)m * (u128)A;  // m < 2^53, A < 2^40 -> fits
  if (lhs == 0) return X > 0;
  U256 R = mul128(X, X);        // m^2 A^2
  U256 L = from128(lhs);
  if (e >= 0) {  // lhs < sigma^2 A^2 = R * 4^e
    if (bitlen(R) + 2 * e >= 256) return true;
    return less(L, shl(R, 2 * e));
  }
  int s = -2 * e;  // lhs * 4^(-e) < R
  if (bitlen(L) + s >= 256) return false;  // R < 2^(2*93)
  return less(shl(L, s), R);
}

namespace {

// Pixel sums of the template over rectangles from integral images of t and
// t^2 (int64, (H + 1) x (W + 1), zero first row and column).
struct Tables {
  std::vector<int64_t> s, s2;
  int P;  // row pitch, W + 1
  int64_t box(const std::vector<int64_t> &t, int x, int y, int w, int h) const {
    return t[(size_t)(y + h) * P + x + w] - t[(size_t)(y + h) * P + x] -
           t[(size_t)y * P + x + w] + t[(size_t)y * P + x];
  }
};

struct Rect {
  int x, y, w, h;
};

// The halving rule of split_segment: a rectangle is kept when it is one
// pixel or when its population deviation is below sigma (Eq. (2)); otherwise
// it is cut across its larger side (the width when w > h), the first part
// taking the ceiling.  Rectangles wait on an explicit work list; the leaves
// come out in the list's order, which neither the leaf count nor the merged
// result depends on.
void split_leaves(const Tables &tb, double sigma, int W, int H, std::vector<Seg> &leaves) {
  std::vector<Rect> todo;
  todo.push_back(Rect{0, 0, W, H});
  while (!todo.empty()) {
    const Rect r = todo.back();
    todo.pop_back();
    const int64_t S = tb.box(tb.s, r.x, r.y, r.w, r.h);
    const int64_t A = (int64_t)r.w * r.h;
    if (A == 1 || std_below(S, tb.box(tb.s2, r.x, r.y, r.w, r.h), A, sigma)) {
      leaves.push_back(Seg{r.x, r.y, r.w, r.h, S, A});
    } else if (r.w > r.h) {
      const int a = (r.w + 1) / 2;
      todo.push_back(Rect{r.x + a, r.y, r.w - a, r.h});
      todo.push_back(Rect{r.x, r.y, a, r.h});
    } else {
      const int a = (r.h + 1) / 2;
      todo.push_back(Rect{r.x, r.y + a, r.w, r.h - a});
      todo.push_back(Rect{r.x, r.y, r.w, a});
    }
  }
}

bool same_mean(const Seg &a, const Seg &b) {
  return (__int128)a.sum * b.area == (__int128)b.sum * a.area;
}

}  // namespace

// merge_redundant_segments, as rounds over a grid of the template's pixels
// that holds, at the top-left corner of every live segment, its index (-1
// elsewhere).  In a round every maximal vertical run (segments of equal x and
// width, each starting where the one above ends, equal exact means) becomes
// its top segment, then every maximal horizontal run (equal y and height,
// side by side, equal means) its leftmost one; rounds repeat until one merges
// nothing.  The neighbour below segment s starts at (x_s, y_s + h_s), the one
// to its right at (x_s + w_s, y_s); a row-major walk over the grid reaches a
// run's first segment before the rest of the run.  The segments of a
// partition have distinct corners, so each grid cell holds at most one.  The
// result lists the segments in row-major order of their corners.
void merge_segments(std::vector<Seg> &k, int W, int H) {
  std::vector<int> at((size_t)W * H, -1);
  for (size_t i = 0; i < k.size(); ++i) at[(size_t)k[i].y * W + k[i].x] = (int)i;
  for (bool merged = true; merged;) {
    merged = false;
    for (int vertical = 1; vertical >= 0; --vertical) {
      for (size_t cell = 0; cell < at.size(); ++cell) {
        if (at[cell] < 0) continue;
        Seg &s = k[at[cell]];
        for (;;) {
          const int nx = vertical ? s.x : s.x + s.w, ny = vertical ? s.y + s.h : s.y;
          if (nx >= W || ny >= H) break;
          const size_t nc = (size_t)ny * W + nx;
          if (at[nc] < 0) break;
          const Seg &t = k[at[nc]];
          if ((vertical ? t.w != s.w : t.h != s.h) || !same_mean(s, t)) break;
          if (vertical)
            s.h += t.h;
          else
            s.w += t.w;
          s.sum += t.sum;
          s.area += t.area;
          at[nc] = -1;
          merged = true;
        }
      }
    }
  }
  std::vector<Seg> out;
  for (size_t cell = 0; cell < at.size(); ++cell)
    if (at[cell] >= 0) out.push_back(k[at[cell]]);
  k.swap(out);
}

int segment_template(const uint8_t *t, int W, int H, int stride, double sigma,
                     int K_max, std::vector<Seg> &out, int *k_before_merge,
                     double *sigma_used, double *rho_max) {
  Tables tb;
  tb.P = W + 1;
  const int P = tb.P;
  tb.s.assign((size_t)(H + 1) * P, 0);
  tb.s2.assign((size_t)(H + 1) * P, 0);
  for (int y = 0; y < H; ++y) {
    int64_t row = 0, row2 = 0;
    for (int x = 0; x < W; ++x) {
      int64_t v = t[(size_t)y * stride + x];
      row += v;
      row2 += v * v;
      tb.s[(size_t)(y + 1) * P + x + 1] = tb.s[(size_t)y * P + x + 1] + row;
      tb.s2[(size_t)(y + 1) * P + x + 1] = tb.s2[(size_t)y * P + x + 1] + row2;
    }
  }
  std::vector<Seg> leaves;
  double used = sigma;
  for (;;) {  // the K_max loop: raise the threshold by one until K <= K_max
    leaves.clear();
    split_leaves(tb, sigma, W, H, leaves);
    used = sigma;
    sigma = sigma + 1.0;
    if ((int64_t)leaves.size() <= K_max) break;
  }
  if (k_before_merge) *k_before_merge = (int)leaves.size();
  if (sigma_used) *sigma_used = used;
  merge_segments(leaves, W, H);
  out = leaves;

  const int64_t n = (int64_t)W * H;
  const int64_t T = tb.s[(size_t)H * P + W];
  bool uniform = true;
  for (const Seg &s : out)
    if ((__int128)s.sum * n != (__int128)T * s.area) uniform = false;
  if (uniform) return SNCC_EDEGENERATE;

  if (rho_max) {
    // steps 4-7 of precompute_template_approximation, area-weighted Eq. (17)
    double kbar = 0;
    for (const Seg &s : out) kbar += (double)s.area * ((double)s.sum / (double)s.area);
    kbar /= (double)n;
    double tbar = (double)T / (double)n;
    double num = 0, qk = 0;
    for (const Seg &s : out) {
      double c = (double)s.sum / (double)s.area - kbar;
      num += ((double)s.sum - tbar * (double)s.area) * c;
      qk += (double)s.area * c * c;
    }
    double qt = 0;
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        double d = (double)t[(size_t)y * stride + x] - tbar;
        qt += d * d;
      }
    *rho_max = num / std::sqrt(qt * qk);
  }
  return SNCC_OK;
}

}  // namespace sncc
