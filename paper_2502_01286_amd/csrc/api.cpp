// C-ABI of libsncc: argument checks, device memory of handles, the tile
// planner (LDS passes, work list) and the graph-captured batch.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "sncc_internal.hpp"

namespace sncc {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

}  // namespace sncc

using namespace sncc;

#define SNCC_FAIL(code, ...)  \
  do {                        \
    set_error(__VA_ARGS__);   \
    return (code);            \
  } while (0)

#define HIPCHK(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) SNCC_FAIL(SNCC_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

#define CHK(x)                 \
  do {                         \
    int r_ = (x);              \
    if (r_ != SNCC_OK) return r_; \
  } while (0)

namespace {

// Failure injection for tests of the allocation-failure paths: with
// SNCC_TEST_FAIL_ALLOC set to a positive byte count in the environment, every
// device allocation of at least that many bytes fails as if the device were
// out of memory (read at each allocation, so a test can set and clear it).
// With SNCC_TEST_QUEUES=1 in the environment, scoring launches that would run
// one workgroup per item use the work queues instead (read at each launch), so
// that a test can compare the two forms on the same call.
bool queues_forced() {
  const char *v = std::getenv("SNCC_TEST_QUEUES");
  return v && v[0] == '1';
}

bool alloc_fails_by_request(size_t n) {
  const char *v = std::getenv("SNCC_TEST_FAIL_ALLOC");
  if (!v || !*v) return false;
  const long long lim = std::atoll(v);
  return lim > 0 && (long long)n >= lim;
}

// Device buffer owned by a handle; grows on demand, freed on destruction.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  int reserve(size_t n) {
    if (n <= bytes) return SNCC_OK;
    if (p) {
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    if (alloc_fails_by_request(n))
      SNCC_FAIL(SNCC_ENOMEM, "hipMalloc(%zu): refused (SNCC_TEST_FAIL_ALLOC)", n);
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      SNCC_FAIL(SNCC_ENOMEM, "hipMalloc(%zu): %s", n, hipGetErrorString(e));
    }
    bytes = n;
    return SNCC_OK;
  }
  template <class T>
  int upload(const std::vector<T> &v, hipStream_t st) {
    const size_t n = std::max<size_t>(v.size() * sizeof(T), 16);
    CHK(reserve(n));
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T),
                                          hipMemcpyHostToDevice, st));
    return SNCC_OK;
  }
  template <class T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

// ------------------------------------------------------------------ handles
struct PlanDev;

// Everything a one-call tile plan depends on: a repeated call with an equal
// key reuses the plan already on the device instead of building and
// uploading it again.
struct PlanKey {
  int sink = -1;
  uint64_t tmpl = 0, tmpl2 = 0;  // serials of the template sets (0: none)
  int M = 0, N = 0, P = 0, k = 0;
  std::vector<int32_t> pairs;
  std::vector<double> thr;       // thresholds the plan carries
  bool operator==(const PlanKey &o) const {
    return sink == o.sink && tmpl == o.tmpl && tmpl2 == o.tmpl2 && M == o.M && N == o.N &&
           P == o.P && k == o.k && pairs == o.pairs && thr == o.thr;
  }
};

struct sncc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  DevBuf sat_scratch;
  DevBuf map_scratch;
  DevBuf frame_s, frame_s2;  // one frame's tables (global form of sncc_score_frame)
  std::vector<std::unique_ptr<PlanDev>> retired;  // awaiting completion
  bool timing = false;                             // record stage events
  hipEvent_t tev[4] = {};
  int n_stages = 0;                                // stages of the last timed call
  PlanKey cache_key[3];                            // last plan per sink
  std::unique_ptr<PlanDev> cache[3];
  ~sncc_ctx() {
    for (auto &e : tev)
      if (e) (void)hipEventDestroy(e);
  }
  // Records the boundary before stage i (or after the last, i = n) of a call.
  void mark(int i) {
    if (timing && i < 4) (void)hipEventRecord(tev[i], stream);
  }
};

struct sncc_tmpl {
  sncc_ctx *ctx = nullptr;
  uint64_t serial = 0;  // unique per uploaded set (plan cache key)
  int T = 0;
  std::vector<int> W, H, K, seg_off;
  std::vector<std::vector<Seg>> segs;
  std::vector<std::vector<double>> c64;
  std::vector<double> q_k, r64;
  std::vector<DevTmpl> dev;  // generic (plain / refine) descriptors
  DevBuf d_geom, d_c64, d_area, d_dev, d_c32;
};

namespace {

// ------------------------------------------------------------- tile plans
struct PlanHost {
  int cfg = 0;
  TileCfg tc{2, 4, 8, 2, 1};
  int lds_bytes = 0;
  int grid = 0;
  int sink = kSinkTopk;
  int k = 0;
  std::vector<DevTmpl> tmpls;
  std::vector<PassDesc> passes;
  std::vector<Interval> ivs;
  std::vector<TileRec> recs;
  std::vector<PairDesc> pairs;
  std::vector<WorkItem> items;
  std::vector<int> order;       // item indices, queue by queue
  std::vector<int> qbeg;        // nq + 1 offsets into order
  // corner-slot tables: of the slow approximations (two-threshold search)
  // or of the fine ones (refine)
  std::vector<SlowTmpl> slow;
  std::vector<uint32_t> slot_off;
  std::vector<double> slot_w;
  int slow_lds = 0;             // bytes of the largest staged region
  // refine launch classes: pairs whose region leaves room for four
  // workgroups per CU first (refine_n_first of them, regions of at most
  // refine_lds_first bytes), then the others
  std::vector<int> refine_order;
  int refine_n_first = 0, refine_lds_first = 0;
  int run_cap = 0;              // (tile, wave) pairs of the plan
  int64_t coarse_evals = 0, n_offsets = 0;
  int64_t computed_evals = 0;  // including offsets of partial edge tiles
  int64_t n_passes = 0;        // LDS passes summed over used templates
};

int lp_class_for(int width) {
  for (int i = 0; i < kNumLpClasses; ++i)
    if (kLpClasses[i] >= width) return i;
  return -1;
}

// Rows (template-relative, zero-padded coordinates) that the corner rows of
// a segment need for a tile of bv offset rows: [y, y+bv) and [y+h, y+h+bv).
void mark_rows(std::vector<char> &cov, const Seg &g, int bv, int &count) {
  for (int r = g.y; r < g.y + bv; ++r)
    if (!cov[r]) cov[r] = 1, ++count;
  for (int r = g.y + g.h; r < g.y + g.h + bv; ++r)
    if (!cov[r]) cov[r] = 1, ++count;
}

int rows_needed(const std::vector<char> &cov, const Seg &g, int bv) {
  int add = 0;
  for (int r = g.y; r < g.y + bv; ++r) add += !cov[r];
  for (int r = std::max(g.y + g.h, g.y + bv); r < g.y + g.h + bv; ++r) add += !cov[r];
  return add;
}

// Horizontal chains of a segment list: maximal runs of segments with equal
// y and h where each starts at the column the previous one ends, cut into
// pieces of at most max_len segments.  Returns the pieces as index lists,
// in order of first segment.
std::vector<std::vector<int>> horizontal_chains(const std::vector<Seg> &segs,
                                               int max_len = kMaxChain) {
  std::map<std::tuple<int, int, int>, int> at;  // (y, h, x) -> index
  for (size_t i = 0; i < segs.size(); ++i) at[{segs[i].y, segs[i].h, segs[i].x}] = (int)i;
  std::vector<int> next(segs.size(), -1);
  std::vector<char> has_prev(segs.size(), 0);
  for (size_t i = 0; i < segs.size(); ++i) {
    auto it = at.find({segs[i].y, segs[i].h, segs[i].x + segs[i].w});
    if (it != at.end()) {
      next[i] = it->second;
      has_prev[it->second] = 1;
    }
  }
  std::vector<std::vector<int>> pieces;
  for (size_t i = 0; i < segs.size(); ++i) {
    if (has_prev[i]) continue;
    std::vector<int> piece;
    for (int k = (int)i; k >= 0; k = next[k]) {
      piece.push_back(k);
      if ((int)piece.size() == max_len) {
        pieces.push_back(piece);
        piece.clear();
      }
    }
    if (!piece.empty()) pieces.push_back(piece);
  }
  return pieces;
}

// Width of a template's column bands for tiles bu offsets wide: the whole
// template when its staged row fits 512 words, else equal bands of at most
// 512 - bu - 1 columns (multiples of 4, so that band windows start on 16-byte
// chunks).  Rows of at most 512 words leave a staged chain's rows small
// enough for two workgroups per CU where 576-word rows would allow one.
int band_width(int W, int bu) {
  const int widest = (kLpClasses[kNumLpClasses - 2] - bu - 1) & ~3;
  if (W <= widest) return W;
  const int n = (W + widest - 1) / widest;
  return ((W + n - 1) / n + 3) & ~3;
}

// Splits a template into column bands (band_width) and each band's chains
// into passes whose staged rows fit `rows_budget` LDS rows of pitch LP;
// appends passes, intervals and records.  Segments are cut at band edges
// (each piece keeps c_i; its area is its own, so the pieces' integer terms
// F - A b add up to the segment's).  Returns the largest number of rows any
// pass stages, -1 when one chain alone does not fit, -2 when a segment's area
// does not fit the 24-bit multiply.
int plan_template(const sncc_tmpl *tm, int t, const TileCfg &tc, int LP, int rows_budget,
                  PlanHost &ph, DevTmpl &d) {
  const int W = tm->W[t], H = tm->H[t], bv = tc.bv(), bu = tc.bu();
  const int span = H + bv;  // rows 0 .. H + bv - 1
  const std::vector<Seg> &all = tm->segs[t];
  for (const Seg &g : all)
    if (g.area >= (1 << 23)) return -2;
  const int bw = band_width(W, bu);
  d.pass_begin = (int)ph.passes.size();
  int max_rows = 0;
  for (int col0 = 0; col0 < W; col0 += bw) {
    const int col1 = std::min(W, col0 + bw);
    // the band's pieces, in band-relative columns, and their segments' indices
    std::vector<Seg> segs;
    std::vector<int> orig;
    for (size_t k = 0; k < all.size(); ++k) {
      const Seg &g = all[k];
      const int a = std::max(g.x, col0), b = std::min(g.x + g.w, col1);
      if (a >= b) continue;
      segs.push_back(Seg{a - col0, g.y, b - a, g.h, 0, (int64_t)(b - a) * g.h});
      orig.push_back((int)k);
    }
    const int stage_w4 = (bu + (col1 - col0) + 1 + 3) >> 2;
    const std::vector<std::vector<int>> pieces = horizontal_chains(segs);
    size_t i = 0;
    while (i < pieces.size()) {
      std::vector<char> cov(span, 0);
      int count = 0;
      size_t j = i;
      if (span <= rows_budget) {
        std::fill(cov.begin(), cov.end(), 1);
        count = span;
        j = pieces.size();
      } else {
        while (j < pieces.size()) {  // the pieces of a chain share their rows
          const Seg &g = segs[pieces[j][0]];
          const int add = rows_needed(cov, g, bv);
          if (count + add > rows_budget) break;
          mark_rows(cov, g, bv, count);
          ++j;
        }
        if (j == i) return -1;  // one chain does not fit
      }
      PassDesc ps{};
      ps.col0 = col0;
      ps.stage_w4 = stage_w4;
      ps.iv_begin = (int)ph.ivs.size();
      std::vector<int> slot(span, -1);
      int lds_row = 0;
      for (int r = 0; r < span;) {
        if (!cov[r]) {
          ++r;
          continue;
        }
        int e = r;
        while (e < span && cov[e]) ++e;
        Interval iv{r, e - r, lds_row, 0};
        ph.ivs.push_back(iv);
        for (int q = r; q < e; ++q) slot[q] = lds_row + (q - r);
        lds_row += e - r;
        r = e;
      }
      ps.iv_end = (int)ph.ivs.size();
      ps.seg_begin = (int)ph.recs.size();
      for (int L = kMaxChain; L >= 1; --L) {
        ps.n_chain[L - 1] = 0;
        for (size_t q = i; q < j; ++q) {
          const std::vector<int> &pc = pieces[q];
          if ((int)pc.size() != L) continue;
          ++ps.n_chain[L - 1];
          const Seg &g0 = segs[pc[0]];
          const int top = slot[g0.y] * LP, bot = slot[g0.y + g0.h] * LP;
          ph.recs.push_back(TileRec{top + g0.x, bot + g0.x, 0, 0.f});  // left boundary
          for (int k : pc) {
            const Seg &g = segs[k];
            ph.recs.push_back(TileRec{top + g.x + g.w, bot + g.x + g.w, (int)g.area,
                                      (float)tm->c64[t][orig[k]]});
          }
        }
      }
      ps.seg_end = (int)ph.recs.size();
      ph.passes.push_back(ps);
      max_rows = std::max(max_rows, lds_row);
      i = j;
    }
  }
  d.pass_end = (int)ph.passes.size();
  return max_rows;
}

// Direct form of a template for the tile kernel (no LDS staging): one pass
// whose records are pairs of TileRec slots holding a DirectRec (byte offsets
// of the corners in a table of pitch P, 4 w, A_i, c_i).
void plan_direct(const sncc_tmpl *tm, int t, int P, PlanHost &ph, DevTmpl &d) {
  if (ph.recs.size() & 1) ph.recs.push_back(TileRec{0, 0, 0, 0.f});
  d.lp_class = kLpDirect;
  d.pass_begin = (int)ph.passes.size();
  PassDesc ps{};
  ps.iv_begin = ps.iv_end = (int)ph.ivs.size();
  ps.seg_begin = (int)ph.recs.size();
  const std::vector<Seg> &segs = tm->segs[t];
  auto push = [&](int top, int bot, int area, float c) {
    DirectRec dr;
    dr.top = top;
    dr.bot = bot;
    dr.area = area;
    dr.c = c;
    dr.pad[0] = dr.pad[1] = dr.pad[2] = dr.pad[3] = 0;
    TileRec two[2];
    static_assert(sizeof(two) == sizeof(DirectRec), "a direct record spans two slots");
    memcpy(two, &dr, sizeof dr);
    ph.recs.push_back(two[0]);
    ph.recs.push_back(two[1]);
  };
  // one record per boundary column of each horizontal chain: the column's
  // entries in the chain's top and bottom rows, and A_i, c_i of the segment
  // ending there (0 at the chain's first column)
  int nrec = 0;
  for (const std::vector<int> &pc : horizontal_chains(segs, 1 << 30)) {
    const Seg &g0 = segs[pc[0]];
    const int top = g0.y * P, bot = (g0.y + g0.h) * P;
    push((top + g0.x) * 4, (bot + g0.x) * 4, 0, 0.f);
    ++nrec;
    for (int q : pc) {
      const int x = segs[q].x + segs[q].w;
      push((top + x) * 4, (bot + x) * 4, (int)segs[q].area, (float)tm->c64[t][q]);
      ++nrec;
    }
  }
  // padded to whole groups of four with records that add exactly zero
  for (; nrec % 4 != 0; ++nrec) push(0, 0, 0, 0.f);
  ps.seg_end = (int)ph.recs.size();
  ph.passes.push_back(ps);
  d.pass_end = (int)ph.passes.size();
}

// Split of a pair's tile columns between two launches: when the last
// column of main_bu-wide tiles holds at most main_bu / 2 offsets, the main
// launch (kSplitMain) leaves it out and a launch of half-width tiles
// (kSplitEdge) scores it alone.
constexpr int kSplitNone = 0, kSplitMain = 1, kSplitEdge = 2;

bool has_edge(int nu, int main_bu) {
  const int r = nu % main_bu;
  return r > 0 && r <= main_bu / 2;
}

// Tile configuration of the one-call entry points (no tuner): 128 x 32
// tiles in eight-wave workgroups, two per CU (on single frames it beat the
// 128 x 16 four-wave shape the tuner picks for the batches, whose smaller LDS
// budget sends large templates to the direct form), or 64 x 16 tiles when the
// pairs hold fewer 128 x 32 tiles than half the CUs (a small frame would
// leave most CUs idle).
int one_call_cfg(const sncc_tmpl *tm, int M, int N, int n_pairs, const int32_t *pairs,
                 int num_cu) {
  constexpr int kWide = 0, kNarrow = 6;
  const TileCfg tc = tile_cfg(kWide);
  long long tiles = 0;
  for (int p = 0; p < n_pairs; ++p) {
    const int t = pairs[2 * p + 1];
    const long long nu = M - tm->W[t] + 1, nv = N - tm->H[t] + 1;
    tiles += ((nu + tc.bu() - 1) / tc.bu()) * ((nv + tc.bv() - 1) / tc.bv());
  }
  return 2 * tiles >= (long long)std::max(1, num_cu) ? kWide : kNarrow;
}

int build_plan(const sncc_tmpl *tm, int cfg, int M, int N, int P, int n_pairs,
               const int32_t *pairs, int k, int sink, int num_cu, PlanHost &ph,
               const double *thr = nullptr, int split = kSplitNone, int main_bu = 0) {
  if (cfg < 0 || cfg >= tile_cfg_count()) SNCC_FAIL(SNCC_EINVAL, "bad tile config %d", cfg);
  ph = PlanHost();
  ph.cfg = cfg;
  ph.tc = tile_cfg(cfg);
  ph.sink = sink;
  ph.k = k;
  const TileCfg tc = ph.tc;
  const int bu = tc.bu(), bv = tc.bv();
  std::vector<char> used(tm->T, 0);
  for (int p = 0; p < n_pairs; ++p) used[pairs[2 * p + 1]] = 1;

  // LDS budget: tc.wgs workgroups per CU when every template allows it,
  // otherwise one workgroup per CU
  const int topk_bytes = sink == kSinkTopk ? tc.nw * std::max(k, 1) * 8 : 0;
  // the kernel keeps one FP32 scale per offset in LDS ahead of the staged rows
  const int scale_bytes = 64 * tc.nw * tc.ru * tc.rv * 4;
  int budget = tile_max_lds() / tc.wgs - 512 - scale_bytes;
  for (int pass = 0; pass < 2; ++pass) {
    ph.tmpls.assign(tm->T, DevTmpl{});
    ph.passes.clear();
    ph.ivs.clear();
    ph.recs.clear();
    ph.n_passes = 0;
    bool ok = true;
    int max_bytes = topk_bytes;
    for (int t = 0; t < tm->T; ++t) {
      DevTmpl d = tm->dev[t];
      d.pass_begin = d.pass_end = 0;
      d.thr = thr ? (float)thr[t] : 0.f;
      if (used[t]) {
        // LDS staging (in column bands when one LDS row cannot hold the
        // template's width) when every segment fits the packed record and
        // each chain's rows fit the budget; the direct form otherwise
        const int cls = lp_class_for(bu + band_width(tm->W[t], bu) + 1);
        const size_t mark_recs = ph.recs.size(), mark_ivs = ph.ivs.size();
        const size_t mark_passes = ph.passes.size();
        int rows = -2;
        if (cls >= 0) {
          const int LP = kLpClasses[cls];
          d.lp_class = cls;
          rows = plan_template(tm, t, tc, LP, budget / (LP * 4), ph, d);
          if (rows >= 0) max_bytes = std::max(max_bytes, scale_bytes + rows * LP * 4);
        }
        if (rows == -1 && pass == 0) {  // rows do not fit: retry with one workgroup per CU
          ok = false;
          break;
        }
        if (rows < 0) {
          ph.recs.resize(mark_recs);
          ph.ivs.resize(mark_ivs);
          ph.passes.resize(mark_passes);
          plan_direct(tm, t, P, ph, d);
          max_bytes = std::max(max_bytes, scale_bytes);
        }
      }
      ph.tmpls[t] = d;
      ph.n_passes += d.pass_end - d.pass_begin;
    }
    if (ok) {
      ph.lds_bytes = (max_bytes + 255) & ~255;
      break;
    }
    budget = tile_max_lds() - 1024 - scale_bytes;
  }

  // pairs and work items
  const int occ = std::max(1, tile_occupancy(cfg, sink, ph.lds_bytes));
  const int slots = std::max(1, num_cu) * occ;
  std::vector<double> tile_cost(n_pairs);
  double total = 0;
  ph.pairs.resize(n_pairs);
  for (int p = 0; p < n_pairs; ++p) {
    const int t = pairs[2 * p + 1];
    PairDesc &pd = ph.pairs[p];
    pd.frame = pairs[2 * p];
    pd.tmpl = t;
    pd.nu = M - tm->W[t] + 1;
    pd.nv = N - tm->H[t] + 1;
    pd.ntu = (pd.nu + bu - 1) / bu;
    pd.ntv = (pd.nv + bv - 1) / bv;
    pd.u_base = 0;
    if (split == kSplitMain && has_edge(pd.nu, bu)) pd.ntu = pd.nu / bu;
    if (split == kSplitEdge) {
      pd.u_base = pd.nu / main_bu * main_bu;
      pd.ntu = has_edge(pd.nu, main_bu) ? 1 : 0;
    }
    const double staged = (double)(bu + tm->W[t] + 1) * (double)(bv + tm->H[t] + 1);
    tile_cost[p] = (double)bu * bv * (tm->K[t] + 8.0) + 0.5 * staged;
    total += tile_cost[p] * pd.ntu * pd.ntv;
    if (split != kSplitEdge) {  // the split's evaluations are counted once, by the main plan
      ph.coarse_evals += (int64_t)pd.nu * pd.nv * tm->K[t];
      ph.n_offsets += (int64_t)pd.nu * pd.nv;
    }
    ph.computed_evals += (int64_t)pd.ntu * bu * pd.ntv * bv * tm->K[t];
  }
  const double target = std::max(total, 1.0) / (slots * 6.0);
  std::vector<double> item_cost;
  ph.order.clear();
  if (tc.frame_major) {
    // Items are bands of offset rows of one pair (split further only when a
    // band alone exceeds the target cost).  A group is one band of one frame
    // over all of that frame's templates.  Queues, one per XCD, take whole
    // frames (frame mod kMaxQueues) when there are enough frames, else groups
    // round-robin; each queue runs its groups in frame and band order, so the
    // workgroups of one XCD read the same frame rows from their shared L2,
    // and a pair's later bands start with the floor its earlier bands
    // published.  Within a group the costliest items go first.  A band is
    // kRowsInFlight / (workgroups per CU) rows high: an XCD's workgroups then
    // work on about that many consecutive offset rows of a frame at once
    // (plus the template height), whose two tables fit its L2.
    constexpr int kRowsInFlight = 64;
    const int band_tiles = std::max(1, kRowsInFlight / std::max(1, tc.wgs) / bv);
    std::vector<int64_t> group_of;
    for (int p = 0; p < n_pairs; ++p) {
      PairDesc &pd = ph.pairs[p];
      pd.item_begin = (int)ph.items.size();
      for (int b = 0; pd.ntu > 0 && b * band_tiles < pd.ntv; ++b) {
        const int t0 = b * band_tiles * pd.ntu;
        const int t1 = std::min(pd.ntv, (b + 1) * band_tiles) * pd.ntu;
        const int ntiles = t1 - t0;
        int per = (int)std::max(1.0, std::floor(target / tile_cost[p]));
        per = std::min(per, ntiles);
        const int nitems = (ntiles + per - 1) / per;
        per = (ntiles + nitems - 1) / nitems;
        for (int a = t0; a < t1; a += per) {
          WorkItem it{p, a, std::min(t1, a + per), 0};
          ph.items.push_back(it);
          item_cost.push_back(tile_cost[p] * (it.tile_end - it.tile_begin));
          group_of.push_back((int64_t)pd.frame << 32 | b);
        }
      }
      pd.item_end = (int)ph.items.size();
    }
    std::vector<int> idx(ph.items.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
      return group_of[a] != group_of[b] ? group_of[a] < group_of[b] : item_cost[a] > item_cost[b];
    });
    int n_groups = 0, n_frames = 0;
    std::vector<int> gid(idx.size()), fid(idx.size());
    for (size_t i = 0; i < idx.size(); ++i) {
      if (i > 0 && group_of[idx[i]] != group_of[idx[i - 1]]) ++n_groups;
      if (i > 0 && group_of[idx[i]] >> 32 != group_of[idx[i - 1]] >> 32) ++n_frames;
      gid[i] = n_groups;
      fid[i] = n_frames;
    }
    if (!idx.empty()) ++n_groups, ++n_frames;
    const int nq = std::max(1, std::min(kMaxQueues, n_groups));
    const bool by_frame = n_frames >= nq;
    ph.qbeg.assign(1, 0);
    for (int q = 0; q < nq; ++q) {
      for (size_t i = 0; i < idx.size(); ++i)
        if ((by_frame ? fid[i] : gid[i]) % nq == q) ph.order.push_back(idx[i]);
      ph.qbeg.push_back((int)ph.order.size());
    }
  } else {
    for (int p = 0; p < n_pairs; ++p) {
      PairDesc &pd = ph.pairs[p];
      const int ntiles = pd.ntu * pd.ntv;
      pd.item_begin = pd.item_end = (int)ph.items.size();
      if (ntiles == 0) continue;
      int per = (int)std::max(1.0, std::floor(target / tile_cost[p]));
      per = std::min(per, ntiles);
      const int nitems = (ntiles + per - 1) / per;
      per = (ntiles + nitems - 1) / nitems;  // even out
      for (int a = 0; a < ntiles; a += per) {
        WorkItem it{p, a, std::min(ntiles, a + per), 0};
        ph.items.push_back(it);
        item_cost.push_back(tile_cost[p] * (it.tile_end - it.tile_begin));
      }
      pd.item_end = (int)ph.items.size();
    }
    // one queue, costliest items first
    ph.order.resize(ph.items.size());
    for (size_t i = 0; i < ph.order.size(); ++i) ph.order[i] = (int)i;
    std::stable_sort(ph.order.begin(), ph.order.end(),
                     [&](int a, int b) { return item_cost[a] > item_cost[b]; });
    ph.qbeg = {0, (int)ph.order.size()};
  }
  ph.grid = (int)std::min<size_t>(ph.items.size(), (size_t)slots);
  if (ph.grid < 1) ph.grid = 1;
  return SNCC_OK;
}

// Plan of a one-call entry point: one_call_cfg's shape; when the wide
// 128 x 32 tiles' rows do not fit two workgroups per CU (tall templates: the
// plan fell back to one), the 128 x 16 eight-wave shape instead if its rows,
// half as many per segment, keep two (3840 x 2160 with a 256 x 256
// template: 8.5 -> 7.3 ms).
int build_one_call_plan(const sncc_tmpl *tm, int M, int N, int P, int n_pairs,
                        const int32_t *pairs, int k, int sink, int num_cu, PlanHost &ph) {
  constexpr int kWide = 0, kTall = 3;
  static_assert(kCfgs[kTall].entry == 3 && kTileShapes[3][0] == 2 && kTileShapes[3][1] == 2 &&
                    kTileShapes[3][2] == 8 && kCfgs[kTall].wgs == 2,
                "kTall: 128 x 16 tiles, eight waves, two workgroups per CU");
  const int cfg = one_call_cfg(tm, M, N, n_pairs, pairs, num_cu);
  CHK(build_plan(tm, cfg, M, N, P, n_pairs, pairs, k, sink, num_cu, ph));
  if (cfg == kWide && ph.lds_bytes > tile_max_lds() / 2) {
    PlanHost alt;
    if (build_plan(tm, kTall, M, N, P, n_pairs, pairs, k, sink, num_cu, alt) == SNCC_OK &&
        alt.lds_bytes <= tile_max_lds() / 2)
      ph = std::move(alt);
    g_err.clear();
  }
  return SNCC_OK;
}

// Boundary-slot tables (see SlowTmpl) of a template set for runs of
// span_u x span_v offsets: a template whose region, (span_v + H) rows of
// span_u + W + 1 words, exceeds max_words keeps tbl = -1 (global form).
void plan_slots(const sncc_tmpl *tm, int span_u, int span_v, int max_words, PlanHost &ph,
                int narrow_u = 0, int narrow_v = 0) {
  ph.slow.assign(tm->T, SlowTmpl{-1, 0, 0, 0});
  ph.slot_off.clear();
  ph.slot_w.clear();
  ph.slow_lds = 0;
  for (int t = 0; t < tm->T; ++t) {
    const int W = tm->W[t], H = tm->H[t];
    // the region of (span_u, span_v) offsets, or of the narrower spans when
    // that one exceeds the budget
    int pitch = span_u + W + 1, rows = span_v + H;
    if ((long long)pitch * rows > max_words && narrow_u > 0) {
      pitch = narrow_u + W + 1;
      rows = narrow_v + H;
    }
    if ((long long)pitch * rows > max_words) continue;
    const std::vector<Seg> &segs = tm->segs[t];
    // corners of the segments with their summed weights (W_p: +c at the
    // top-left and bottom-right corner of a segment, -c at the other two),
    // zero sums dropped, in raster order
    std::map<std::pair<int, int>, double> corner;
    const std::vector<double> &c = tm->c64[t];
    for (size_t i = 0; i < segs.size(); ++i) {
      const Seg &g = segs[i];
      corner[{g.y, g.x}] += c[i];
      corner[{g.y + g.h, g.x + g.w}] += c[i];
      corner[{g.y, g.x + g.w}] -= c[i];
      corner[{g.y + g.h, g.x}] -= c[i];
    }
    SlowTmpl st;
    st.tbl = (int)ph.slot_off.size();
    st.pitch = pitch;
    st.rows = rows;
    std::vector<std::pair<uint32_t, double>> raster;
    for (const auto &e : corner)
      if (e.second != 0.0)
        raster.emplace_back((uint32_t)((e.first.first * pitch + e.first.second) * 4), e.second);
    // Slot order for the LDS banks (32 banks of 4 bytes per half-wave; a
    // window's base shifts every lane's bank alike): groups of 32 slots, each
    // taking first, among the next kWindow slots in raster order, slots of
    // the banks with the most slots still to place, at most one per bank,
    // then the least conflicting ones.  The sum does not depend on the order.
    constexpr size_t kWindow = 4096;
    auto bank = [&](size_t i) { return (int)((raster[i].first >> 2) & 31); };
    int rem[32] = {0};
    for (size_t i = 0; i < raster.size(); ++i) ++rem[bank(i)];
    std::vector<size_t> pool(raster.size());
    for (size_t i = 0; i < pool.size(); ++i) pool[i] = i;
    std::vector<size_t> cand, grp;
    std::vector<char> in_grp(raster.size(), 0);
    while (!pool.empty()) {
      cand.assign(pool.begin(), pool.begin() + std::min(pool.size(), kWindow));
      std::stable_sort(cand.begin(), cand.end(),
                       [&](size_t x, size_t y) { return rem[bank(x)] > rem[bank(y)]; });
      int used[32] = {0};
      grp.clear();
      auto take = [&](size_t i) {
        grp.push_back(i);
        in_grp[i] = 1;
        ++used[bank(i)];
      };
      for (size_t i : cand) {
        if (grp.size() == 32) break;
        if (!used[bank(i)]) take(i);
      }
      while (grp.size() < 32) {
        size_t best = raster.size();
        int best_cost = 1 << 30;
        for (size_t i : cand) {
          if (in_grp[i]) continue;
          if (used[bank(i)] < best_cost) best = i, best_cost = used[bank(i)];
        }
        if (best == raster.size()) break;
        take(best);
      }
      for (size_t i : grp) {
        --rem[bank(i)];
        ph.slot_off.push_back(raster[i].first);
        ph.slot_w.push_back(raster[i].second);
      }
      size_t k = 0;
      for (size_t i : pool)
        if (!in_grp[i]) pool[k++] = i;
      pool.resize(k);
    }
    while (ph.slot_off.size() % 64 != 0) {
      ph.slot_off.push_back(0);
      ph.slot_w.push_back(0.0);
    }
    st.n_iter = ((int)ph.slot_off.size() - st.tbl) / 64;
    ph.slow[t] = st;
    ph.slow_lds = std::max(ph.slow_lds, pitch * rows * 4);
  }
}

// Refine launch classes over the plan's pairs (after plan_slots of the fine
// approximations): the offset list of n_cand (2 radius + 1)^2 entries and a
// region that fits refine_region_budget(np, 4) let four eight-wave
// workgroups share a CU instead of the three that the largest region allows.
void plan_refine_order(PlanHost &ph, int n_cand, int radius) {
  ph.refine_order.clear();
  ph.refine_n_first = ph.refine_lds_first = 0;
  const int total = n_cand * (2 * radius + 1) * (2 * radius + 1);
  int np = 1;
  while (np < total) np <<= 1;
  const int budget = refine_region_budget(np, 4);
  std::vector<int> rest;
  for (int p = 0; p < (int)ph.pairs.size(); ++p) {
    const SlowTmpl &st = ph.slow[ph.pairs[p].tmpl];
    const int region = st.tbl >= 0 ? st.pitch * st.rows * 4 : 0;
    if (region <= budget) {
      ph.refine_order.push_back(p);
      ph.refine_lds_first = std::max(ph.refine_lds_first, region);
    } else {
      rest.push_back(p);
    }
  }
  ph.refine_n_first = (int)ph.refine_order.size();
  ph.refine_order.insert(ph.refine_order.end(), rest.begin(), rest.end());
}

// Slot tables of the slow approximations for the slow pass, whose runs are
// one wave's part of kRunCols columns of a tile of shape `tc`, and the run
// capacity.
void plan_slow(const sncc_tmpl *slow, const TileCfg &tc, PlanHost &ph) {
  plan_slots(slow, kRunCols, tc.rv, kSlowRegionWords, ph);
  long long tiles = 0;
  for (const WorkItem &it : ph.items) tiles += it.tile_end - it.tile_begin;
  ph.run_cap = (int)std::min<long long>(tiles * tc.nw * tc.ru * (64 / kRunCols), 1 << 30);
}

}  // namespace

// Device copy of a plan plus its completion event.
struct PlanDev {
  PlanHost h;
  DevBuf d_tmpls, d_passes, d_ivs, d_recs, d_pairs, d_items, d_order, d_qbeg, d_queue,
      d_partial, d_thr, d_slow, d_slot_off, d_slot_w, d_runs, d_refine_order;
  hipEvent_t done = nullptr;
  ~PlanDev() {
    if (done) (void)hipEventDestroy(done);
  }
  int upload(hipStream_t st) {
    CHK(d_tmpls.upload(h.tmpls, st));
    CHK(d_passes.upload(h.passes, st));
    CHK(d_ivs.upload(h.ivs, st));
    CHK(d_recs.upload(h.recs, st));
    CHK(d_pairs.upload(h.pairs, st));
    CHK(d_items.upload(h.items, st));
    CHK(d_order.upload(h.order, st));
    CHK(d_qbeg.upload(h.qbeg, st));
    CHK(d_queue.reserve(zero_ints() * sizeof(int)));
    if (h.sink == kSinkTopk)
      CHK(d_partial.reserve(std::max<size_t>(16, h.items.size() * h.k * 8)));
    if (!h.slow.empty()) {
      CHK(d_slow.upload(h.slow, st));
      CHK(d_slot_off.upload(h.slot_off, st));
      CHK(d_slot_w.upload(h.slot_w, st));
    }
    if (!h.refine_order.empty()) CHK(d_refine_order.upload(h.refine_order, st));
    if (h.sink == kSinkCompact)
      CHK(d_runs.reserve(std::max<size_t>(16, (size_t)h.run_cap * sizeof(RunDesc))));
    return SNCC_OK;
  }
  SlotTables slots() {
    const bool classes = !h.refine_order.empty();
    return SlotTables{d_slow.as<SlowTmpl>(),
                      d_slot_off.as<uint32_t>(),
                      d_slot_w.as<double>(),
                      h.slow_lds,
                      classes ? d_refine_order.as<int>() : nullptr,
                      h.refine_n_first,
                      h.refine_lds_first};
  }
  // work counters, then one floor key per pair (top-k sink) or the run and
  // slow-pass counters (compacting sink), zeroed per launch
  int zero_ints() const {
    return kQueueInts + (h.sink == kSinkTopk ? 2 * (int)h.pairs.size()
                                             : h.sink == kSinkCompact ? 16 : 0);
  }
  TileArgs args(const uint32_t *s, const uint32_t *s2, long long fs, int P, int M, int N) {
    TileArgs a;
    a.s = s;
    a.s2 = s2;
    a.frame_stride = fs;
    a.sat_pitch = P;
    a.M = M;
    a.N = N;
    a.tmpls = d_tmpls.as<DevTmpl>();
    a.passes = d_passes.as<PassDesc>();
    a.ivs = d_ivs.as<Interval>();
    a.recs = d_recs.as<TileRec>();
    a.pairs = d_pairs.as<PairDesc>();
    a.items = d_items.as<WorkItem>();
    a.order = d_order.as<int>();
    a.qbeg = d_qbeg.as<int>();
    // one workgroup per item: no queues (the kernel takes order[blockIdx])
    a.nq = h.grid == (int)h.items.size() && !queues_forced() ? 0 : (int)h.qbeg.size() - 1;
    a.n_items = (int)h.items.size();
    a.queue = d_queue.as<int>();
    a.k = h.k;
    a.partial = d_partial.as<unsigned long long>();
    a.pair_floor =
        h.sink == kSinkTopk ? reinterpret_cast<unsigned long long *>(a.queue + kQueueInts)
                            : nullptr;
    a.co = CompactOut{nullptr, 0, nullptr, nullptr, 0, nullptr};
    if (h.sink == kSinkCompact) {
      a.co.runs = d_runs.as<RunDesc>();
      a.co.run_cap = h.run_cap;
      a.co.run_count = a.queue + kQueueInts;
    }
    a.n_zero = zero_ints();
    a.rho = nullptr;
    a.rho_pitch = 0;
    a.degen = nullptr;
    return a;
  }
};

namespace {

// Frees retired plans whose work has completed (all of them when `wait`).
void reap(sncc_ctx *ctx, bool wait) {
  auto &v = ctx->retired;
  for (size_t i = 0; i < v.size();) {
    bool finished = true;
    if (v[i]->done) {
      if (wait)
        (void)hipEventSynchronize(v[i]->done);
      else
        finished = hipEventQuery(v[i]->done) == hipSuccess;
    }
    if (finished) {
      v.erase(v.begin() + i);
    } else {
      ++i;
    }
  }
}

int retire(sncc_ctx *ctx, std::unique_ptr<PlanDev> pd) {
  HIPCHK(hipEventCreateWithFlags(&pd->done, hipEventDisableTiming));
  HIPCHK(hipEventRecord(pd->done, ctx->stream));
  ctx->retired.push_back(std::move(pd));
  if (ctx->retired.size() > 32) reap(ctx, false);
  return SNCC_OK;
}

// The context's plan for `key` (key.sink's slot), built and uploaded by
// `make` on a miss; the plan it replaces is retired, since work queued with
// it may still be running.  Calls on one context are ordered by its stream,
// so reusing a plan while earlier work still reads it is safe.
template <class Make>
int cached_plan(sncc_ctx *ctx, PlanKey key, Make make, PlanDev **out) {
  const int slot = key.sink;
  if (ctx->cache[slot] && ctx->cache_key[slot] == key) {
    *out = ctx->cache[slot].get();
    return SNCC_OK;
  }
  if (ctx->cache[slot]) CHK(retire(ctx, std::move(ctx->cache[slot])));
  ctx->cache_key[slot] = PlanKey{};
  std::unique_ptr<PlanDev> pd(new PlanDev());
  CHK(make(*pd));
  CHK(pd->upload(ctx->stream));
  ctx->cache[slot] = std::move(pd);
  ctx->cache_key[slot] = std::move(key);
  *out = ctx->cache[slot].get();
  return SNCC_OK;
}

int check_ctx(sncc_ctx *ctx) {
  if (!ctx) SNCC_FAIL(SNCC_EINVAL, "NULL context");
  HIPCHK(hipSetDevice(ctx->device));
  return SNCC_OK;
}

int check_sats(const uint32_t *s, const uint32_t *s2, int M, int N, int P) {
  if (!s || !s2) SNCC_FAIL(SNCC_EINVAL, "NULL sum table");
  if (!aligned16(s) || !aligned16(s2)) SNCC_FAIL(SNCC_EINVAL, "sum tables must be 16-byte aligned");
  if (M < 1 || N < 1) SNCC_FAIL(SNCC_EINVAL, "bad image size %dx%d", M, N);
  int need = 0;
  sncc_sat_pitch(M, &need);
  if (P < need || P % 64 != 0)
    SNCC_FAIL(SNCC_EINVAL, "sat_pitch %d: need a multiple of 64 >= %d", P, need);
  // the scoring kernels address one frame's table with 32-bit byte offsets
  if ((long long)(N + 1) * P * 4 > (long long)SNCC_MAX_TABLE_BYTES)
    SNCC_FAIL(SNCC_EINVAL, "sum table of %lld bytes per frame exceeds %lld",
              (long long)(N + 1) * P * 4, (long long)SNCC_MAX_TABLE_BYTES);
  return SNCC_OK;
}

int check_pairs(const sncc_tmpl *tm, int B, int M, int N, int n_pairs, const int32_t *pairs) {
  if (!tm) SNCC_FAIL(SNCC_EINVAL, "NULL template set");
  if (n_pairs < 1 || !pairs) SNCC_FAIL(SNCC_EINVAL, "no pairs");
  for (int p = 0; p < n_pairs; ++p) {
    const int f = pairs[2 * p], t = pairs[2 * p + 1];
    if (f < 0 || f >= B || t < 0 || t >= tm->T)
      SNCC_FAIL(SNCC_EINVAL, "pair %d = (%d, %d) out of range", p, f, t);
    if (tm->W[t] > M || tm->H[t] > N)
      SNCC_FAIL(SNCC_EINVAL, "template %d (%dx%d) larger than image %dx%d", t, tm->W[t],
                tm->H[t], M, N);
  }
  return SNCC_OK;
}

// Checks T segment lists (each must partition its W x H template) and fills
// the host side of a template set: sizes, segment lists and the constants of
// Section 5, steps 3-4 (Eq. (7), c_i, q_k), plus the generic per-segment
// arrays the device copies are made from.  No device work.
int fill_templates(sncc_tmpl *tm, int T, const sncc_segment *const *segs, const int *K,
                   const int *W, const int *H, std::vector<int4> &geom,
                   std::vector<double> &c64all, std::vector<int> &areas) {
  for (int t = 0; t < T; ++t) {
    const int w = W[t], h = H[t], k = K[t];
    if (w < 1 || h < 1 || k < 1 || !segs[t]) SNCC_FAIL(SNCC_EINVAL, "template %d: bad size or list", t);
    const long long n = (long long)w * h;
    if (n > SNCC_MAX_TEMPLATE_AREA || w > kMaxSqBoxArea)
      SNCC_FAIL(SNCC_ERANGE, "template %d: %dx%d outside the exact range (area <= %d, width <= %d)",
                t, w, h, SNCC_MAX_TEMPLATE_AREA, kMaxSqBoxArea);
    std::vector<char> cover((size_t)n, 0);
    std::vector<Seg> list;
    int64_t total = 0;
    for (int i = 0; i < k; ++i) {
      const sncc_segment &g = segs[t][i];
      if (g.w < 1 || g.h < 1 || g.x < 0 || g.y < 0 || g.x + g.w > w || g.y + g.h > h ||
          g.area != g.w * g.h || g.sum < 0 || g.sum > 255LL * g.area)
        SNCC_FAIL(SNCC_EINVAL, "template %d segment %d invalid", t, i);
      for (int y = g.y; y < g.y + g.h; ++y)
        for (int x = g.x; x < g.x + g.w; ++x) {
          if (cover[(size_t)y * w + x]) SNCC_FAIL(SNCC_EINVAL, "template %d: segments overlap", t);
          cover[(size_t)y * w + x] = 1;
        }
      list.push_back(Seg{g.x, g.y, g.w, g.h, g.sum, g.area});
      total += g.sum;
    }
    for (char c : cover)
      if (!c) SNCC_FAIL(SNCC_EINVAL, "template %d: segments do not cover the template", t);
    bool uniform = true;
    for (const Seg &g : list)
      if ((__int128)g.sum * n != (__int128)total * g.area) uniform = false;
    if (uniform) SNCC_FAIL(SNCC_EDEGENERATE, "template %d: uniform approximation (q_k = 0)", t);
    // Eq. (7) and the zero-mean values of step 3; q_k of step 4 (area-weighted)
    double kbar = 0;
    for (const Seg &g : list) kbar += (double)g.area * ((double)g.sum / (double)g.area);
    kbar /= (double)n;
    std::vector<double> c(k);
    double qk = 0, r = 0;
    for (int i = 0; i < k; ++i) {
      c[i] = (double)list[i].sum / (double)list[i].area - kbar;
      qk += (double)list[i].area * c[i] * c[i];
      r += (double)list[i].area * c[i];
    }
    DevTmpl d{};
    d.W = w;
    d.H = h;
    d.K = k;
    d.n = (int)n;
    d.q_k = qk;
    d.r64 = r;
    d.sq_rows = n <= kMaxSqBoxArea ? h : kMaxSqBoxArea / w;
    d.seg_off = (int)geom.size();
    tm->W.push_back(w);
    tm->H.push_back(h);
    tm->K.push_back(k);
    tm->seg_off.push_back(d.seg_off);
    tm->q_k.push_back(qk);
    tm->r64.push_back(r);
    for (int i = 0; i < k; ++i) {
      geom.push_back(make_int4(list[i].x, list[i].y, list[i].w, list[i].h));
      c64all.push_back(c[i]);
      areas.push_back((int)list[i].area);
    }
    tm->segs.push_back(std::move(list));
    tm->c64.push_back(std::move(c));
    tm->dev.push_back(d);
  }
  return SNCC_OK;
}

}  // namespace

// ================================================================ C-ABI
extern "C" {

const char *sncc_status_string(int status) {
  switch (status) {
    case SNCC_OK: return "ok";
    case SNCC_EINVAL: return "invalid argument";
    case SNCC_ENOMEM: return "out of memory";
    case SNCC_ENOSPC: return "output capacity too small";
    case SNCC_ERANGE: return "size outside the exact range";
    case SNCC_EDEGENERATE: return "uniform template approximation";
    case SNCC_EDEVICE: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char *sncc_last_error(void) { return g_err.c_str(); }

int sncc_version(void) { return 10000; }

int sncc_segment_template(const uint8_t *t, int W, int H, int t_stride, double sigma_max,
                          int K_max, sncc_segment *out, int cap, int *K_out,
                          double *sigma_used, double *rho_max) {
  g_err.clear();
  if (!t || !K_out) SNCC_FAIL(SNCC_EINVAL, "NULL argument");
  if (W < 1 || H < 1 || t_stride < W) SNCC_FAIL(SNCC_EINVAL, "bad template size %dx%d stride %d", W, H, t_stride);
  if (K_max < 1) SNCC_FAIL(SNCC_EINVAL, "K_max must be >= 1");
  if (std::isnan(sigma_max)) SNCC_FAIL(SNCC_EINVAL, "sigma_max is NaN");
  std::vector<Seg> segs;
  int kbm = 0;
  double su = 0, rm = 0;
  const int st = segment_template(t, W, H, t_stride, sigma_max, K_max, segs, &kbm, &su, &rm);
  *K_out = (int)segs.size();
  if (sigma_used) *sigma_used = su;
  if (st != SNCC_OK) SNCC_FAIL(st, "uniform template approximation (all segment means equal)");
  if (rho_max) *rho_max = rm;
  if (cap < (int)segs.size() || (!out && !segs.empty()))
    SNCC_FAIL(SNCC_ENOSPC, "need %zu segments, capacity %d", segs.size(), cap);
  for (size_t i = 0; i < segs.size(); ++i) {
    out[i].x = segs[i].x;
    out[i].y = segs[i].y;
    out[i].w = segs[i].w;
    out[i].h = segs[i].h;
    out[i].sum = segs[i].sum;
    out[i].area = (int32_t)segs[i].area;
    out[i].reserved = 0;
  }
  return SNCC_OK;
}

int sncc_segment_templates(int T, const uint8_t *const *t, const int *W, const int *H,
                           const int *t_stride, const double *sigma_max, int K_max,
                           int n_threads, sncc_segment *out, int64_t out_cap, int64_t *seg_off,
                           double *sigma_used, double *rho_max, int *status) {
  g_err.clear();
  if (T < 1 || !t || !W || !H || !t_stride || !sigma_max || !seg_off)
    SNCC_FAIL(SNCC_EINVAL, "NULL argument or T < 1");
  if (K_max < 1) SNCC_FAIL(SNCC_EINVAL, "K_max must be >= 1");
  for (int i = 0; i < T; ++i) {
    if (!t[i] || W[i] < 1 || H[i] < 1 || t_stride[i] < W[i])
      SNCC_FAIL(SNCC_EINVAL, "template %d: bad pointer, size %dx%d or stride %d", i,
                W[i], H[i], t_stride[i]);
    if (std::isnan(sigma_max[i])) SNCC_FAIL(SNCC_EINVAL, "template %d: sigma_max is NaN", i);
  }
  std::vector<std::vector<Seg>> lists(T);
  std::vector<int> st(T, SNCC_OK);
  std::vector<double> su(T, 0.0), rm(T, 0.0);
  std::atomic<int> next{0};
  auto worker = [&]() {
    for (int i = next.fetch_add(1); i < T; i = next.fetch_add(1)) {
      int kbm = 0;
      st[i] = segment_template(t[i], W[i], H[i], t_stride[i], sigma_max[i], K_max, lists[i],
                               &kbm, &su[i], &rm[i]);
    }
  };
  int nt = n_threads > 0 ? n_threads : (int)std::thread::hardware_concurrency();
  nt = std::max(1, std::min(nt, T));
  if (nt == 1) {
    worker();
  } else {
    std::vector<std::thread> pool;
    try {
      for (int k = 1; k < nt; ++k) pool.emplace_back(worker);
    } catch (...) {
      // fewer threads than asked for: the ones running (and this one) finish the work
    }
    worker();
    for (auto &th : pool) th.join();
  }
  int64_t total = 0;
  int first_bad = SNCC_OK, bad_index = -1;
  for (int i = 0; i < T; ++i) {
    seg_off[i] = total;
    total += (int64_t)lists[i].size();
    if (sigma_used) sigma_used[i] = su[i];
    if (rho_max) rho_max[i] = st[i] == SNCC_OK ? rm[i] : std::nan("");
    if (status) status[i] = st[i];
    if (st[i] != SNCC_OK && first_bad == SNCC_OK) first_bad = st[i], bad_index = i;
  }
  seg_off[T] = total;
  if (total > out_cap || (!out && total > 0))
    SNCC_FAIL(SNCC_ENOSPC, "need %lld segments, capacity %lld", (long long)total,
              (long long)out_cap);
  for (int i = 0; i < T; ++i) {
    sncc_segment *o = out + seg_off[i];
    for (const Seg &g : lists[i]) {
      o->x = g.x;
      o->y = g.y;
      o->w = g.w;
      o->h = g.h;
      o->sum = g.sum;
      o->area = (int32_t)g.area;
      o->reserved = 0;
      ++o;
    }
  }
  if (first_bad != SNCC_OK)
    SNCC_FAIL(first_bad, "template %d: uniform template approximation", bad_index);
  return SNCC_OK;
}

int sncc_ctx_create(int device, uintptr_t hip_stream, sncc_ctx **out) {
  g_err.clear();
  if (!out) SNCC_FAIL(SNCC_EINVAL, "NULL output");
  *out = nullptr;
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) SNCC_FAIL(SNCC_EINVAL, "device %d of %d", device, n);
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  // set-up of the allocation-free entry point on this device (its static
  // scratch's address, looked up once per device with the device current)
  if (sat_noalloc_init(device) != 0)
    SNCC_FAIL(SNCC_EDEVICE, "static scratch address on device %d: %s", device,
              hipGetErrorString(hipGetLastError()));
  sncc_ctx *c = new (std::nothrow) sncc_ctx();
  if (!c) SNCC_FAIL(SNCC_ENOMEM, "context allocation");
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->num_cu = prop.multiProcessorCount;
  *out = c;
  return SNCC_OK;
}

int sncc_ctx_destroy(sncc_ctx *ctx) {
  g_err.clear();
  if (!ctx) return SNCC_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  reap(ctx, true);
  delete ctx;
  return SNCC_OK;
}

int sncc_ctx_set_timing(sncc_ctx *ctx, int enable) {
  g_err.clear();
  CHK(check_ctx(ctx));
  if (enable)
    for (auto &e : ctx->tev)
      if (!e) HIPCHK(hipEventCreate(&e));
  ctx->timing = enable != 0;
  ctx->n_stages = 0;
  return SNCC_OK;
}

int sncc_ctx_stage_ms(sncc_ctx *ctx, float *ms, int cap, int *n) {
  g_err.clear();
  CHK(check_ctx(ctx));
  if (!n || (cap > 0 && !ms)) SNCC_FAIL(SNCC_EINVAL, "NULL output");
  *n = ctx->n_stages;
  if (ctx->n_stages == 0) return SNCC_OK;
  HIPCHK(hipEventSynchronize(ctx->tev[ctx->n_stages]));
  for (int i = 0; i < ctx->n_stages && i < cap; ++i)
    HIPCHK(hipEventElapsedTime(&ms[i], ctx->tev[i], ctx->tev[i + 1]));
  return SNCC_OK;
}

int sncc_sync(sncc_ctx *ctx) {
  g_err.clear();
  CHK(check_ctx(ctx));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  reap(ctx, true);
  HIPCHK(hipGetLastError());
  return SNCC_OK;
}

int sncc_sat_pitch(int M, int *pitch_elems) {
  if (M < 1 || !pitch_elems) SNCC_FAIL(SNCC_EINVAL, "bad width");
  *pitch_elems = ((M + 1) + 63) / 64 * 64;
  return SNCC_OK;
}

int sncc_build_sats(sncc_ctx *ctx, const uint8_t *d_f, int B, int M, int N, int f_pitch,
                    uint32_t *d_s, uint32_t *d_s2, int sat_pitch) {
  g_err.clear();
  CHK(check_ctx(ctx));
  if (!d_f) SNCC_FAIL(SNCC_EINVAL, "NULL frames");
  if (B < 1) SNCC_FAIL(SNCC_EINVAL, "B must be >= 1");
  if (f_pitch < M) SNCC_FAIL(SNCC_EINVAL, "f_pitch %d < M %d", f_pitch, M);
  CHK(check_sats(d_s, d_s2, M, N, sat_pitch));
  CHK(ctx->sat_scratch.reserve(sat_scratch_words(B, M, N) * 4));
  if (launch_sat(d_f, B, M, N, f_pitch, d_s, d_s2, sat_pitch,
                 ctx->sat_scratch.as<uint32_t>(), ctx->stream) != 0)
    SNCC_FAIL(SNCC_EDEVICE, "sum-table launch: %s", hipGetErrorString(hipGetLastError()));
  return SNCC_OK;
}

int sncc_build_sats_noalloc(sncc_ctx *ctx, const uint8_t *d_f, int B, int M, int N,
                            int f_pitch, uint32_t *d_s, uint32_t *d_s2, int sat_pitch) {
  g_err.clear();
  CHK(check_ctx(ctx));
  if (!d_f) SNCC_FAIL(SNCC_EINVAL, "NULL frames");
  if (B < 1) SNCC_FAIL(SNCC_EINVAL, "B must be >= 1");
  if (f_pitch < M) SNCC_FAIL(SNCC_EINVAL, "f_pitch %d < M %d", f_pitch, M);
  CHK(check_sats(d_s, d_s2, M, N, sat_pitch));
  const size_t need = sat_scratch_words(B, M, N) * 4;
  if (need > (size_t)SNCC_NOALLOC_SCRATCH_BYTES)
    SNCC_FAIL(SNCC_ENOSPC,
              "%d frames of %dx%d need %zu bytes of carries; the static scratch holds %d "
              "(split the frames into several calls)", B, M, N, need,
              SNCC_NOALLOC_SCRATCH_BYTES);
  uint32_t *scratch = sat_noalloc_addr(ctx->device);
  if (!scratch) SNCC_FAIL(SNCC_EDEVICE, "static scratch not set up on device %d", ctx->device);
  if (launch_sat(d_f, B, M, N, f_pitch, d_s, d_s2, sat_pitch, scratch, ctx->stream) != 0)
    SNCC_FAIL(SNCC_EDEVICE, "sum-table launch: %s", hipGetErrorString(hipGetLastError()));
  return SNCC_OK;
}

int sncc_upload_templates(sncc_ctx *ctx, int T, const sncc_segment *const *segs, const int *K,
                          const int *W, const int *H, sncc_tmpl **out) {
  g_err.clear();
  CHK(check_ctx(ctx));
  if (!out || !segs || !K || !W || !H || T < 1) SNCC_FAIL(SNCC_EINVAL, "bad template arguments");
  *out = nullptr;
  std::unique_ptr<sncc_tmpl> tm(new (std::nothrow) sncc_tmpl());
  if (!tm) SNCC_FAIL(SNCC_ENOMEM, "template allocation");
  static std::atomic<uint64_t> serials{0};
  tm->ctx = ctx;
  tm->serial = ++serials;
  tm->T = T;
  std::vector<int4> geom;
  std::vector<double> c64all;
  std::vector<int> areas;
  CHK(fill_templates(tm.get(), T, segs, K, W, H, geom, c64all, areas));
  std::vector<float> c32all(c64all.begin(), c64all.end());
  CHK(tm->d_geom.upload(geom, ctx->stream));
  CHK(tm->d_c64.upload(c64all, ctx->stream));
  CHK(tm->d_c32.upload(c32all, ctx->stream));
  CHK(tm->d_area.upload(areas, ctx->stream));
  CHK(tm->d_dev.upload(tm->dev, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *out = tm.release();
  return SNCC_OK;
}

int sncc_tmpl_destroy(sncc_tmpl *tm) {
  g_err.clear();
  if (!tm) return SNCC_OK;
  if (tm->ctx) {
    (void)hipSetDevice(tm->ctx->device);
    (void)hipStreamSynchronize(tm->ctx->stream);
  }
  delete tm;
  return SNCC_OK;
}

int sncc_tmpl_info(const sncc_tmpl *tm, int index, int *W, int *H, int *K, double *q_k) {
  g_err.clear();
  if (!tm || index < 0 || index >= tm->T) SNCC_FAIL(SNCC_EINVAL, "bad template index");
  if (W) *W = tm->W[index];
  if (H) *H = tm->H[index];
  if (K) *K = tm->K[index];
  if (q_k) *q_k = tm->q_k[index];
  return SNCC_OK;
}

int sncc_tmpl_count(const sncc_tmpl *tm, int *T) {
  g_err.clear();
  if (!tm || !T) SNCC_FAIL(SNCC_EINVAL, "NULL template set or output");
  *T = tm->T;
  return SNCC_OK;
}

int sncc_score(sncc_ctx *ctx, const sncc_tmpl *tm, int index, const uint32_t *d_s,
               const uint32_t *d_s2, int M, int N, int sat_pitch, int precision, void *d_rho,
               int rho_pitch, uint8_t *d_degenerate) {
  g_err.clear();
  CHK(check_ctx(ctx));
  CHK(check_sats(d_s, d_s2, M, N, sat_pitch));
  if (!tm || index < 0 || index >= tm->T) SNCC_FAIL(SNCC_EINVAL, "bad template index");
  if (!d_rho || !aligned16(d_rho)) SNCC_FAIL(SNCC_EINVAL, "NULL or misaligned rho map");
  const int nu = M - tm->W[index] + 1, nv = N - tm->H[index] + 1;
  if (nu < 1 || nv < 1) SNCC_FAIL(SNCC_EINVAL, "template larger than image");
  if (rho_pitch < nu) SNCC_FAIL(SNCC_EINVAL, "rho_pitch %d < %d", rho_pitch, nu);
  if (precision == SNCC_FP64) {
    PlainArgs a;
    a.s = d_s;
    a.s2 = d_s2;
    a.sat_pitch = sat_pitch;
    a.nu = nu;
    a.nv = nv;
    a.W = tm->W[index];
    a.H = tm->H[index];
    a.K = tm->K[index];
    a.sq_rows = tm->dev[index].sq_rows;
    a.q_k = tm->q_k[index];
    a.r64 = tm->r64[index];
    a.geom = tm->d_geom.as<int4>() + tm->seg_off[index];
    a.c64 = tm->d_c64.as<double>() + tm->seg_off[index];
    a.area = tm->d_area.as<int>() + tm->seg_off[index];
    a.rho = static_cast<double *>(d_rho);
    a.rho_pitch = rho_pitch;
    a.degen = d_degenerate;
    if (launch_plain(a, ctx->stream) != 0)
      SNCC_FAIL(SNCC_EDEVICE, "plain launch: %s", hipGetErrorString(hipGetLastError()));
    return SNCC_OK;
  }
  if (precision != SNCC_FP32_KAHAN) SNCC_FAIL(SNCC_EINVAL, "unknown precision %d", precision);
  // the plan of the last map call is kept and reused when the call repeats
  // (same template set and index, sizes and pitch)
  const int32_t pair[2] = {0, index};
  PlanKey key;
  key.sink = kSinkMap;
  key.tmpl = tm->serial;
  key.M = M;
  key.N = N;
  key.P = sat_pitch;
  key.pairs.assign(pair, pair + 2);
  PlanDev *pd = nullptr;
  CHK(cached_plan(ctx, std::move(key), [&](PlanDev &d) {
    return build_one_call_plan(tm, M, N, sat_pitch, 1, pair, 0, kSinkMap, ctx->num_cu, d.h);
  }, &pd));
  TileArgs a = pd->args(d_s, d_s2, (long long)(N + 1) * sat_pitch, sat_pitch, M, N);
  a.rho = d_rho;
  a.rho_pitch = rho_pitch;
  a.degen = d_degenerate;
  // the map sink uses no counters but the queues' (none with one workgroup
  // per item)
  if ((a.nq != 0 && launch_zero(a.queue, a.n_zero, ctx->stream) != 0) ||
      launch_tile(pd->h.cfg, kSinkMap, a, pd->h.grid, pd->h.lds_bytes, ctx->stream) != 0)
    SNCC_FAIL(SNCC_EDEVICE, "tile launch: %s", hipGetErrorString(hipGetLastError()));
  return SNCC_OK;
}

constexpr int kTileLocalMaxK = 40;
constexpr long long kTileLocalMaxOffsets = 1 << 19;

int sncc_score_frame(sncc_ctx *ctx, const sncc_tmpl *tm, int index, const uint8_t *d_f,
                     int M, int N, int f_pitch, int form, float *d_rho, int rho_pitch,
                     uint8_t *d_degenerate, int64_t *d_energy, int *form_used) {
  g_err.clear();
  CHK(check_ctx(ctx));
  if (!tm || index < 0 || index >= tm->T) SNCC_FAIL(SNCC_EINVAL, "bad template index");
  if (!d_f || !aligned16(d_f)) SNCC_FAIL(SNCC_EINVAL, "NULL or misaligned frame");
  if (M < 1 || N < 1 || f_pitch < M) SNCC_FAIL(SNCC_EINVAL, "bad frame size %dx%d, pitch %d", M,
                                                N, f_pitch);
  if (!d_rho || !aligned16(d_rho)) SNCC_FAIL(SNCC_EINVAL, "NULL or misaligned rho map");
  if (d_energy && ((uintptr_t)d_energy & 7u)) SNCC_FAIL(SNCC_EINVAL, "misaligned energy map");
  if (form < SNCC_FORM_AUTO || form > SNCC_FORM_GLOBAL) SNCC_FAIL(SNCC_EINVAL, "bad form %d", form);
  const int W = tm->W[index], H = tm->H[index];
  const int nu = M - W + 1, nv = N - H + 1;
  if (nu < 1 || nv < 1) SNCC_FAIL(SNCC_EINVAL, "template larger than image");
  if (rho_pitch < nu) SNCC_FAIL(SNCC_EINVAL, "rho_pitch %d < %d", rho_pitch, nu);
  const bool local_ok = (long long)W * H <= kMaxSqBoxArea && fused_lp(W) > 0 &&
                        fused_lds_bytes(W, H) <= (size_t)kFusedMaxLds;
  if (form == SNCC_FORM_TILE_LOCAL && !local_ok)
    SNCC_FAIL(SNCC_ERANGE, "template %dx%d does not allow the tile-local form", W, H);
  // automatic choice: the tile-local form reads four LDS entries per segment
  // and offset where the batched kernel's chains read fewer, and each tile
  // builds its region's tables, so it wins only on small frames with few
  // segments, where the launches of the frame's tables dominate (measured on
  // one MI355X: 640 x 480 at K = 23, 20.8 vs 30 us; 1920 x 1080 at K = 12,
  // 66.5 vs 46 us, at K = 72, 106 vs 73 us)
  const bool local =
      form == SNCC_FORM_TILE_LOCAL ||
      (form == SNCC_FORM_AUTO && local_ok && tm->K[index] <= kTileLocalMaxK &&
       (long long)nu * nv <= kTileLocalMaxOffsets);
  const int used = local ? SNCC_FORM_TILE_LOCAL : SNCC_FORM_GLOBAL;
  if (used == SNCC_FORM_TILE_LOCAL) {
    FusedArgs a;
    a.f = d_f;
    a.M = M;
    a.N = N;
    a.f_pitch = f_pitch;
    a.W = W;
    a.H = H;
    a.K = tm->K[index];
    a.nu = nu;
    a.nv = nv;
    a.geom = tm->d_geom.as<int4>() + tm->seg_off[index];
    a.area = tm->d_area.as<int>() + tm->seg_off[index];
    a.c32 = tm->d_c32.as<float>() + tm->seg_off[index];
    a.q_k = tm->q_k[index];
    a.rho = d_rho;
    a.rho_pitch = rho_pitch;
    a.degen = d_degenerate;
    a.energy = reinterpret_cast<long long *>(d_energy);
    if (launch_fused(a, ctx->stream) != 0)
      SNCC_FAIL(SNCC_EDEVICE, "tile-local launch: %s", hipGetErrorString(hipGetLastError()));
  } else {
    int P = 0;
    sncc_sat_pitch(M, &P);
    const size_t bytes = (size_t)(N + 1) * P * 4;
    CHK(ctx->frame_s.reserve(bytes));
    CHK(ctx->frame_s2.reserve(bytes));
    CHK(ctx->sat_scratch.reserve(sat_scratch_words(1, M, N) * 4));
    uint32_t *s = ctx->frame_s.as<uint32_t>(), *s2 = ctx->frame_s2.as<uint32_t>();
    if (launch_sat(d_f, 1, M, N, f_pitch, s, s2, P, ctx->sat_scratch.as<uint32_t>(),
                   ctx->stream) != 0)
      SNCC_FAIL(SNCC_EDEVICE, "sum-table launch: %s", hipGetErrorString(hipGetLastError()));
    CHK(sncc_score(ctx, tm, index, s, s2, M, N, P, SNCC_FP32_KAHAN, d_rho, rho_pitch,
                   d_degenerate));
    if (d_energy && launch_energy(s, s2, P, nu, nv, W, H, tm->dev[index].sq_rows,
                                  reinterpret_cast<long long *>(d_energy), rho_pitch,
                                  ctx->stream) != 0)
      SNCC_FAIL(SNCC_EDEVICE, "energy launch: %s", hipGetErrorString(hipGetLastError()));
  }
  if (form_used) *form_used = used;
  return SNCC_OK;
}

int sncc_topk(sncc_ctx *ctx, const sncc_tmpl *tm, const uint32_t *d_s, const uint32_t *d_s2,
              int B, int M, int N, int sat_pitch, int n_pairs, const int32_t *pairs, int k,
              int precision, sncc_match *d_out) {
  g_err.clear();
  CHK(check_ctx(ctx));
  CHK(check_sats(d_s, d_s2, M, N, sat_pitch));
  if (B < 1) SNCC_FAIL(SNCC_EINVAL, "B must be >= 1");
  CHK(check_pairs(tm, B, M, N, n_pairs, pairs));
  if (k < 1 || k > 64) SNCC_FAIL(SNCC_EINVAL, "k must be in 1..64");
  if (!d_out || !aligned16(d_out)) SNCC_FAIL(SNCC_EINVAL, "NULL or misaligned output");
  const long long fs = (long long)(N + 1) * sat_pitch;
  if (precision == SNCC_FP32_KAHAN) {
    PlanKey key;
    key.sink = kSinkTopk;
    key.tmpl = tm->serial;
    key.M = M;
    key.N = N;
    key.P = sat_pitch;
    key.k = k;
    key.pairs.assign(pairs, pairs + 2 * n_pairs);
    PlanDev *pd = nullptr;
    CHK(cached_plan(ctx, std::move(key), [&](PlanDev &d) {
      return build_one_call_plan(tm, M, N, sat_pitch, n_pairs, pairs, k, kSinkTopk,
                                 ctx->num_cu, d.h);
    }, &pd));
    TileArgs a = pd->args(d_s, d_s2, fs, sat_pitch, M, N);
    ctx->n_stages = 0;
    // one workgroup per item: no queue counters and no pair floors to reset
    if (a.nq != 0 && launch_zero(a.queue, a.n_zero, ctx->stream) != 0)
      SNCC_FAIL(SNCC_EDEVICE, "top-k launch: %s", hipGetErrorString(hipGetLastError()));
    ctx->mark(0);
    if (launch_tile(pd->h.cfg, kSinkTopk, a, pd->h.grid, pd->h.lds_bytes, ctx->stream) != 0)
      SNCC_FAIL(SNCC_EDEVICE, "top-k launch: %s", hipGetErrorString(hipGetLastError()));
    ctx->mark(1);
    if (launch_merge(pd->d_pairs.as<PairDesc>(), nullptr, n_pairs, a.partial, nullptr, k, d_out,
                     ctx->stream) != 0)
      SNCC_FAIL(SNCC_EDEVICE, "top-k launch: %s", hipGetErrorString(hipGetLastError()));
    ctx->mark(2);
    if (ctx->timing) ctx->n_stages = 2;
    return SNCC_OK;
  }
  if (precision != SNCC_FP64) SNCC_FAIL(SNCC_EINVAL, "unknown precision %d", precision);
  std::unique_ptr<PlanDev> pd(new PlanDev());
  // plain form: one FP64 map per pair, then chunked top-k and the merge
  const int chunk = 64 * 1024;
  PlanHost &h = pd->h;
  h.k = k;
  size_t max_map = 0;
  int n_chunks = 0;
  h.pairs.resize(n_pairs);
  for (int p = 0; p < n_pairs; ++p) {
    const int t = pairs[2 * p + 1];
    PairDesc &q = h.pairs[p];
    q.frame = pairs[2 * p];
    q.tmpl = t;
    q.nu = M - tm->W[t] + 1;
    q.nv = N - tm->H[t] + 1;
    q.ntu = q.ntv = 0;
    const long long tot = (long long)q.nu * q.nv;
    q.item_begin = n_chunks;
    n_chunks += (int)((tot + chunk - 1) / chunk);
    q.item_end = n_chunks;
    max_map = std::max(max_map, (size_t)tot);
  }
  CHK(ctx->map_scratch.reserve(max_map * sizeof(double)));
  CHK(pd->d_pairs.upload(h.pairs, ctx->stream));
  CHK(pd->d_partial.reserve((size_t)n_chunks * k * sizeof(Key96)));
  Key96 *partial = pd->d_partial.as<Key96>();
  for (int p = 0; p < n_pairs; ++p) {
    const PairDesc &q = h.pairs[p];
    const int t = q.tmpl;
    PlainArgs a;
    a.s = d_s + (long long)q.frame * fs;
    a.s2 = d_s2 + (long long)q.frame * fs;
    a.sat_pitch = sat_pitch;
    a.nu = q.nu;
    a.nv = q.nv;
    a.W = tm->W[t];
    a.H = tm->H[t];
    a.K = tm->K[t];
    a.sq_rows = tm->dev[t].sq_rows;
    a.q_k = tm->q_k[t];
    a.r64 = tm->r64[t];
    a.geom = tm->d_geom.as<int4>() + tm->seg_off[t];
    a.c64 = tm->d_c64.as<double>() + tm->seg_off[t];
    a.area = tm->d_area.as<int>() + tm->seg_off[t];
    a.rho = ctx->map_scratch.as<double>();
    a.rho_pitch = q.nu;
    a.degen = nullptr;
    if (launch_plain(a, ctx->stream) != 0 ||
        launch_map_topk64(a.rho, q.nu, q.nu, q.nv, chunk, k,
                          partial + (size_t)q.item_begin * k, ctx->stream) != 0)
      SNCC_FAIL(SNCC_EDEVICE, "plain top-k launch: %s", hipGetErrorString(hipGetLastError()));
  }
  if (launch_merge64(pd->d_pairs.as<PairDesc>(), n_pairs, partial, k, d_out, ctx->stream) != 0)
    SNCC_FAIL(SNCC_EDEVICE, "merge launch: %s", hipGetErrorString(hipGetLastError()));
  return retire(ctx, std::move(pd));
}

int sncc_argmax(sncc_ctx *ctx, const sncc_tmpl *tm, const uint32_t *d_s, const uint32_t *d_s2,
                int B, int M, int N, int sat_pitch, int n_pairs, const int32_t *pairs,
                int precision, sncc_match *d_out) {
  return sncc_topk(ctx, tm, d_s, d_s2, B, M, N, sat_pitch, n_pairs, pairs, 1, precision, d_out);
}

static int check_fine(const sncc_tmpl *fine, int B, int M, int N, int n_pairs,
                      const int32_t *pairs, int n_cand, int radius) {
  CHK(check_pairs(fine, B, M, N, n_pairs, pairs));
  if (n_cand < 1 || radius < 0 || radius > 7)
    SNCC_FAIL(SNCC_EINVAL, "bad candidate count %d or radius %d", n_cand, radius);
  if (n_cand * (2 * radius + 1) * (2 * radius + 1) > 4096)
    SNCC_FAIL(SNCC_EINVAL, "n_cand * (2 radius + 1)^2 must be <= 4096");
  return SNCC_OK;
}

int sncc_refine(sncc_ctx *ctx, const sncc_tmpl *fine, const uint32_t *d_s, const uint32_t *d_s2,
                int B, int M, int N, int sat_pitch, int n_pairs, const int32_t *pairs,
                const sncc_match *d_cand, int n_cand, int radius, sncc_match64 *d_out,
                int32_t *d_count) {
  g_err.clear();
  CHK(check_ctx(ctx));
  CHK(check_sats(d_s, d_s2, M, N, sat_pitch));
  if (B < 1) SNCC_FAIL(SNCC_EINVAL, "B must be >= 1");
  CHK(check_fine(fine, B, M, N, n_pairs, pairs, n_cand, radius));
  if (!d_cand || !d_out || !aligned16(d_out)) SNCC_FAIL(SNCC_EINVAL, "NULL or misaligned buffers");
  std::unique_ptr<PlanDev> pd(new PlanDev());
  PlanHost &h = pd->h;
  h.pairs.resize(n_pairs);
  for (int p = 0; p < n_pairs; ++p) {
    const int t = pairs[2 * p + 1];
    PairDesc &q = h.pairs[p];
    q = PairDesc{};
    q.frame = pairs[2 * p];
    q.tmpl = t;
    q.nu = M - fine->W[t] + 1;
    q.nv = N - fine->H[t] + 1;
  }
  CHK(pd->d_pairs.upload(h.pairs, ctx->stream));
  plan_slots(fine, kRefineWideSpanU, kRefineWideSpanV, kRefineRegionWords, h, kRefineSpanU,
             kRefineSpanV);
  plan_refine_order(h, n_cand, radius);
  CHK(pd->d_slow.upload(h.slow, ctx->stream));
  CHK(pd->d_slot_off.upload(h.slot_off, ctx->stream));
  CHK(pd->d_slot_w.upload(h.slot_w, ctx->stream));
  CHK(pd->d_refine_order.upload(h.refine_order, ctx->stream));
  if (launch_refine(d_s, d_s2, (long long)(N + 1) * sat_pitch, sat_pitch,
                    fine->d_dev.as<DevTmpl>(), fine->d_geom.as<int4>(), fine->d_c64.as<double>(),
                    pd->slots(), pd->d_pairs.as<PairDesc>(), n_pairs, d_cand, n_cand, radius,
                    d_out, d_count, ctx->stream) != 0)
    SNCC_FAIL(SNCC_EDEVICE, "refine launch: %s", hipGetErrorString(hipGetLastError()));
  return retire(ctx, std::move(pd));
}

int sncc_threshold_match(sncc_ctx *ctx, const sncc_tmpl *fast, const sncc_tmpl *slow,
                         const double *thr_fast, const double *thr_slow, const uint32_t *d_s,
                         const uint32_t *d_s2, int B, int M, int N, int sat_pitch, int n_pairs,
                         const int32_t *pairs, sncc_hit *d_cand, int cand_cap, sncc_hit *d_out,
                         int out_cap, int32_t *d_counts) {
  g_err.clear();
  CHK(check_ctx(ctx));
  CHK(check_sats(d_s, d_s2, M, N, sat_pitch));
  if (B < 1) SNCC_FAIL(SNCC_EINVAL, "B must be >= 1");
  if (!fast || !slow) SNCC_FAIL(SNCC_EINVAL, "NULL template set");
  if (fast->T != slow->T) SNCC_FAIL(SNCC_EINVAL, "fast and slow sets differ in size");
  for (int t = 0; t < fast->T; ++t)
    if (fast->W[t] != slow->W[t] || fast->H[t] != slow->H[t])
      SNCC_FAIL(SNCC_EINVAL, "slow template %d differs in size from the fast one", t);
  CHK(check_pairs(fast, B, M, N, n_pairs, pairs));
  if (!thr_fast || !thr_slow) SNCC_FAIL(SNCC_EINVAL, "NULL thresholds");
  for (int t = 0; t < fast->T; ++t)
    if (!std::isfinite(thr_fast[t]) || !std::isfinite(thr_slow[t]))
      SNCC_FAIL(SNCC_EINVAL, "threshold of template %d is not finite", t);
  if (cand_cap < 1 || out_cap < 1) SNCC_FAIL(SNCC_EINVAL, "capacities must be >= 1");
  if (!d_cand || !d_out || !d_counts || !aligned16(d_cand) || !aligned16(d_out) ||
      !aligned16(d_counts))
    SNCC_FAIL(SNCC_EINVAL, "NULL or misaligned buffers");
  const long long fs = (long long)(N + 1) * sat_pitch;
  PlanKey key;
  key.sink = kSinkCompact;
  key.tmpl = fast->serial;
  key.tmpl2 = slow->serial;
  key.M = M;
  key.N = N;
  key.P = sat_pitch;
  key.pairs.assign(pairs, pairs + 2 * n_pairs);
  key.thr.assign(thr_fast, thr_fast + fast->T);
  key.thr.insert(key.thr.end(), thr_slow, thr_slow + slow->T);
  PlanDev *pd = nullptr;
  CHK(cached_plan(ctx, std::move(key), [&](PlanDev &d) {
    CHK(build_plan(fast, 0, M, N, sat_pitch, n_pairs, pairs, 1, kSinkCompact, ctx->num_cu, d.h,
                   thr_fast));
    plan_slow(slow, d.h.tc, d.h);
    std::vector<double> ts(thr_slow, thr_slow + slow->T);
    return d.d_thr.upload(ts, ctx->stream);
  }, &pd));
  TileArgs a = pd->args(d_s, d_s2, fs, sat_pitch, M, N);
  a.co.hits = d_cand;
  a.co.cap = cand_cap;
  a.co.count = d_counts;
  ctx->n_stages = 0;
  if (launch_zero(a.queue, a.n_zero, ctx->stream) != 0 ||
      launch_zero(d_counts, 2, ctx->stream) != 0)
    SNCC_FAIL(SNCC_EDEVICE, "threshold search launch: %s", hipGetErrorString(hipGetLastError()));
  ctx->mark(0);
  if (launch_tile(pd->h.cfg, kSinkCompact, a, pd->h.grid, pd->h.lds_bytes, ctx->stream) != 0)
    SNCC_FAIL(SNCC_EDEVICE, "threshold search launch: %s", hipGetErrorString(hipGetLastError()));
  ctx->mark(1);
  SlowArgs sa;
  sa.s = d_s;
  sa.s2 = d_s2;
  sa.frame_stride = fs;
  sa.P = sat_pitch;
  sa.N = N;
  sa.tmpls = slow->d_dev.as<DevTmpl>();
  sa.geom = slow->d_geom.as<int4>();
  sa.c64 = slow->d_c64.as<double>();
  sa.stmpl = pd->d_slow.as<SlowTmpl>();
  sa.slot_off = pd->d_slot_off.as<uint32_t>();
  sa.slot_w = pd->d_slot_w.as<double>();
  sa.pairs = pd->d_pairs.as<PairDesc>();
  sa.thr = pd->d_thr.as<double>();
  sa.cand = d_cand;
  sa.cand_count = d_counts;
  sa.cand_cap = cand_cap;
  sa.runs = a.co.runs;
  sa.run_count = a.co.run_count;
  sa.run_cap = a.co.run_cap;
  sa.work = a.queue + kQueueInts + 8;
  sa.out = d_out;
  sa.out_cap = out_cap;
  sa.out_count = d_counts + 1;
  const int slow_lds = pd->h.slow_lds;
  const int slow_grid = std::max(1, std::min(pd->h.run_cap, ctx->num_cu * slow_occupancy(slow_lds)));
  if (launch_slow(sa, slow_grid, slow_lds, ctx->stream) != 0)
    SNCC_FAIL(SNCC_EDEVICE, "threshold search launch: %s", hipGetErrorString(hipGetLastError()));
  ctx->mark(2);
  if (ctx->timing) ctx->n_stages = 2;
  return SNCC_OK;
}

}  // extern "C"

// ================================================================= batches
struct sncc_batch {
  sncc_ctx *ctx = nullptr;
  sncc_batch_desc d{};
  std::vector<int32_t> pairs;
  std::unique_ptr<PlanDev> plan;
  std::unique_ptr<PlanDev> edge;  // narrow last tile columns (second scoring launch)
  DevBuf sat_scratch;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev[5] = {};
  bool timed = false;
  std::string capture_note;  // why the timed graph was not built, if it was not
  ~sncc_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

// Enqueues stage `stage` of one run of the batch on stream `st`:
// 0 sum tables, 1 scoring, 2 top-k merge, 3 FP64 refinement.
int enqueue_stage(sncc_batch *b, int stage, hipStream_t st) {
  const sncc_batch_desc &d = b->d;
  PlanDev &pd = *b->plan;
  const long long fs = (long long)(d.N + 1) * d.sat_pitch;
  TileArgs a = pd.args(d.d_s, d.d_s2, fs, d.sat_pitch, d.M, d.N);
  switch (stage) {
    case 0:
      if (d.d_f && launch_sat(d.d_f, d.B, d.M, d.N, d.f_pitch, d.d_s, d.d_s2, d.sat_pitch,
                              b->sat_scratch.as<uint32_t>(), st) != 0)
        SNCC_FAIL(SNCC_EDEVICE, "sum-table launch");
      return SNCC_OK;
    case 1:
      if (launch_zero(a.queue, a.n_zero, st) != 0 ||
          launch_tile(pd.h.cfg, kSinkTopk, a, pd.h.grid, pd.h.lds_bytes, st) != 0)
        SNCC_FAIL(SNCC_EDEVICE, "scoring launch");
      if (b->edge) {
        // the last columns start from the floors the main launch published
        PlanDev &pe = *b->edge;
        TileArgs ae = pe.args(d.d_s, d.d_s2, fs, d.sat_pitch, d.M, d.N);
        ae.pair_floor = a.pair_floor;
        if (launch_zero(ae.queue, kQueueInts, st) != 0 ||
            launch_tile(pe.h.cfg, kSinkTopk, ae, pe.h.grid, pe.h.lds_bytes, st) != 0)
          SNCC_FAIL(SNCC_EDEVICE, "scoring launch (last columns)");
      }
      return SNCC_OK;
    case 2:
      if (launch_merge(pd.d_pairs.as<PairDesc>(),
                       b->edge ? b->edge->d_pairs.as<PairDesc>() : nullptr, d.n_pairs, a.partial,
                       b->edge ? b->edge->d_partial.as<unsigned long long>() : nullptr, d.k,
                       d.d_topk, st) != 0)
        SNCC_FAIL(SNCC_EDEVICE, "merge launch");
      return SNCC_OK;
    case 3:
      if (d.fine &&
          launch_refine(d.d_s, d.d_s2, fs, d.sat_pitch, d.fine->d_dev.as<DevTmpl>(),
                        d.fine->d_geom.as<int4>(), d.fine->d_c64.as<double>(), pd.slots(),
                        pd.d_pairs.as<PairDesc>(), d.n_pairs, d.d_topk,
                        d.k, d.radius, d.d_best, d.d_count, st) != 0)
        SNCC_FAIL(SNCC_EDEVICE, "refine launch");
      return SNCC_OK;
  }
  return SNCC_OK;
}

bool stage_used(const sncc_batch *b, int stage) {
  return stage == 1 || stage == 2 || (stage == 0 && b->d.d_f) || (stage == 3 && b->d.fine);
}

int capture_stage(sncc_batch *b, int stage, hipGraph_t *out) {
  *out = nullptr;
  HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  const int st = enqueue_stage(b, stage, b->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (st != SNCC_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    SNCC_FAIL(st != SNCC_OK ? st : SNCC_EDEVICE, "capture of stage %d failed: %s", stage,
              hipGetErrorString(e));
  }
  *out = g;
  return SNCC_OK;
}

// One graph per run: each stage captured as a child graph; with `timed`,
// event-record nodes between the stages give per-stage device times.
int capture(sncc_batch *b, bool timed) {
  hipGraph_t parent = nullptr;
  HIPCHK(hipGraphCreate(&parent, 0));
  hipGraphNode_t prev = nullptr;
  int rc = SNCC_OK;
  auto fail = [&](int code) {
    (void)hipGraphDestroy(parent);
    (void)hipGetLastError();
    return code;
  };
  auto add_event = [&](hipEvent_t e) -> int {
    hipGraphNode_t n = nullptr;
    if (hipGraphAddEventRecordNode(&n, parent, prev ? &prev : nullptr, prev ? 1 : 0, e) !=
        hipSuccess)
      SNCC_FAIL(SNCC_EDEVICE, "event-record node: %s", hipGetErrorString(hipGetLastError()));
    prev = n;
    return SNCC_OK;
  };
  if (timed && (rc = add_event(b->ev[0])) != SNCC_OK) return fail(rc);
  for (int stage = 0; stage < 4; ++stage) {
    if (stage_used(b, stage)) {
      hipGraph_t g = nullptr;
      if ((rc = capture_stage(b, stage, &g)) != SNCC_OK) return fail(rc);
      hipGraphNode_t n = nullptr;
      const hipError_t e =
          hipGraphAddChildGraphNode(&n, parent, prev ? &prev : nullptr, prev ? 1 : 0, g);
      (void)hipGraphDestroy(g);  // the child node holds its own copy
      if (e != hipSuccess) {
        set_error("child graph node: %s", hipGetErrorString(e));
        return fail(SNCC_EDEVICE);
      }
      prev = n;
    }
    if (timed && (rc = add_event(b->ev[stage + 1])) != SNCC_OK) return fail(rc);
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, parent, nullptr, nullptr, 0) != hipSuccess) {
    set_error("graph instantiation: %s", hipGetErrorString(hipGetLastError()));
    return fail(SNCC_EDEVICE);
  }
  b->graph = parent;
  b->exec = x;
  b->timed = timed;
  return SNCC_OK;
}

std::string tune_key(const sncc_batch_desc &d) {
  std::ostringstream os;
  os << "gfx950|M" << d.M << "|N" << d.N << "|B" << d.B << "|P" << d.n_pairs << "|k" << d.k;
  unsigned long long h = 1469598103934665603ull;
  for (int t = 0; t < d.coarse->T; ++t) {
    for (long long v : {(long long)d.coarse->W[t], (long long)d.coarse->H[t],
                        (long long)d.coarse->K[t]}) {
      h ^= (unsigned long long)v;
      h *= 1099511628211ull;
    }
  }
  os << "|h" << std::hex << h;
  return os.str();
}

int read_cache(const char *path, const std::string &key) {
  if (!path) return -1;
  std::ifstream in(path);
  if (!in) return -1;
  std::string line;
  while (std::getline(in, line)) {
    const size_t a = line.find('"' + key + '"');
    if (a == std::string::npos) continue;
    const size_t c = line.find(':', a);
    if (c == std::string::npos) continue;
    return std::atoi(line.c_str() + c + 1);
  }
  return -1;
}

void write_cache(const char *path, const std::string &key, int cfg) {
  if (!path) return;
  std::vector<std::string> lines;
  {
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line))
      if (line.find('"') != std::string::npos && line.find('"' + key + '"') == std::string::npos)
        lines.push_back(line);
  }
  std::ofstream out(path);
  out << "{\n";
  for (auto &l : lines) {
    std::string s = l;
    while (!s.empty() && (s.back() == ',' || s.back() == ' ')) s.pop_back();
    out << s << ",\n";
  }
  out << "  \"" << key << "\": " << cfg << "\n}\n";
}

// Times the scoring launch of each tile configuration on this batch and
// returns the fastest.
int autotune(sncc_batch *b, int *best_cfg) {
  const sncc_batch_desc &d = b->d;
  const long long fs = (long long)(d.N + 1) * d.sat_pitch;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best = 1e30f;
  *best_cfg = 0;
  for (int c = 0; c < tile_cfg_count(); ++c) {
    PlanDev pd;
    if (build_plan(d.coarse, c, d.M, d.N, d.sat_pitch, d.n_pairs, b->pairs.data(), d.k, kSinkTopk,
                   b->ctx->num_cu, pd.h) != SNCC_OK)
      continue;
    if (pd.upload(b->ctx->stream) != SNCC_OK) continue;
    TileArgs a = pd.args(d.d_s, d.d_s2, fs, d.sat_pitch, d.M, d.N);
    float ms = 0;
    for (int rep = 0; rep < 2; ++rep) {
      launch_zero(a.queue, a.n_zero, b->ctx->stream);
      HIPCHK(hipEventRecord(e0, b->ctx->stream));
      launch_tile(c, kSinkTopk, a, pd.h.grid, pd.h.lds_bytes, b->ctx->stream);
      HIPCHK(hipEventRecord(e1, b->ctx->stream));
      HIPCHK(hipEventSynchronize(e1));
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    }
    if (getenv("SNCC_TUNE_LOG")) {
      const TileCfg tc = tile_cfg(c);
      fprintf(stderr, "[sncc tune] cfg %d: tile %dx%d, %d threads, %d WG/CU budget, %s order, "
              "LDS %d B, %zu items: %.3f ms\n", c, tc.bu(), tc.bv(), tc.threads(), tc.wgs,
              tc.frame_major ? "frame-major" : "cost", pd.h.lds_bytes, pd.h.items.size(), ms);
    }
    if (ms < best) {
      best = ms;
      *best_cfg = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return SNCC_OK;
}

}  // namespace

extern "C" {

int sncc_batch_create(sncc_ctx *ctx, const sncc_batch_desc *desc, sncc_batch **out) {
  g_err.clear();
  CHK(check_ctx(ctx));
  if (!desc || !out) SNCC_FAIL(SNCC_EINVAL, "NULL argument");
  *out = nullptr;
  const sncc_batch_desc &d = *desc;
  CHK(check_sats(d.d_s, d.d_s2, d.M, d.N, d.sat_pitch));
  if (d.B < 1) SNCC_FAIL(SNCC_EINVAL, "B must be >= 1");
  CHK(check_pairs(d.coarse, d.B, d.M, d.N, d.n_pairs, d.pairs));
  if (d.k < 1 || d.k > 64) SNCC_FAIL(SNCC_EINVAL, "k must be in 1..64");
  if (!d.d_topk || !aligned16(d.d_topk)) SNCC_FAIL(SNCC_EINVAL, "NULL or misaligned d_topk");
  if (d.d_f && d.f_pitch < d.M) SNCC_FAIL(SNCC_EINVAL, "f_pitch < M");
  if (d.fine) {
    CHK(check_fine(d.fine, d.B, d.M, d.N, d.n_pairs, d.pairs, d.k, d.radius));
    if (!d.d_best || !aligned16(d.d_best)) SNCC_FAIL(SNCC_EINVAL, "NULL or misaligned d_best");
    if (d.fine->T != d.coarse->T) SNCC_FAIL(SNCC_EINVAL, "fine and coarse sets differ in size");
    for (int t = 0; t < d.coarse->T; ++t)
      if (d.fine->W[t] != d.coarse->W[t] || d.fine->H[t] != d.coarse->H[t])
        SNCC_FAIL(SNCC_EINVAL, "fine template %d differs in size from the coarse one", t);
  }
  std::unique_ptr<sncc_batch> b(new (std::nothrow) sncc_batch());
  if (!b) SNCC_FAIL(SNCC_ENOMEM, "batch allocation");
  b->ctx = ctx;
  b->d = d;
  b->pairs.assign(d.pairs, d.pairs + 2 * (size_t)d.n_pairs);
  b->d.pairs = b->pairs.data();
  if (d.d_f) CHK(b->sat_scratch.reserve(sat_scratch_words(d.B, d.M, d.N) * 4));

  int cfg = 0;
  if (d.tune) {
    const std::string key = tune_key(d);
    cfg = read_cache(d.tune_cache, key);
    if (cfg < 0 || cfg >= tile_cfg_count()) {
      if (d.d_f) {  // the candidates are timed on real sum tables
        if (launch_sat(d.d_f, d.B, d.M, d.N, d.f_pitch, d.d_s, d.d_s2, d.sat_pitch,
                       b->sat_scratch.as<uint32_t>(), ctx->stream) != 0)
          SNCC_FAIL(SNCC_EDEVICE, "sum-table launch");
      }
      CHK(autotune(b.get(), &cfg));
      write_cache(d.tune_cache, key, cfg);
    }
  }
  // a second launch of half-width tiles for last tile columns that are at
  // most half full, when the chosen shape has a half-width twin
  const TileCfg main_tc = tile_cfg(cfg);
  int edge_cfg = -1;
  for (int c = 0; c < tile_cfg_count() && main_tc.ru == 2; ++c) {
    const TileCfg t = tile_cfg(c);
    if (t.ru == 1 && t.rv == main_tc.rv && t.nw == main_tc.nw && t.wgs == main_tc.wgs &&
        t.frame_major == main_tc.frame_major)
      edge_cfg = c;
  }
  bool any_edge = false;
  for (int p = 0; p < d.n_pairs && edge_cfg >= 0; ++p)
    any_edge |= has_edge(d.M - d.coarse->W[b->pairs[2 * p + 1]] + 1, main_tc.bu());
  const int split = any_edge ? kSplitMain : kSplitNone;
  b->plan.reset(new PlanDev());
  CHK(build_plan(d.coarse, cfg, d.M, d.N, d.sat_pitch, d.n_pairs, b->pairs.data(), d.k, kSinkTopk,
                 ctx->num_cu, b->plan->h, nullptr, split));
  if (d.fine) {
    plan_slots(d.fine, kRefineWideSpanU, kRefineWideSpanV, kRefineRegionWords, b->plan->h,
               kRefineSpanU, kRefineSpanV);
    plan_refine_order(b->plan->h, d.k, d.radius);
  }
  CHK(b->plan->upload(ctx->stream));
  if (any_edge) {
    b->edge.reset(new PlanDev());
    CHK(build_plan(d.coarse, edge_cfg, d.M, d.N, d.sat_pitch, d.n_pairs, b->pairs.data(), d.k,
                   kSinkTopk, ctx->num_cu, b->edge->h, nullptr, kSplitEdge, main_tc.bu()));
    CHK(b->edge->upload(ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));

  HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  for (auto &e : b->ev) HIPCHK(hipEventCreate(&e));
  if (capture(b.get(), true) != SNCC_OK) {
    b->capture_note = sncc_last_error();
    CHK(capture(b.get(), false));
  }
  *out = b.release();
  return SNCC_OK;
}

int sncc_batch_run(sncc_batch *b) {
  g_err.clear();
  if (!b) SNCC_FAIL(SNCC_EINVAL, "NULL batch");
  CHK(check_ctx(b->ctx));
  HIPCHK(hipGraphLaunch(b->exec, b->ctx->stream));
  return SNCC_OK;
}

int sncc_batch_stats_get(sncc_batch *b, sncc_batch_stats *st) {
  g_err.clear();
  if (!b || !st) SNCC_FAIL(SNCC_EINVAL, "NULL argument");
  const PlanHost &h = b->plan->h;
  memset(st, 0, sizeof *st);
  st->coarse_evals = h.coarse_evals;
  st->computed_evals = h.computed_evals + (b->edge ? b->edge->h.computed_evals : 0);
  st->n_passes = h.n_passes;
  st->n_offsets = h.n_offsets;
  st->work_items = (int64_t)h.items.size() + (b->edge ? (int64_t)b->edge->h.items.size() : 0);
  st->n_launch_classes = b->edge ? 2 : 1;
  st->tile_u = h.tc.bu();
  st->tile_v = h.tc.bv();
  st->wg_threads = h.tc.threads();
  st->lds_bytes = h.lds_bytes;
  st->timed = b->timed ? 1 : 0;
  st->ms_sat = st->ms_score = st->ms_select = st->ms_refine = st->ms_total = -1.f;
  if (b->timed && hipEventQuery(b->ev[4]) == hipSuccess) {
    (void)hipEventElapsedTime(&st->ms_sat, b->ev[0], b->ev[1]);
    (void)hipEventElapsedTime(&st->ms_score, b->ev[1], b->ev[2]);
    (void)hipEventElapsedTime(&st->ms_select, b->ev[2], b->ev[3]);
    (void)hipEventElapsedTime(&st->ms_refine, b->ev[3], b->ev[4]);
    (void)hipEventElapsedTime(&st->ms_total, b->ev[0], b->ev[4]);
    (void)hipGetLastError();
  }
  return SNCC_OK;
}

int sncc_batch_destroy(sncc_batch *b) {
  g_err.clear();
  if (!b) return SNCC_OK;
  (void)hipSetDevice(b->ctx->device);
  (void)hipStreamSynchronize(b->ctx->stream);
  delete b;
  return SNCC_OK;
}

}  // extern "C"
