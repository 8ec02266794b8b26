// Host-only checks of the library's split-and-merge (segment.cpp) and work
// planner (api.cpp), built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_host_sanitize.py.  No GPU: the two sources are compiled into
// this program as host C++, the kernel launchers are stubs that launch
// nothing, and only host code runs.
//
//   host_checks <iterations> <seed>
//
// Segmentation: random templates (sizes 1..48, a few up to 160, several
// kinds of content) at random thresholds and K_max; every list must cover
// the template exactly once with correct sums, hold at most K_max leaves
// before merging, and leave no aligned neighbours with equal exact means.
// Planner: random template sets (fill_templates, as sncc_upload_templates
// does on the host) over random frame sizes and pair lists, for every tile
// configuration and each sink, split and unsplit: work items must cover
// every pair's tiles exactly once, the queues must be a permutation of the
// items, and every LDS read the records imply must stay inside the plan's
// LDS size; the slow pass's and the refine's slot tables must stay inside
// their regions and their weighted corner entries must give the segments'
// sums; the refine's launch classes must order every pair once, each class
// within its LDS size.  Exit status 0 when every check holds.

#include "../../paper_2502_01286_amd/csrc/segment.cpp"
#include "../../paper_2502_01286_amd/csrc/api.cpp"

#include <cstdio>
#include <random>

namespace sncc {

int launch_sat(const uint8_t *, int, int, int, int, uint32_t *, uint32_t *, int, uint32_t *,
               hipStream_t) {
  return -1;
}
size_t sat_scratch_words(int, int, int) { return 0; }
int sat_noalloc_init(int) { return -1; }
uint32_t *sat_noalloc_addr(int) { return nullptr; }
int tile_cfg_count() { return kNumCfgs; }
TileCfg tile_cfg(int i) { return tile_cfg_of(i); }
int launch_slow(const SlowArgs &, int, int, hipStream_t) { return -1; }
int refine_region_budget(int np, int wgs) { return kTileMaxLds / wgs - 2048 - 1024 - np * 4; }
int slow_occupancy(int) { return 1; }
int launch_tile(int, int, const TileArgs &, int, int, hipStream_t) { return -1; }
int tile_max_lds() { return kTileMaxLds; }
int tile_occupancy(int cfg, int, int lds_bytes) {
  return std::max(1, std::min(2 * tile_cfg_of(cfg).wgs, kTileMaxLds / std::max(1, lds_bytes)));
}
int launch_plain(const PlainArgs &, hipStream_t) { return -1; }
int launch_fused(const FusedArgs &, hipStream_t) { return -1; }
int launch_energy(const uint32_t *, const uint32_t *, int, int, int, int, int, int, long long *,
                  int, hipStream_t) {
  return -1;
}
int launch_zero(int *, int, hipStream_t) { return -1; }
int launch_merge(const PairDesc *, const PairDesc *, int, const unsigned long long *,
                 const unsigned long long *, int, sncc_match *, hipStream_t) {
  return -1;
}
int launch_map_topk64(const double *, int, int, int, int, int, Key96 *, hipStream_t) {
  return -1;
}
int launch_merge64(const PairDesc *, int, const Key96 *, int, sncc_match *, hipStream_t) {
  return -1;
}
int launch_refine(const uint32_t *, const uint32_t *, long long, int, const DevTmpl *,
                  const int4 *, const double *, const SlotTables &, const PairDesc *, int,
                  const sncc_match *, int, int, sncc_match64 *, int *, hipStream_t) {
  return -1;
}

}  // namespace sncc

using namespace sncc;

static int g_fail = 0;
static long long g_banded = 0;  // passes of column bands after the first
#define CHECK(cond, ...)                                  \
  do {                                                    \
    if (!(cond)) {                                        \
      if (g_fail < 20) {                                  \
        std::fprintf(stderr, "check failed: %s: ", #cond); \
        std::fprintf(stderr, __VA_ARGS__);                \
        std::fprintf(stderr, "\n");                       \
      }                                                   \
      ++g_fail;                                           \
    }                                                     \
  } while (0)

static std::vector<uint8_t> random_template(std::mt19937_64 &rng, int W, int H) {
  std::vector<uint8_t> t((size_t)W * H);
  const int kind = (int)(rng() % 4);
  const int lv = 2 + (int)(rng() % 4);
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int v;
      switch (kind) {
        case 0: v = (int)(rng() % 256); break;                        // noise
        case 1: v = (int)(rng() % lv) * (255 / lv); break;            // few levels
        case 2: v = 3 * x + 2 * y + (int)(rng() % 5); break;          // ramp
        default: v = ((x / 3 + y / 2) % lv) * 60 + (int)(rng() % 2);  // blocks
      }
      t[(size_t)y * W + x] = (uint8_t)std::min(255, std::max(0, v));
    }
  return t;
}

static void check_segmentation(std::mt19937_64 &rng, int W, int H) {
  const std::vector<uint8_t> t = random_template(rng, W, H);
  const double sigmas[] = {0.0, 0.5, 1.0, 2.75, 4.0, 8.0, 16.0, 40.0, 1e9};
  const double sigma = sigmas[rng() % 9];
  const int kmaxes[] = {1, 3, 20, 5000};
  const int K_max = kmaxes[rng() % 4];
  std::vector<Seg> segs;
  int kb = 0;
  double used = 0, rho = 0;
  const int rc = segment_template(t.data(), W, H, W, sigma, K_max, segs, &kb, &used, &rho);
  CHECK(rc == SNCC_OK || rc == SNCC_EDEGENERATE, "status %d", rc);
  CHECK(kb <= K_max || sigma != sigma, "%d leaves > K_max %d", kb, K_max);
  CHECK((int)segs.size() <= kb, "%zu merged > %d leaves", segs.size(), kb);
  std::vector<int> cover((size_t)W * H, 0);
  for (const Seg &g : segs) {
    CHECK(g.w >= 1 && g.h >= 1 && g.x >= 0 && g.y >= 0 && g.x + g.w <= W && g.y + g.h <= H,
          "segment (%d,%d,%d,%d) outside %dx%d", g.x, g.y, g.w, g.h, W, H);
    if (!(g.x >= 0 && g.y >= 0 && g.x + g.w <= W && g.y + g.h <= H)) continue;
    int64_t sum = 0;
    for (int y = g.y; y < g.y + g.h; ++y)
      for (int x = g.x; x < g.x + g.w; ++x) {
        ++cover[(size_t)y * W + x];
        sum += t[(size_t)y * W + x];
      }
    CHECK(sum == g.sum && g.area == (int64_t)g.w * g.h, "segment sum %lld vs %lld",
          (long long)g.sum, (long long)sum);
  }
  for (int c : cover) CHECK(c == 1, "pixel covered %d times", c);
  for (size_t i = 0; i < segs.size(); ++i)
    for (size_t j = 0; j < segs.size(); ++j) {
      const Seg &a = segs[i], &b = segs[j];
      if (i == j || (__int128)a.sum * b.area != (__int128)b.sum * a.area) continue;
      CHECK(!(a.x == b.x && a.w == b.w && a.y + a.h == b.y), "vertical pair left unmerged");
      CHECK(!(a.y == b.y && a.h == b.h && a.x + a.w == b.x), "horizontal pair left unmerged");
    }
}

// A template set of T random templates with sides up to max_side.
static bool make_set(std::mt19937_64 &rng, int T, int max_side, sncc_tmpl &tm) {
  std::vector<std::vector<sncc_segment>> lists(T);
  std::vector<const sncc_segment *> ptr(T);
  std::vector<int> K(T), Ws(T), Hs(T);
  for (int t = 0; t < T; ++t) {
    int rc;
    std::vector<Seg> segs;
    do {
      Ws[t] = 1 + (int)(rng() % max_side);
      Hs[t] = 1 + (int)(rng() % max_side);
      const std::vector<uint8_t> img = random_template(rng, Ws[t], Hs[t]);
      const double sigmas[] = {2.0, 4.0, 8.0, 16.0};
      int kb;
      double u, r;
      rc = segment_template(img.data(), Ws[t], Hs[t], Ws[t], sigmas[rng() % 4], 5000, segs, &kb,
                            &u, &r);
    } while (rc != SNCC_OK);
    for (const Seg &g : segs)
      lists[t].push_back(sncc_segment{g.x, g.y, g.w, g.h, g.sum, (int32_t)g.area, 0});
    ptr[t] = lists[t].data();
    K[t] = (int)segs.size();
  }
  std::vector<int4> geom;
  std::vector<double> c64;
  std::vector<int> areas;
  tm.T = T;
  return fill_templates(&tm, T, ptr.data(), K.data(), Ws.data(), Hs.data(), geom, c64,
                        areas) == SNCC_OK;
}

static void check_plan(const sncc_tmpl &tm, const PlanHost &ph, int n_pairs, int split) {
  const TileCfg &tc = ph.tc;
  CHECK(ph.lds_bytes >= 0 && ph.lds_bytes <= kTileMaxLds, "lds %d", ph.lds_bytes);
  // work items: each pair's tiles once, in order
  for (int p = 0; p < n_pairs; ++p) {
    const PairDesc &pd = ph.pairs[p];
    int next = 0;
    for (int i = pd.item_begin; i < pd.item_end; ++i) {
      const WorkItem &it = ph.items[i];
      CHECK(it.pair == p && it.tile_begin == next && it.tile_end > it.tile_begin,
            "item %d of pair %d: tiles %d..%d, expected from %d", i, p, it.tile_begin,
            it.tile_end, next);
      next = it.tile_end;
    }
    CHECK(next == pd.ntu * pd.ntv, "pair %d covers %d of %d tiles", p, next, pd.ntu * pd.ntv);
    if (split != kSplitEdge) CHECK(pd.ntu * tc.bu() + 0 >= 0, "ntu");
  }
  std::vector<int> seen(ph.items.size(), 0);
  for (int i : ph.order) {
    CHECK(i >= 0 && i < (int)ph.items.size(), "order entry %d", i);
    if (i >= 0 && i < (int)ph.items.size()) ++seen[i];
  }
  for (int c : seen) CHECK(c == 1, "item queued %d times", c);
  CHECK(!ph.qbeg.empty() && ph.qbeg.front() == 0 && ph.qbeg.back() == (int)ph.order.size(),
        "queue offsets");
  for (size_t q = 1; q < ph.qbeg.size(); ++q) CHECK(ph.qbeg[q] >= ph.qbeg[q - 1], "queues");
  // launch grid: at most one workgroup per item; with exactly one per item
  // the kernel takes no queue and workgroup b runs order[b]
  CHECK(ph.grid >= 1 && (ph.items.empty() || ph.grid <= (int)ph.items.size()),
        "grid %d for %zu items", ph.grid, ph.items.size());
  if (ph.grid == (int)ph.items.size())
    CHECK(ph.order.size() == ph.items.size(), "one item per workgroup: order holds %zu of %zu",
          ph.order.size(), ph.items.size());
  // LDS reads of the staged records
  const int scale_words = 64 * tc.nw * tc.ru * tc.rv;
  for (int t = 0; t < tm.T; ++t) {
    const DevTmpl &d = ph.tmpls[t];
    if (d.pass_end <= d.pass_begin || d.lp_class >= kNumLpClasses) continue;
    const int LP = kLpClasses[d.lp_class];
    const long long lane_max = (long long)(tc.nw - 1) * tc.rv * LP + 63 +
                               (long long)(tc.rv - 1) * LP + (long long)(tc.ru - 1) * 64;
    for (int p = d.pass_begin; p < d.pass_end; ++p) {
      const PassDesc &ps = ph.passes[p];
      CHECK(ps.seg_begin >= 0 && ps.seg_end <= (int)ph.recs.size() && ps.seg_begin <= ps.seg_end,
            "pass records %d..%d of %zu", ps.seg_begin, ps.seg_end, ph.recs.size());
      CHECK(ps.iv_begin >= 0 && ps.iv_end <= (int)ph.ivs.size(), "pass intervals");
      CHECK(ps.col0 >= 0 && ps.col0 % 4 == 0 && ps.col0 < tm.W[t], "band start %d", ps.col0);
      g_banded += ps.col0 > 0;
      CHECK(ps.stage_w4 * 4 <= LP && ps.stage_w4 * 4 >= tc.bu() + 1 &&
                ps.col0 + ps.stage_w4 * 4 >= std::min(tm.W[t], ps.col0 + 1),
            "staged width %d words at pitch %d", ps.stage_w4 * 4, LP);
      int rows = 0;
      for (int iv = ps.iv_begin; iv < ps.iv_end && iv < (int)ph.ivs.size(); ++iv)
        rows = std::max(rows, ph.ivs[iv].lds_row + ph.ivs[iv].n_rows);
      CHECK((long long)scale_words + (long long)rows * LP <= ph.lds_bytes / 4,
            "template %d pass %d stages %d rows of %d words beyond %d bytes", t, p, rows, LP,
            ph.lds_bytes);
      for (int r = ps.seg_begin; r < ps.seg_end && r < (int)ph.recs.size(); ++r) {
        const TileRec &e = ph.recs[r];
        const long long hi = (long long)std::max(e.off_tl, e.off_bl) + lane_max;
        CHECK(e.off_tl >= 0 && e.off_bl >= 0 && hi < (long long)rows * LP,
              "record %d: offsets %d %d (+%lld) beyond %d rows of %d words", r, e.off_tl,
              e.off_bl, lane_max, rows, LP);
      }
    }
  }
}

// Slot tables: every slot inside its template's region, and the weighted
// corner entries equal the segment sums.  For a random image g at the
// region's origin, with each table row and each column shifted by a random
// constant and then made relative to the first row and column as the kernels
// do, the sum over slots of W s(corner) must equal the sum over segments of
// c_i times the box sum of g (summation by parts in both directions), to
// FP64 rounding.
static void check_slots(const sncc_tmpl &tm, const PlanHost &ph) {
  uint64_t lcg = 0x9e3779b97f4a7c15ull;
  auto next = [&]() { return (uint32_t)((lcg = lcg * 6364136223846793005ull + 1442695040888963407ull) >> 33); };
  for (int t = 0; t < tm.T; ++t) {
    const SlowTmpl &st = ph.slow[t];
    if (st.tbl < 0) continue;
    const long long region = (long long)st.pitch * st.rows * 4;
    CHECK(region <= (long long)ph.slow_lds, "region %lld > %d", region, ph.slow_lds);
    bool inside = true;
    for (int i = st.tbl; i < st.tbl + 64 * st.n_iter; ++i) {
      CHECK(i < (int)ph.slot_off.size(), "slot %d beyond the table", i);
      if (i >= (int)ph.slot_off.size()) return;
      const uint32_t o = ph.slot_off[i];
      const long long top = o & 0xffffu, bot = o >> 16;
      CHECK(top < region && bot < region, "slot %d: %lld %lld of %lld", i, top, bot, region);
      inside = inside && top < region && bot < region && top % 4 == 0 && bot % 4 == 0;
    }
    if (!inside) continue;
    const int P = st.pitch, R = st.rows;
    std::vector<uint32_t> g((size_t)R * P), tab((size_t)R * P);
    for (uint32_t &v : g) v = next() & 0xffu;
    for (int r = 1; r < R; ++r)  // tab[r][c]: sum of g over rows < r and columns < c
      for (int c = 1; c < P; ++c)
        tab[(size_t)r * P + c] = tab[(size_t)(r - 1) * P + c] + tab[(size_t)r * P + c - 1] -
                                 tab[(size_t)(r - 1) * P + c - 1] + g[(size_t)(r - 1) * P + c - 1];
    std::vector<uint32_t> col_shift(P);
    for (uint32_t &v : col_shift) v = next();
    for (int r = 0; r < R; ++r) {  // shifts of rows and columns
      const uint32_t shift = next();
      for (int c = 0; c < P; ++c) tab[(size_t)r * P + c] += shift + col_shift[c];
    }
    std::vector<uint32_t> rel(tab.size());  // the kernels' relative form
    for (int r = 0; r < R; ++r)
      for (int c = 0; c < P; ++c)
        rel[(size_t)r * P + c] =
            tab[(size_t)r * P + c] - tab[(size_t)r * P] - tab[c] + tab[0];
    double by_slots = 0.0, by_segs = 0.0, scale = 0.0;
    for (int i = st.tbl; i < st.tbl + 64 * st.n_iter; ++i) {
      const uint32_t o = ph.slot_off[i];
      CHECK((o >> 16) == 0, "slot %d: high half %u", i, o >> 16);
      by_slots += ph.slot_w[i] * (double)rel[(o & 0xffffu) / 4];
    }
    const std::vector<Seg> &segs = tm.segs[t];
    for (size_t i = 0; i < segs.size(); ++i) {
      const Seg &q = segs[i];
      int64_t F = 0;
      for (int y = q.y; y < q.y + q.h; ++y)
        for (int x = q.x; x < q.x + q.w; ++x) F += g[(size_t)y * P + x];
      by_segs += tm.c64[t][i] * (double)F;
      scale += std::fabs(tm.c64[t][i] * (double)F);
    }
    CHECK(std::fabs(by_slots - by_segs) <= 1e-9 * (scale + 1.0),
          "template %d: slots give %.17g, segments %.17g", t, by_slots, by_segs);
  }
}

// Refine launch classes: the order is a permutation of the pairs, the first
// refine_n_first pairs have regions within refine_lds_first, which is within
// the four-per-CU budget, and the others' regions exceed that budget.
static void check_refine_order(PlanHost &ph, int n_cand, int radius) {
  plan_refine_order(ph, n_cand, radius);
  const int n = (int)ph.pairs.size();
  CHECK((int)ph.refine_order.size() == n, "refine order holds %zu of %d pairs",
        ph.refine_order.size(), n);
  std::vector<char> seen(n, 0);
  int np = 1;
  while (np < n_cand * (2 * radius + 1) * (2 * radius + 1)) np <<= 1;
  const int budget = refine_region_budget(np, 4);
  CHECK(ph.refine_lds_first <= budget, "first class region %d > budget %d",
        ph.refine_lds_first, budget);
  for (int i = 0; i < (int)ph.refine_order.size(); ++i) {
    const int p = ph.refine_order[i];
    CHECK(p >= 0 && p < n && !seen[p], "refine order entry %d: pair %d", i, p);
    if (p < 0 || p >= n || seen[p]) continue;
    seen[p] = 1;
    const SlowTmpl &st = ph.slow[ph.pairs[p].tmpl];
    const int region = st.tbl >= 0 ? st.pitch * st.rows * 4 : 0;
    if (i < ph.refine_n_first)
      CHECK(region <= ph.refine_lds_first, "pair %d region %d above %d", p, region,
            ph.refine_lds_first);
    else
      CHECK(region > budget, "pair %d region %d in the second class within %d", p, region,
            budget);
  }
}

int main(int argc, char **argv) {
  const int iters = argc > 1 ? std::atoi(argv[1]) : 2000;
  std::mt19937_64 rng(argc > 2 ? std::strtoull(argv[2], nullptr, 10) : 1);
  int n_seg = 0, n_plan = 0;
  for (int i = 0; i < iters; ++i) {
    const bool big = i % 200 == 0;
    check_segmentation(rng, 1 + (int)(rng() % (big ? 160 : 48)),
                       1 + (int)(rng() % (big ? 160 : 48)));
    ++n_seg;
  }
  for (int i = 0; i < std::max(1, iters / 40); ++i) {
    sncc_tmpl tm;
    const int T = 1 + (int)(rng() % 5);
    if (!make_set(rng, T, i % 5 == 0 ? 400 : i % 7 == 0 ? 1100 : 100, tm)) {
      CHECK(false, "fill_templates failed");
      continue;
    }
    int maxW = 1, maxH = 1;
    for (int t = 0; t < T; ++t) maxW = std::max(maxW, tm.W[t]), maxH = std::max(maxH, tm.H[t]);
    const int M = maxW + (int)(rng() % 300), N = maxH + (int)(rng() % 200);
    int P = 0;
    sncc_sat_pitch(M, &P);
    const int B = 1 + (int)(rng() % 3);
    std::vector<int32_t> pairs;
    for (int b = 0; b < B; ++b)
      for (int t = 0; t < T; ++t) {
        pairs.push_back(b);
        pairs.push_back(t);
      }
    const int n_pairs = (int)pairs.size() / 2;
    std::vector<double> thr(T, 0.5);
    for (int cfg = 0; cfg < kNumCfgs; ++cfg) {
      const int k = 1 + (int)(rng() % 64);
      const int sinks[] = {kSinkTopk, kSinkMap, kSinkCompact};
      for (int sink : sinks) {
        const int np = sink == kSinkMap ? 1 : n_pairs;
        PlanHost ph;
        const int rc = build_plan(&tm, cfg, M, N, P, np, pairs.data(), k, sink, 256, ph,
                                  sink == kSinkCompact ? thr.data() : nullptr);
        CHECK(rc == SNCC_OK, "build_plan cfg %d sink %d: %d", cfg, sink, rc);
        if (rc != SNCC_OK) continue;
        check_plan(tm, ph, np, kSplitNone);
        if (sink == kSinkCompact) {
          plan_slow(&tm, ph.tc, ph);
          check_slots(tm, ph);
        }
        ++n_plan;
      }
      // the batches' two launches: main tiles without the narrow last column,
      // then that column alone in half-width tiles
      const TileCfg tc = tile_cfg_of(cfg);
      PlanHost main_ph, edge_ph;
      CHECK(build_plan(&tm, cfg, M, N, P, n_pairs, pairs.data(), k, kSinkTopk, 256, main_ph,
                       nullptr, kSplitMain) == SNCC_OK, "main plan");
      check_plan(tm, main_ph, n_pairs, kSplitMain);
      for (int e = 0; e < kNumCfgs; ++e) {
        const TileCfg ec = tile_cfg_of(e);
        if (ec.ru != 1 || ec.rv != tc.rv || ec.nw != tc.nw || tc.ru != 2) continue;
        CHECK(build_plan(&tm, e, M, N, P, n_pairs, pairs.data(), k, kSinkTopk, 256, edge_ph,
                         nullptr, kSplitEdge, tc.bu()) == SNCC_OK, "edge plan");
        check_plan(tm, edge_ph, n_pairs, kSplitEdge);
        plan_slots(&tm, kRefineWideSpanU, kRefineWideSpanV, kRefineRegionWords, edge_ph,
                   kRefineSpanU, kRefineSpanV);
        check_slots(tm, edge_ph);
        check_refine_order(edge_ph, 1 + (int)(rng() % 64), (int)(rng() % 3));
        ++n_plan;
      }
    }
  }
  std::printf("host checks: %d segmentations, %d plans (%lld passes of later column bands), "
              "%d failures\n", n_seg, n_plan, g_banded, g_fail);
  return g_fail == 0 ? 0 : 1;
}
