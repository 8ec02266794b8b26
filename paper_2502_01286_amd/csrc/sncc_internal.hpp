// Internal structures shared by the host planner and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/sncc.h"

namespace sncc {

// ---------------------------------------------------------------- host side
struct Seg {
  int x, y, w, h;
  int64_t sum;
  int64_t area;
};

bool std_below(int64_t S, int64_t S2, int64_t A, double sigma);
void merge_segments(std::vector<Seg> &k, int W, int H);
int segment_template(const uint8_t *t, int W, int H, int stride, double sigma,
                     int K_max, std::vector<Seg> &out, int *k_before_merge,
                     double *sigma_used, double *rho_max);

void set_error(const char *fmt, ...);

// ------------------------------------------------- device-visible records
// Per template constants (Section 5, steps 3-4).
struct DevTmpl {
  int W, H, K, n;      // n = W * H
  double q_k;          // sum_i A_i c_i^2 (area-weighted Eq. (17))
  double r64;          // sum_i A_i c_i in FP64 (zero up to rounding)
  int seg_off;         // first segment in the generic arrays
  int lp_class;        // LDS pitch class of the tile kernel
  int pass_begin;      // tile plan: passes of this template
  int pass_end;
  float thr;           // survivor threshold of the compacting sink
  int sq_rows;         // rows per band of the f^2 window sum (>= H: one box)
};

// Largest box whose sum of f^2 stays below 2^32 (255^2 * 66051 < 2^32): larger
// windows take their f^2 sum band by band (sq_rows rows of W pixels each).
constexpr int kMaxSqBoxArea = 66051;

// One boundary column of a horizontal chain for the staged tile kernel: LDS
// dword offsets (relative to the lane's base) of the column's entries in the
// chain's top row y and bottom row y + h, and A_i, c_i of the segment that
// ends at this column (0, 0 for the chain's first column).  The segment's box
// sum (Eq. (11)) is the difference of the column differences of its right
// and left boundaries.
struct TileRec {
  int off_tl;
  int off_bl;
  int w_area;  // A_i (staged form); see DirectRec for the direct form
  float c;
};

// One boundary column of a horizontal chain for the tile kernel's direct
// form (entries read from the global table, no LDS): byte offsets of the
// column's entries in the chain's top and bottom rows relative to the
// window's top-left entry, and A_i, c_i of the segment ending at this column
// (0, 0 for the chain's first column).  Two TileRec slots.
struct DirectRec {
  int top, bot, area;
  float c;
  int pad[4];
};

// Rows [rel_row, rel_row + n_rows) of the window (template-relative,
// zero-padded table coordinates) staged to LDS rows starting at lds_row.
struct Interval {
  int rel_row, n_rows, lds_row, pad;
};

// A staged pass: its row intervals, its column window and its records.  A
// template too wide for one LDS row is split into column bands (segments cut
// at band edges; a box sum is the sum of its pieces' box sums), each staged
// by passes of its own.  The records form
// horizontal chains (segments with equal y and h, each starting where the
// previous one ends); a chain of L segments has L + 1 records, one per
// boundary column.  Chains are grouped by length: n_chain[L - 1] chains of
// length L = 4, 3, 2, 1 in that order.  (The direct form uses seg_begin,
// seg_end only.)
struct PassDesc {
  int seg_begin, seg_end;  // TileRec range
  int iv_begin, iv_end;    // Interval range
  int n_chain[4];          // chains of length 1, 2, 3, 4
  int col0;                // first template column of the staged window (a
                           // multiple of 4; 0 unless the template is split
                           // into column bands)
  int stage_w4;            // 16-byte chunks staged per row
  int pad[2];
};

constexpr int kMaxChain = 4;  // longer chains are cut into pieces

struct PairDesc {
  int frame, tmpl;
  int nu, nv;              // offsets along u and v
  int ntu, ntv;            // tiles along u and v
  int item_begin, item_end;
  int u_base;              // column of the first tile column (nonzero for the
                           // narrow last column a second launch scores)
};

struct WorkItem {
  int pair;
  int tile_begin, tile_end;
  int pad;
};

// Sinks of the persistent tile kernel: per-item top-k partials, a rho map,
// or a compacted list of the offsets whose rho reaches a threshold.
constexpr int kSinkTopk = 0;
constexpr int kSinkMap = 1;
constexpr int kSinkCompact = 2;

// A run of the survivor list: the survivors one wave found in one group of
// kRunCols columns of a tile, written together at hits[start, start + count)
// (entries at or beyond the list's capacity were not written).  They lie in
// offset rows [v0, v0 + RV) and columns [u0, u0 + kRunCols) of pair `pair`.
constexpr int kRunCols = 32;
struct RunDesc {
  int start, count, pair, u0, v0;
  int pad[3];
};

struct CompactOut {
  sncc_hit *hits;  // cap entries
  int cap;
  int *count;      // entries wanted (may exceed cap; zero at launch)
  RunDesc *runs;   // run_cap entries, one per (tile, wave) with survivors
  int run_cap;
  int *run_count;  // zero at launch
};

// Slow pass of the two-threshold search.  A template whose region (the
// table rows and columns that the windows of one run's offsets cover) fits
// the LDS budget is scored from LDS through a corner-slot table.  By
// summation by parts in both directions, the sum over segments of c_i times
// the box sum F_i (Eq. (11)) equals the sum over the template's distinct
// rectangle corners p of W_p s(p), where s is the sum table at the corner
// (relative to the window's top-left entry) and W_p collects +c_i for the
// top-left and bottom-right corners of segment i and -c_i for the other two.
// The weights add to zero along every row and every column of corners, so s
// may be taken from a table shifted by a constant per row and per column,
// such as the staged region made relative to its first row and column.
// Slot j holds the corner's LDS byte offset (low 16 bits) and W_j; the
// slots are padded to whole waves (offset 0, weight 0).
struct SlowTmpl {
  int tbl;     // first slot (-1: scored from the global tables)
  int n_iter;  // slots / 64
  int pitch;   // LDS row pitch (words) of the region
  int rows;    // region rows
};

// Region of a run: rows [v0, v0 + RV + H), columns [u0, u0 + kRunCols + W]
// of the frame's table; at most this many words.
constexpr int kSlowRegionWords = 13312;  // 52 KB
static_assert(kSlowRegionWords * 4 <= 65536, "slot byte offsets are 16-bit");

// The refine kernel scores its offsets in chunks: a chunk whose offsets span
// at most span_u columns and span_v rows is scored from a staged region like
// the slow pass's, of (span_v + H) rows of span_u + W + 1 words.  The spans
// are the wide ones when that region fits kRefineRegionWords (fewer, larger
// chunks: less of the table is staged per offset), else the narrow ones.
constexpr int kRefineSpanU = 16, kRefineSpanV = 8;
constexpr int kRefineWideSpanU = 32, kRefineWideSpanV = 16;
constexpr int kRefineRegionWords = 12032;  // 47 KB beside the 16 KB offset list and 1 KB of sums
static_assert(kRefineRegionWords * 4 <= 65536, "slot byte offsets are 16-bit");

// Device view of a template set's slot tables.
struct SlotTables {
  const SlowTmpl *tmpl;
  const uint32_t *off;
  const double *w;
  int lds_bytes;  // largest region of a staged template (0: none)
  // refine launch classes (optional): the pairs in order[0 .. n_first) have
  // regions of at most lds_first bytes and run in a launch of their own,
  // which fits more workgroups per CU; order[n_first ..) run in a second one
  const int *order;
  int n_first;
  int lds_first;
};

struct SlowArgs {
  const uint32_t *s;
  const uint32_t *s2;
  long long frame_stride;
  int P, N;
  const DevTmpl *tmpls;     // slow approximations
  const int4 *geom;
  const double *c64;
  const SlowTmpl *stmpl;
  const uint32_t *slot_off;
  const double *slot_w;
  const PairDesc *pairs;
  const double *thr;        // per template
  const sncc_hit *cand;
  const int *cand_count;
  int cand_cap;
  const RunDesc *runs;
  const int *run_count;
  int run_cap;
  int *work;                // run counter, zero at launch
  sncc_hit *out;
  int out_cap;
  int *out_count;
};

// Kernel arguments of the persistent tile kernel.
struct TileArgs {
  const uint32_t *s;
  const uint32_t *s2;
  long long frame_stride;  // elements between frames of the sum tables
  int sat_pitch;
  int M, N;
  const DevTmpl *tmpls;
  const PassDesc *passes;
  const Interval *ivs;
  const TileRec *recs;
  const PairDesc *pairs;
  const WorkItem *items;
  const int *order;        // execution order of items, queue by queue
  const int *qbeg;         // nq + 1 offsets into order
  int nq;                  // work queues (1..kMaxQueues; 0: one workgroup per item)
  int n_items;
  int *queue;              // counters at queue[16 j], then (TOPK sink) the
                           // pair floors; kQueueInts + 2 n_pairs ints zeroed
                           // at launch
  int k;                   // top-k (TOPK sink)
  unsigned long long *partial;  // n_items x k keys (TOPK sink)
  unsigned long long *pair_floor;  // n_pairs keys, zero at launch (TOPK sink)
  void *rho;               // MAP sink: float map
  int rho_pitch;
  uint8_t *degen;          // MAP sink: nullable
  CompactOut co;           // compacting sink
  int n_zero;              // ints of `queue` to zero before a launch (host side)
};

// Kernel arguments of the plain FP64 per-pair kernel.
struct PlainArgs {
  const uint32_t *s;
  const uint32_t *s2;
  int sat_pitch;
  int nu, nv;
  int W, H, K;
  int sq_rows;             // rows per band of the f^2 window sum
  double q_k, r64;
  const int4 *geom;        // x, y, w, h
  const double *c64;
  const int *area;
  double *rho;
  int rho_pitch;
  uint8_t *degen;
};

// Tile-local form (fused_kernel.hip): one frame, one template, sum tables
// built per tile in LDS from the frame.
struct FusedArgs {
  const uint8_t *f;
  int M, N, f_pitch;
  int W, H, K, nu, nv;
  const int4 *geom;        // x, y, w, h
  const int *area;
  const float *c32;        // c_i rounded to FP32
  double q_k;
  float *rho;
  int rho_pitch;
  uint8_t *degen;
  long long *energy;
};
constexpr int kFusedMaxLds = 160 * 1024 - 64;
constexpr int kFusedRV = 4;                    // offset rows per lane
constexpr int kFusedNW = 4;                    // waves per workgroup
constexpr int kFusedBU = 64;                   // offset columns per tile
constexpr int kFusedBV = kFusedRV * kFusedNW;  // offset rows per tile

// Tile kernel configuration: offsets per lane RU (u, stride 64) x RV (v),
// NW waves per workgroup, each wave owning RV offset rows; `wgs` is the
// number of workgroups per CU the LDS budget is sized for; with
// `frame_major`, work items run frame by frame (largest first within a
// frame) so that concurrent workgroups share a frame's sum tables in cache,
// otherwise largest first overall.
struct TileCfg {
  int ru, rv, nw, wgs, frame_major;
  int bu() const { return 64 * ru; }
  int bv() const { return nw * rv; }
  int threads() const { return 64 * nw; }
};

constexpr int kMaxQueues = 8;  // one per XCD of an MI355X
constexpr int kQueueInts = 16 * kMaxQueues;

// LDS row pitches (words) the scoring kernel is compiled for; a template
// uses the smallest one that holds a tile's staged row (tile width + W + 1,
// rounded up to 16 bytes).
constexpr int kNumLpClasses = 11;
constexpr int kLpClasses[kNumLpClasses] = {128, 160, 192, 224, 256, 288, 320, 384, 448, 512, 576};
// lp_class of a template scored in the direct form
constexpr int kLpDirect = kNumLpClasses;

// Tile shapes of the scoring kernel: offsets per lane along u (RU) and v
// (RV) and waves per workgroup (NW); a tile is 64 RU x NW RV offsets.
constexpr int kNumTileShapes = 6;
constexpr int kTileShapes[kNumTileShapes][3] = {
    {2, 4, 8},  // 128 x 32
    {2, 4, 4},  // 128 x 16
    {1, 8, 8},  //  64 x 64
    {2, 2, 8},  // 128 x 16
    {1, 4, 8},  //  64 x 32
    {1, 4, 4},  //  64 x 16
};
// Tile configurations the planner and the tuner choose from: tile shape
// (index into kTileShapes), workgroups per CU the LDS budget is sized for,
// and the work order (frame-major queues per XCD, or one queue).
struct CfgEntry {
  int entry, wgs, frame_major;
};
constexpr CfgEntry kCfgs[] = {
    {0, 2, 1}, {0, 2, 0}, {1, 4, 1}, {3, 2, 1}, {3, 3, 1}, {4, 2, 1}, {5, 4, 1}, {2, 2, 1},
};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);
constexpr int kTileMaxLds = 160 * 1024;  // LDS of one CU (gfx950)
inline TileCfg tile_cfg_of(int i) {
  const int e = kCfgs[i].entry;
  return TileCfg{kTileShapes[e][0], kTileShapes[e][1], kTileShapes[e][2], kCfgs[i].wgs,
                 kCfgs[i].frame_major};
}

// Host stubs of tile shape i's kernels (tile_entry.hip), one per sink.
const void *tile_fn_0(int sink);
const void *tile_fn_1(int sink);
const void *tile_fn_2(int sink);
const void *tile_fn_3(int sink);
const void *tile_fn_4(int sink);
const void *tile_fn_5(int sink);

// Launch wrappers (kernels.hip).
int launch_sat(const uint8_t *f, int B, int M, int N, int f_pitch, uint32_t *s,
               uint32_t *s2, int sat_pitch, uint32_t *scratch, hipStream_t st);
size_t sat_scratch_words(int B, int M, int N);
// Device address of the static carry scratch of the allocation-free sum-table
// entry point: looked up once per device (that device current) by
// sat_noalloc_init, nullptr before.
int sat_noalloc_init(int device);
uint32_t *sat_noalloc_addr(int device);

int tile_cfg_count();
TileCfg tile_cfg(int i);
int launch_slow(const SlowArgs &a, int grid, int lds_bytes, hipStream_t st);
int slow_occupancy(int lds_bytes);
int launch_tile(int cfg, int sink, const TileArgs &a, int grid,
                int lds_bytes, hipStream_t st);
int tile_max_lds();
int tile_occupancy(int cfg, int sink, int lds_bytes);
int launch_plain(const PlainArgs &a, hipStream_t st);
// LDS row pitch (words) of the tile-local form for templates W wide: the
// smallest pitch class holding the region's 64 + W + 1 table columns (0: none).
inline int fused_lp(int W) {
  for (int i = 0; i < kNumLpClasses; ++i)
    if (kLpClasses[i] >= kFusedBU + W + 1) return kLpClasses[i];
  return 0;
}
// LDS bytes of the tile-local form's region table: 16 + H + 1 rows.
inline size_t fused_lds_bytes(int W, int H) {
  const int LP = fused_lp(W);
  return LP ? (size_t)(kFusedBV + H + 1) * LP * 4 : 0;
}
int launch_fused(const FusedArgs &a, hipStream_t st);
int launch_energy(const uint32_t *s, const uint32_t *s2, int P, int nu, int nv, int W, int H,
                  int sq_rows, long long *energy, int pitch, hipStream_t st);
int launch_zero(int *p, int n, hipStream_t st);
int launch_merge(const PairDesc *pairs, const PairDesc *pairs2, int n_pairs,
                 const unsigned long long *partial, const unsigned long long *partial2,
                 int k, sncc_match *out, hipStream_t st);
// Exact selection key of an FP64 value: order code of the double, then the
// complement of the index (ties to the smaller index).
struct Key96 {
  unsigned long long hi;
  uint32_t lo;
  uint32_t pad;
};
int launch_map_topk64(const double *map, int pitch, int nu, int nv, int chunk, int k,
                      Key96 *partial, hipStream_t st);
int launch_merge64(const PairDesc *pairs, int n_pairs, const Key96 *partial, int k,
                   sncc_match *out, hipStream_t st);
// Region bytes that leave room for `wgs` refine workgroups per CU when the
// offset list holds np entries (0 when none fit).
int refine_region_budget(int np, int wgs);
int launch_refine(const uint32_t *s, const uint32_t *s2, long long frame_stride,
                  int sat_pitch, const DevTmpl *tmpls, const int4 *geom,
                  const double *c64, const SlotTables &slots, const PairDesc *pairs,
                  int n_pairs, const sncc_match *cand, int n_cand, int radius,
                  sncc_match64 *out, int *count, hipStream_t st);

}  // namespace sncc
