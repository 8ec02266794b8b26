// HIP kernels for segmented NCC on gfx950 (CDNA4, wave64).
//
//  * Sum tables (Eqs. (10), (14)): two launches.  Per 64 x 256 tile,
//    sat_totals writes column totals, row totals and the tile total;
//    sat_scan sums from them the carries its tile needs (the rows above per
//    column, the columns to the left per row, the tiles above-left), then
//    rebuilds the tile with running column sums and one wavefront scan per
//    row and writes s and s^2.  f is read twice, s and s^2 written once:
//    about 10 bytes of HBM traffic per pixel.
//  * Scoring (Eqs. (11)-(18)): a persistent kernel pulls work items
//    (pair, range of offset tiles) from an atomic counter.  For each tile the
//    rows of the sum table that the template's corner rows touch are staged
//    in LDS; every lane then owns RU x RV offsets, streams the segment list
//    (wave-uniform scalar loads) and forms each box sum from four LDS reads in
//    32-bit modular arithmetic (exact), subtracts area x (window mean rounded
//    to an integer) in integers and accumulates the product with c_i in FP32
//    with Kahan compensation.  The window energy is exact in 64-bit integers;
//    rho is formed in FP32.  Results go either to a map or to a per-wave
//    register-resident top-k list.
//  * Plain FP64 kernel: one thread per offset, segments from global memory,
//    FP64 accumulation; used for the FP64 map, the per-pair baseline and the
//    fine re-scoring.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "device_util.hpp"

namespace sncc {

// ---------------------------------------------------------------- sum tables
constexpr int SAT_TY = 64;
constexpr int SAT_TX = 256;

struct SatScratch {
  uint32_t *colT, *rowT, *T;
  int nTX, nTY;
};

__host__ __device__ inline SatScratch sat_layout(uint32_t *base, int B, int M, int N) {
  SatScratch sc;
  sc.nTX = (M + SAT_TX - 1) / SAT_TX;
  sc.nTY = (N + SAT_TY - 1) / SAT_TY;
  sc.colT = base;                                          // [2][B][nTY][M]
  sc.rowT = sc.colT + (size_t)2 * B * sc.nTY * M;          // [2][B][nTX][N]
  sc.T = sc.rowT + (size_t)2 * B * N * sc.nTX;             // [2][B][nTY][nTX]
  return sc;
}

size_t sat_scratch_words(int B, int M, int N) {
  size_t nTX = (M + SAT_TX - 1) / SAT_TX, nTY = (N + SAT_TY - 1) / SAT_TY;
  return (size_t)2 * B * (nTY * (size_t)M + (size_t)N * nTX + nTY * nTX);
}

// Pixels x0 .. x0 + 3 of a row packed into one word (byte q = pixel x0 + q,
// 0 beyond M): one 32-bit load when all four are inside the row and the
// address is 4-byte aligned, else byte loads.
__device__ __forceinline__ uint32_t load_pk4(const uint8_t *row, int x0, int M) {
  if (x0 + 3 < M && ((reinterpret_cast<uintptr_t>(row + x0) & 3) == 0))
    return *reinterpret_cast<const uint32_t *>(row + x0);
  uint32_t w = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (x0 + q < M) w |= (uint32_t)row[x0 + q] << (8 * q);
  return w;
}

// Table columns x0 .. x0 + 3 of a row (x0 a multiple of 4, the row 256-byte
// aligned): one aligned 16-byte store when all four are columns 0 .. M, else
// dword stores of the columns below the pitch P, 0 past column M.
__device__ __forceinline__ void store_cols4(uint32_t *o, int x0, int M, int P,
                                            const uint32_t (&w)[4]) {
  if (x0 + 3 <= M) {
    uint4 q4;
    q4.x = w[0];
    q4.y = w[1];
    q4.z = w[2];
    q4.w = w[3];
    *reinterpret_cast<uint4 *>(o + x0) = q4;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (x0 + q < P) o[x0 + q] = x0 + q <= M ? w[q] : 0u;
  }
}

// Each 64 x 256 tile is one workgroup of four waves; wave w takes the tile's
// rows 16w .. 16w + 15 (a short serial chain per wave), lanes four columns.
constexpr int SAT_WAVES = 4;
constexpr int SAT_WR = SAT_TY / SAT_WAVES;  // rows per wave

// A lane's four columns over one wave's rows, requested before any is used.
__device__ __forceinline__ void load_wave_rows(const uint8_t *fb, int y0, int r0, int rows,
                                               int f_pitch, int x0, int M,
                                               uint32_t (&pk)[SAT_WR]) {
#pragma unroll
  for (int r = 0; r < SAT_WR; ++r)
    pk[r] = (r0 + r < rows && x0 < M) ? load_pk4(fb + (size_t)(y0 + r0 + r) * f_pitch, x0, M)
                                      : 0u;
}

// DPP add within quads of lanes: lanes 0-1 and 2-3 exchanged (quad_perm
// [1,0,3,2]), then the pairs (quad_perm [2,3,0,1]); every lane of a quad
// ends with the quad's sum.
__device__ __forceinline__ uint32_t quad_sum(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false);
  return v;
}

// Column totals, row totals and the tile total of f and f^2.  A lane's row
// sums over its four pixels are byte dot products (with ones for f, with
// themselves for f^2), added over quads of lanes with DPP; the quads' sums
// go through LDS, where lane r of the wave adds row r's sixteen, so that a
// wave's sixteen row totals leave as one coalesced store per table.
__global__ __launch_bounds__(256) void sat_totals(const uint8_t *__restrict__ f,
                                                  int B, int M, int N, int f_pitch,
                                                  uint32_t *__restrict__ scratch) {
  __shared__ uint32_t wcol[SAT_WAVES][8][64];   // per wave: column totals of f, f^2
  __shared__ uint2 rq[SAT_WAVES][SAT_WR][17];   // per wave and row: quads' sums (padded)
  SatScratch sc = sat_layout(scratch, B, M, N);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int J = blockIdx.x, I = blockIdx.y, b = blockIdx.z;
  const int x0 = J * SAT_TX + 4 * lane;
  const int y0 = I * SAT_TY;
  const int rows = min(SAT_TY, N - y0);
  const int r0 = w * SAT_WR;
  const uint8_t *fb = f + (size_t)b * N * f_pitch;
  uint32_t pk[SAT_WR];
  load_wave_rows(fb, y0, r0, rows, f_pitch, x0, M, pk);  // 0 past the frame
  // column sums: f as two 16-bit halves of a word (16 rows of bytes stay
  // below 2^16), f^2 as byte dot products of one byte each
  uint32_t lo = 0, hi = 0, t2[4] = {0, 0, 0, 0};
#pragma unroll
  for (int r = 0; r < SAT_WR; ++r) {
    const uint32_t x = pk[r];
    lo += x & 0x00ff00ffu;         // columns 0 and 2
    hi += (x >> 8) & 0x00ff00ffu;  // columns 1 and 3
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t m = x & (0xffu << (8 * q));
      t2[q] = __builtin_amdgcn_udot4(m, m, t2[q], false);
    }
  }
#pragma unroll
  for (int r = 0; r < SAT_WR; ++r) {
    const uint32_t a = quad_sum(__builtin_amdgcn_udot4(pk[r], 0x01010101u, 0u, false));
    const uint32_t a2 = quad_sum(__builtin_amdgcn_udot4(pk[r], pk[r], 0u, false));
    if ((lane & 3) == 0) rq[w][r][lane >> 2] = make_uint2(a, a2);
  }
  uint32_t cs[4] = {lo & 0xffffu, hi & 0xffffu, lo >> 16, hi >> 16}, cs2[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cs2[q] = t2[q];
    wcol[w][q][lane] = cs[q];
    wcol[w][4 + q][lane] = cs2[q];
  }
  __syncthreads();
  if (lane < SAT_WR && r0 + lane < rows) {
    uint32_t a = 0, a2 = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint2 e = rq[w][lane][i];
      a += e.x;
      a2 += e.y;
    }
    const size_t o = ((size_t)b * sc.nTX + J) * N + y0 + r0 + lane;
    sc.rowT[o] = a;
    sc.rowT[(size_t)B * N * sc.nTX + o] = a2;
  }
  if (w == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      for (int u = 1; u < SAT_WAVES; ++u) {
        cs[q] += wcol[u][q][lane];
        cs2[q] += wcol[u][4 + q][lane];
      }
    const size_t plane_col = (size_t)B * sc.nTY * M;
    const size_t o = ((size_t)b * sc.nTY + I) * M + x0;
    if (x0 + 3 < M && (M & 3) == 0) {  // 16-byte aligned: M and x0 are multiples of 4
      *reinterpret_cast<uint4 *>(sc.colT + o) = make_uint4(cs[0], cs[1], cs[2], cs[3]);
      *reinterpret_cast<uint4 *>(sc.colT + plane_col + o) =
          make_uint4(cs2[0], cs2[1], cs2[2], cs2[3]);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (x0 + q < M) {
          sc.colT[o + q] = cs[q];
          sc.colT[plane_col + o + q] = cs2[q];
        }
    }
    uint32_t tt = wave_sum(cs[0] + cs[1] + cs[2] + cs[3]);
    uint32_t tt2 = wave_sum(cs2[0] + cs2[1] + cs2[2] + cs2[3]);
    if (lane == 0) {
      const size_t ot = ((size_t)b * sc.nTY + I) * sc.nTX + J;
      const size_t plane_t = (size_t)B * sc.nTY * sc.nTX;
      sc.T[ot] = tt;
      sc.T[plane_t + ot] = tt2;
    }
  }
}

__global__ __launch_bounds__(256) void sat_scan(const uint8_t *__restrict__ f,
                                                int B, int M, int N, int f_pitch,
                                                const uint32_t *__restrict__ scratch,
                                                uint32_t *__restrict__ s,
                                                uint32_t *__restrict__ s2,
                                                int P) {
  __shared__ uint32_t wcol[SAT_WAVES][8][64];  // per wave: column totals of f, f^2
  __shared__ uint32_t wcar[SAT_WAVES][8][64];  // per wave: its part of the column carries
  SatScratch sc = sat_layout(const_cast<uint32_t *>(scratch), B, M, N);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int J = blockIdx.x, I = blockIdx.y, b = blockIdx.z;
  const int x0 = J * SAT_TX + 4 * lane;
  const int y0 = I * SAT_TY;
  const int rows = min(SAT_TY, N - y0);
  const int r0 = w * SAT_WR;
  const uint8_t *fb = f + (size_t)b * N * f_pitch;
  uint32_t *sb = s + (size_t)b * (N + 1) * P;
  uint32_t *s2b = s2 + (size_t)b * (N + 1) * P;

  uint32_t pk[SAT_WR];
  load_wave_rows(fb, y0, r0, rows, f_pitch, x0, M, pk);
  // this wave's column totals, for the waves below it (rows past the frame
  // are 0).  Sums of f as two 16-bit halves of a word (16 rows of bytes stay
  // below 2^16), squares as byte dot products: other instructions than the
  // row loop's, so the compiler does not keep the products of all 16 rows
  // live for the loop to reuse.
  {
    uint32_t lo = 0, hi = 0, t2[4] = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < SAT_WR; ++r) {
      const uint32_t x = pk[r];
      lo += x & 0x00ff00ffu;           // columns 0 and 2
      hi += (x >> 8) & 0x00ff00ffu;    // columns 1 and 3
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t m = x & (0xffu << (8 * q));
        t2[q] = __builtin_amdgcn_udot4(m, m, t2[q], false);
      }
    }
    wcol[w][0][lane] = lo & 0xffffu;
    wcol[w][1][lane] = hi & 0xffffu;
    wcol[w][2][lane] = lo >> 16;
    wcol[w][3][lane] = hi >> 16;
#pragma unroll
    for (int q = 0; q < 4; ++q) wcol[w][4 + q][lane] = t2[q];
  }
  // The carries, summed here from sat_totals' totals (modulo 2^32, so in any
  // order): the column totals of the tile rows above (the waves take every
  // fourth tile row and add their parts through LDS), each row's totals of
  // the tile columns to its left (lane r: row y0 + r), and the tile totals
  // above-left (spread over the lanes, then a wave sum).
  uint32_t cs[4] = {0, 0, 0, 0}, cs2[4] = {0, 0, 0, 0};
  const size_t plane_col = (size_t)B * sc.nTY * M;
  for (int Ip = w; Ip < I; Ip += SAT_WAVES) {
    const size_t o = ((size_t)b * sc.nTY + Ip) * M + x0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (x0 + q < M) {
        cs[q] += sc.colT[o + q];
        cs2[q] += sc.colT[plane_col + o + q];
      }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    wcar[w][q][lane] = cs[q];
    wcar[w][4 + q][lane] = cs2[q];
  }
  const size_t plane_row = (size_t)B * N * sc.nTX;
  uint32_t rl = 0, rl2 = 0;
  if (lane < rows)
    for (int Jp = 0; Jp < J; ++Jp) {
      const size_t o = ((size_t)b * sc.nTX + Jp) * N + y0 + lane;
      rl += sc.rowT[o];
      rl2 += sc.rowT[plane_row + o];
    }
  const size_t plane_t = (size_t)B * sc.nTY * sc.nTX;
  uint32_t ct = 0, ct2 = 0;
  for (int e = lane; e < I * J; e += 64) {
    const int Ip = e / J, Jp = e - Ip * J;
    const size_t o = ((size_t)b * sc.nTY + Ip) * sc.nTX + Jp;
    ct += sc.T[o];
    ct2 += sc.T[plane_t + o];
  }
  // left carry of row y0 + r (held by lane r): tile corner + rows' left sums
  const uint32_t L = wave_sum(ct) + wave_incl_scan(rl);
  const uint32_t L2 = wave_sum(ct2) + wave_incl_scan(rl2);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cs[q] = 0;
    cs2[q] = 0;
  }
  for (int u = 0; u < SAT_WAVES; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cs[q] += wcar[u][q][lane] + (u < w ? wcol[u][q][lane] : 0u);
      cs2[q] += wcar[u][4 + q][lane] + (u < w ? wcol[u][4 + q][lane] : 0u);
    }

#pragma unroll
  for (int r = 0; r < SAT_WR; ++r) {
    if (r0 + r >= rows) continue;  // uniform; every pk index stays a constant
    const int y = y0 + r0 + r;
    uint32_t p[4], p2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t v = (pk[r] >> (8 * q)) & 0xffu;
      cs[q] += v;
      cs2[q] += v * v;
      p[q] = (q ? p[q - 1] : 0u) + cs[q];
      p2[q] = (q ? p2[q - 1] : 0u) + cs2[q];
    }
    const uint32_t ex = wave_incl_scan(p[3]) - p[3];
    const uint32_t ex2 = wave_incl_scan(p2[3]) - p2[3];
    const uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)L, r0 + r) + ex;
    const uint32_t base2 = (uint32_t)__builtin_amdgcn_readlane((int)L2, r0 + r) + ex2;
    // the lane writes table columns x0 .. x0 + 3, whose entries sum the
    // pixel columns left of them: its base plus the exclusive prefix of its
    // quad (column 0 of the first tile gets 0).  The 16-byte stores are then
    // aligned, and a wave's row is whole cache lines
    uint32_t *o = sb + (size_t)(y + 1) * P;
    uint32_t *o2 = s2b + (size_t)(y + 1) * P;
    uint32_t wv[4], wv2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      wv[q] = base + (q ? p[q - 1] : 0u);
      wv2[q] = base2 + (q ? p2[q - 1] : 0u);
    }
    store_cols4(o, x0, M, P, wv);
    store_cols4(o2, x0, M, P, wv2);
    if (J == sc.nTX - 1) {
      // column M (the row's total) when it lies past the last tile, then
      // the padding columns M+1 .. P-1 past the last tile
      if (M == SAT_TX * sc.nTX && lane == 63) {
        o[M] = base + p[3];
        o2[M] = base2 + p2[3];
      }
      for (int c = max(M + 1, SAT_TX * sc.nTX) + lane; c < P; c += 64) {
        o[c] = 0;
        o2[c] = 0;
      }
    }
    // rows one after another: keeps the scheduler from interleaving all of a
    // wave's rows (which held every row's partial sums live at once)
    __builtin_amdgcn_sched_barrier(0);
  }
  if (I == 0 && w == 0) {  // padded row 0
    for (int c = J * SAT_TX + lane; c < (J + 1) * SAT_TX + (J == sc.nTX - 1 ? P : 0) && c < P;
         c += 64) {
      sb[c] = 0;
      s2b[c] = 0;
    }
  }
}

int launch_sat(const uint8_t *f, int B, int M, int N, int f_pitch, uint32_t *s,
               uint32_t *s2, int sat_pitch, uint32_t *scratch, hipStream_t st) {
  const int nTX = (M + SAT_TX - 1) / SAT_TX, nTY = (N + SAT_TY - 1) / SAT_TY;
  dim3 grid(nTX, nTY, B);
  hipLaunchKernelGGL(sat_totals, grid, dim3(64 * SAT_WAVES), 0, st, f, B, M, N, f_pitch,
                     scratch);
  hipLaunchKernelGGL(sat_scan, grid, dim3(64 * SAT_WAVES), 0, st, f, B, M, N, f_pitch, scratch,
                     s, s2, sat_pitch);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------ allocation-free sum tables
// Carries of sncc_build_sats_noalloc: one static array in each device's
// memory, reserved while the process runs.  In host code the array's name is
// only a stand-in for the symbol, not a device address: host code uses the
// address hipGetSymbolAddress returns for each device, looked up once with
// that device current (sat_noalloc_init, called when a context is created).
constexpr size_t kNoallocScratchWords = SNCC_NOALLOC_SCRATCH_BYTES / 4;
static __device__ __align__(256) uint32_t sat_noalloc_scratch[kNoallocScratchWords];

constexpr int kMaxDevices = 64;
static uint32_t *g_noalloc_addr[kMaxDevices] = {};
static std::mutex g_noalloc_mu;

int sat_noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_addr[device]) return 0;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(sat_noalloc_scratch)) != hipSuccess || !p) return -1;
  g_noalloc_addr[device] = static_cast<uint32_t *>(p);
  return 0;
}

uint32_t *sat_noalloc_addr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  return g_noalloc_addr[device];
}

// ------------------------------------------------------------ tile scoring
// One entry per tile shape (kTileShapes); the kernels live in the
// translation units built from tile_entry.hip.
struct TileEntry {
  int ru, rv, nw;
  const void *(*fn)(int sink);
};
static const TileEntry kTileEntries[] = {
    {kTileShapes[0][0], kTileShapes[0][1], kTileShapes[0][2], tile_fn_0},
    {kTileShapes[1][0], kTileShapes[1][1], kTileShapes[1][2], tile_fn_1},
    {kTileShapes[2][0], kTileShapes[2][1], kTileShapes[2][2], tile_fn_2},
    {kTileShapes[3][0], kTileShapes[3][1], kTileShapes[3][2], tile_fn_3},
    {kTileShapes[4][0], kTileShapes[4][1], kTileShapes[4][2], tile_fn_4},
    {kTileShapes[5][0], kTileShapes[5][1], kTileShapes[5][2], tile_fn_5},
};
static_assert(sizeof(kTileEntries) / sizeof(kTileEntries[0]) == kNumTileShapes,
              "one table entry per tile shape");
static const int kNumTileEntries = kNumTileShapes;

int tile_cfg_count() { return kNumCfgs; }
TileCfg tile_cfg(int i) { return tile_cfg_of(i); }
int tile_max_lds() { return kTileMaxLds; }

static const void *tile_fn(int cfg, int sink) {
  return kTileEntries[kCfgs[cfg].entry].fn(sink);
}

// Allows a tile kernel dynamic LDS up to what its static LDS leaves of a CU's.
static hipError_t allow_dynamic_lds(const void *fn) {
  hipFuncAttributes fa;
  const hipError_t e = hipFuncGetAttributes(&fa, fn);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                             tile_max_lds() - (int)fa.sharedSizeBytes);
}

int tile_occupancy(int cfg, int sink, int lds_bytes) {
  if (cfg < 0 || cfg >= kNumCfgs) return 0;
  const void *fn = tile_fn(cfg, sink);
  if (allow_dynamic_lds(fn) != hipSuccess) return 0;
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, tile_cfg(cfg).threads(),
                                                   (size_t)lds_bytes) != hipSuccess)
    return 0;
  return blocks;
}

int launch_tile(int cfg, int sink, const TileArgs &a, int grid, int lds_bytes,
                hipStream_t st) {
  if (cfg < 0 || cfg >= kNumCfgs || sink < kSinkTopk || sink > kSinkCompact) return -1;
  const void *fn = tile_fn(cfg, sink);
  static bool attr_done[3][kNumTileEntries] = {};
  const int ent = kCfgs[cfg].entry;
  if (!attr_done[sink][ent]) {
    if (allow_dynamic_lds(fn) != hipSuccess) return -1;
    attr_done[sink][ent] = true;
  }
  long long fs = a.frame_stride;
  int P = a.sat_pitch, N = a.N, nq = a.nq, k = a.k, rp = a.rho_pitch;
  const uint32_t *s = a.s, *s2 = a.s2;
  const DevTmpl *tm = a.tmpls;
  const PassDesc *ps = a.passes;
  const Interval *iv = a.ivs;
  const TileRec *rc = a.recs;
  const PairDesc *pr = a.pairs;
  const WorkItem *it = a.items;
  const int *ord = a.order, *qbeg = a.qbeg;
  int *queue = a.queue;
  u64 *partial = a.partial, *pfloor = a.pair_floor;
  float *rho = static_cast<float *>(a.rho);
  uint8_t *dg = a.degen;
  CompactOut co = a.co;
  void *args[] = {&s,  &s2, &fs, &P,  &N,     &tm,      &ps,  &iv,  &rc,  &pr,
                  &it, &ord, &qbeg, &nq, &queue, &k, &partial, &pfloor, &rho, &rp,
                  &dg, &co};
  hipError_t err = hipLaunchKernel(fn, dim3(grid), dim3(tile_cfg(cfg).threads()), args,
                                   (size_t)lds_bytes, st);
  return err == hipSuccess ? 0 : -1;
}

// --------------------------------------------------------------- plain FP64
// rho at one offset, segments read from global memory, FP64 accumulation of
// box_i * c_i; Eq. (12)'s mean term is fbar * sum_i A_i c_i.
__device__ __forceinline__ double rho_plain(const uint32_t *__restrict__ S,
                                            const uint32_t *__restrict__ S2, int P, int u,
                                            int v, int W, int H, int K, int sq_rows,
                                            double q_k, double r64,
                                            const int4 *__restrict__ geom,
                                            const double *__restrict__ c64, bool &flat) {
  const uint32_t *a0 = S + (long long)v * P + u;
  const uint32_t *a1 = a0 + (long long)H * P;
  const uint32_t sf = (a1[W] - a1[0]) - (a0[W] - a0[0]);
  const u64 sf2 = window_sq(S2 + (long long)v * P + u, W, H, P, sq_rows);  // Eq. (15)
  const int n = W * H;
  const long long V = (long long)((u64)(uint32_t)n * sf2 - (u64)sf * sf);
  double acc = 0.0;
  for (int i = 0; i < K; ++i) {
    const int4 g = geom[i];  // x, y, width, height
    const uint32_t *q0 = a0 + (long long)g.y * P + g.x;
    const uint32_t *q2 = q0 + (long long)g.w * P;
    const uint32_t F = (q2[g.z] - q2[0]) - (q0[g.z] - q0[0]);
    acc = __builtin_fma((double)F, c64[i], acc);
  }
  flat = V == 0;
  const double fbar = (double)sf / (double)n;
  const double num = acc - fbar * r64;
  return flat ? 0.0 : num / sqrt((double)V / (double)n * q_k);
}

__global__ __launch_bounds__(256) void plain_kernel(
    const uint32_t *__restrict__ S, const uint32_t *__restrict__ S2, int P, int nu, int nv,
    int W, int H, int K, int sq_rows, double q_k, double r64, const int4 *__restrict__ geom,
    const double *__restrict__ c64, double *__restrict__ rho, int rho_pitch,
    uint8_t *__restrict__ degen) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int u = blockIdx.x * 64 + lane, v = blockIdx.y * 4 + wave;
  if (u >= nu || v >= nv) return;
  bool flat;
  const double r = rho_plain(S, S2, P, u, v, W, H, K, sq_rows, q_k, r64, geom, c64, flat);
  rho[(long long)v * rho_pitch + u] = r;
  if (degen) degen[(long long)v * rho_pitch + u] = flat ? 1 : 0;
}

int launch_plain(const PlainArgs &a, hipStream_t st) {
  dim3 grid((a.nu + 63) / 64, (a.nv + 3) / 4);
  hipLaunchKernelGGL(plain_kernel, grid, dim3(256), 0, st, a.s, a.s2, a.sat_pitch, a.nu,
                     a.nv, a.W, a.H, a.K, a.sq_rows, a.q_k, a.r64, a.geom, a.c64, a.rho,
                     a.rho_pitch,
                     a.degen);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Exact window energy V = n * sum f^2 - (sum f)^2 (n times Eq. (16)) at every
// offset, from the frame's tables (the f^2 sum banded when the window exceeds
// one exact box).
__global__ __launch_bounds__(256) void energy_kernel(const uint32_t *__restrict__ S,
                                                     const uint32_t *__restrict__ S2, int P,
                                                     int nu, int nv, int W, int H, int sq_rows,
                                                     long long *__restrict__ energy, int pitch) {
  const int u = blockIdx.x * 64 + (threadIdx.x & 63), v = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (u >= nu || v >= nv) return;
  const uint32_t *a0 = S + (long long)v * P + u;
  const uint32_t *a1 = a0 + (long long)H * P;
  const uint32_t sf = (a1[W] - a1[0]) - (a0[W] - a0[0]);
  const u64 sf2 = window_sq(S2 + (long long)v * P + u, W, H, P, sq_rows);
  const u64 n = (u64)W * (u64)H;
  energy[(long long)v * pitch + u] = (long long)(n * sf2 - (u64)sf * sf);
}

int launch_energy(const uint32_t *s, const uint32_t *s2, int P, int nu, int nv, int W, int H,
                  int sq_rows, long long *energy, int pitch, hipStream_t st) {
  dim3 grid((nu + 63) / 64, (nv + 3) / 4);
  hipLaunchKernelGGL(energy_kernel, grid, dim3(256), 0, st, s, s2, P, nu, nv, W, H, sq_rows,
                     energy, pitch);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------- small kernels
__global__ void zero_kernel(int *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

int launch_zero(int *p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// One wave per pair: merges the pair's item partials into the final top-k.
// Per pair, the k best of its items' partial lists: the items of `pairs`
// in `partial` and, when a second launch scored the pair's last tile
// column, those of `pairs2` in `partial2`.
__global__ __launch_bounds__(256) void merge_kernel(const PairDesc *__restrict__ pairs,
                                                    const PairDesc *__restrict__ pairs2,
                                                    int n_pairs,
                                                    const u64 *__restrict__ partial,
                                                    const u64 *__restrict__ partial2, int k,
                                                    sncc_match *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= n_pairs) return;
  const PairDesc pd = pairs[p];
  u64 lkey = 0, thr = 0;
  // one load brings the partial lists of g = 64 / k items (lane l holds key
  // l mod k of item l / k), and the next load is issued before the current
  // keys are used, so its latency overlaps their merge
  const int g = 64 / k;
  auto merge_items = [&](const u64 *part, int ib, int ie) {
    auto load = [&](int item) -> u64 {
      const int mi = item + lane / k;
      return lane < g * k && mi < ie ? part[(long long)mi * k + lane % k] : 0;
    };
    u64 next = ib < ie ? load(ib) : 0;
    for (int item = ib; item < ie; item += g) {
      const u64 mine = next;
      if (item + g < ie) next = load(item + g);
      // only keys above the current k-th can enter.  A few are inserted one
      // by one in lane order, each checked again against the k-th as it
      // rises; more are sorted across the wave and merged in one step (the
      // same k best: keys are distinct)
      u64 cand = __ballot(mine > thr);
      if (__popcll(cand) > 2) {
        topk_merge_sorted(lkey, wave_sort_desc_u64(mine > thr ? mine : 0ull, lane), k, lane);
        thr = lane_u64(lkey, k - 1);
        continue;
      }
      while (cand) {
        const int l = __ffsll((long long)cand) - 1;
        cand &= cand - 1;
        const u64 key = lane_u64(mine, l);
        if (key <= thr) continue;
        topk_insert(lkey, key, k, lane);
        thr = lane_u64(lkey, k - 1);
      }
    }
  };
  merge_items(partial, pd.item_begin, pd.item_end);
  if (pairs2) {
    const PairDesc pe = pairs2[p];
    merge_items(partial2, pe.item_begin, pe.item_end);
  }
  if (lane < k) {
    sncc_match m;
    if (lkey == 0) {
      m.u = -1;
      m.v = -1;
      m.rho = -__builtin_inff();
    } else {
      const int idx = (int)(0xffffffffu - (uint32_t)(lkey & 0xffffffffu));
      m.v = idx / pd.nu;
      m.u = idx - m.v * pd.nu;
      m.rho = float_unorder((uint32_t)(lkey >> 32));
    }
    out[(long long)p * k + lane] = m;
  }
}

int launch_merge(const PairDesc *pairs, const PairDesc *pairs2, int n_pairs, const u64 *partial,
                 const u64 *partial2, int k, sncc_match *out, hipStream_t st) {
  hipLaunchKernelGGL(merge_kernel, dim3((n_pairs + 3) / 4), dim3(256), 0, st, pairs, pairs2,
                     n_pairs, partial, partial2, k, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Top-k over a double map with exact keys (the value's 64-bit order code and
// the index), one chunk of `chunk` offsets per workgroup; partial lists of
// k keys per chunk, best first, as {code, ~index} pairs.
__global__ __launch_bounds__(256) void map_topk64_kernel(const double *__restrict__ map,
                                                         int pitch, int nu, int nv, int chunk,
                                                         int k, Key96 *__restrict__ partial) {
  __shared__ u64 bh[4 * 64];
  __shared__ uint32_t bl[4 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long total = (long long)nu * nv;
  const long long c0 = (long long)blockIdx.x * chunk;
  const long long c1 = min(total, c0 + chunk);
  u64 lh = 0;
  uint32_t ll = 0;
  for (long long e0 = c0 + wave * 64; e0 < c1; e0 += 4 * 64) {
    const long long e = e0 + lane;
    u64 ch = 0;
    uint32_t cl = 0;
    if (e < c1) {
      const int v = (int)(e / nu), u = (int)(e - (long long)v * nu);
      ch = double_order(map[(long long)v * pitch + u]);
      cl = 0xffffffffu - (uint32_t)e;
    }
    // offer the wave's 64 candidates, best first, while they beat the k-th
    u64 th = lane_u64(lh, k - 1);
    uint32_t tl = (uint32_t)__builtin_amdgcn_readlane((int)ll, k - 1);
    if (!key96_gt(ch, cl, th, tl)) ch = 0, cl = 0;
    for (;;) {
      if (__ballot(ch != 0 || cl != 0) == 0) break;
      u64 mh;
      uint32_t ml;
      wave_max96(ch, cl, mh, ml);
      topk96_insert(lh, ll, mh, ml, k, lane);
      if (ch == mh && cl == ml) ch = 0, cl = 0;
      th = lane_u64(lh, k - 1);
      tl = (uint32_t)__builtin_amdgcn_readlane((int)ll, k - 1);
      if (!key96_gt(ch, cl, th, tl)) ch = 0, cl = 0;
    }
  }
  if (lane < k) {
    bh[wave * k + lane] = lh;
    bl[wave * k + lane] = ll;
  }
  __syncthreads();
  if (wave == 0) {
    for (int w = 1; w < 4; ++w)
      for (int j = 0; j < k; ++j) {
        const u64 kh = bh[w * k + j];
        const uint32_t kl = bl[w * k + j];
        const u64 th = lane_u64(lh, k - 1);
        const uint32_t tl = (uint32_t)__builtin_amdgcn_readlane((int)ll, k - 1);
        if (!key96_gt(kh, kl, th, tl)) break;  // each wave's list is in descending order
        topk96_insert(lh, ll, kh, kl, k, lane);
      }
    if (lane < k) partial[(long long)blockIdx.x * k + lane] = Key96{lh, ll, 0};
  }
}

int launch_map_topk64(const double *map, int pitch, int nu, int nv, int chunk, int k,
                      Key96 *partial, hipStream_t st) {
  const long long total = (long long)nu * nv;
  const int blocks = (int)((total + chunk - 1) / chunk);
  hipLaunchKernelGGL(map_topk64_kernel, dim3(blocks), dim3(256), 0, st, map, pitch, nu, nv,
                     chunk, k, partial);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// One wave per pair: the k best of the pair's chunk lists (exact keys); the
// matches report rho rounded to float.
__global__ __launch_bounds__(256) void merge64_kernel(const PairDesc *__restrict__ pairs,
                                                      int n_pairs,
                                                      const Key96 *__restrict__ partial, int k,
                                                      sncc_match *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= n_pairs) return;
  const PairDesc pd = pairs[p];
  u64 lh = 0;
  uint32_t ll = 0;
  for (int item = pd.item_begin; item < pd.item_end; ++item)
    for (int j = 0; j < k; ++j) {
      const Key96 e = partial[(long long)item * k + j];
      const u64 th = lane_u64(lh, k - 1);
      const uint32_t tl = (uint32_t)__builtin_amdgcn_readlane((int)ll, k - 1);
      if (!key96_gt(e.hi, e.lo, th, tl)) break;  // each list is in descending order
      topk96_insert(lh, ll, e.hi, e.lo, k, lane);
    }
  if (lane < k) {
    sncc_match m;
    if (lh == 0 && ll == 0) {
      m.u = -1;
      m.v = -1;
      m.rho = -__builtin_inff();
    } else {
      const int idx = (int)(0xffffffffu - ll);
      m.v = idx / pd.nu;
      m.u = idx - m.v * pd.nu;
      m.rho = (float)double_unorder(lh);
    }
    out[(long long)p * k + lane] = m;
  }
}

int launch_merge64(const PairDesc *pairs, int n_pairs, const Key96 *partial, int k,
                   sncc_match *out, hipStream_t st) {
  hipLaunchKernelGGL(merge64_kernel, dim3((n_pairs + 3) / 4), dim3(256), 0, st, pairs, n_pairs,
                     partial, k, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// --------------------------------------------------- two-threshold search
// Section 5, steps 7g-j for the offsets that passed the fast test: rho with
// the slow approximation in FP64, appended to the output when it reaches the
// template's slow threshold.  Workgroups take runs of the survivor list (the
// survivors one wave of the fast pass found in one group of kRunCols columns
// of a tile: one pair, a few offset rows) from a counter.
//
// Staged form: the workgroup copies the run's region of the frame's table
// (every entry a window of the run reads) to LDS and makes it relative to its
// first row and column; each wave then scores four survivors at a time, lanes
// over the template's corner slots (see SlowTmpl): per slot one LDS read
// gives the table entry at the corner, W times it is accumulated in FP64 per
// lane, and the wave's sum is the sum of c_i F_i over the segments (Eq. (12),
// summation by parts of Eq. (11) over the corners).  Global form (regions too large for LDS): lanes over the
// run's survivors, each scoring its own offset over the shared segment list
// with buffer loads whose scalar offset is the segment's corner, blocks of
// kSlowBlock segments loaded before they are summed in segment order.
constexpr int kSlowBlock = 8;
constexpr int kSlowBatch = 4;  // survivors per wave in the staged form (four registers
                               // in the scoring loop's asm operand list)

// Sum over the segments of c_i F_i (Eq. (12), first term) for the window at
// voff (bytes from the frame table's base); uniform segment list.
__device__ __forceinline__ double slow_sum(__amdgpu_buffer_rsrc_t rs, int voff, int P4,
                                           const int4 *__restrict__ gp,
                                           const double *__restrict__ cp, int K) {
  double acc = 0.0;
  int i = 0;
  for (; i + kSlowBlock <= K; i += kSlowBlock) {
    uint32_t F[kSlowBlock];
#pragma unroll
    for (int j = 0; j < kSlowBlock; ++j) {
      const int4 g = gp[i + j];  // x, y, width, height
      F[j] = window_box(rs, voff, g.y * P4 + g.x * 4, g.z * 4, g.w * P4);  // Eq. (11)
    }
#pragma unroll
    for (int j = 0; j < kSlowBlock; ++j) acc = __builtin_fma((double)F[j], cp[i + j], acc);
  }
  for (; i < K; ++i) {
    const int4 g = gp[i];
    const uint32_t F = window_box(rs, voff, g.y * P4 + g.x * 4, g.z * 4, g.w * P4);
    acc = __builtin_fma((double)F, cp[i], acc);
  }
  return acc;
}

template <int CTRL>
__device__ __forceinline__ double dpp_full_f64(double x) {  // every lane has a source
  const u64 b = (u64)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xf, 0xf, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((u64)hi << 32) | lo));
}

// Wave sums of four values at once: lane l returns the sum of a_(l mod 4)
// over all 64 lanes.  Two exchange steps (lanes l and l ^ 1, then l ^ 2)
// leave each lane with a partial sum of the value of its residue, then
// four more steps (xor 4, 8 within rows of 16 lanes; 16, 32 across rows)
// add the partials of the same residue.
__device__ __forceinline__ double wave_sum4_f64(double a0, double a1, double a2, double a3,
                                                int lane) {
  const bool odd = lane & 1, hi2 = lane & 2;
  double k01 = odd ? a1 : a0, g01 = odd ? a0 : a1;
  double k23 = odd ? a3 : a2, g23 = odd ? a2 : a3;
  k01 += dpp_full_f64<0xb1>(g01);  // quad_perm [1,0,3,2]: lane l ^ 1
  k23 += dpp_full_f64<0xb1>(g23);
  double k = hi2 ? k23 : k01, g = hi2 ? k01 : k23;
  k += dpp_full_f64<0x4e>(g);      // quad_perm [2,3,0,1]: lane l ^ 2
  k += dpp_full_f64<0x124>(k);     // row_ror:4
  k += dpp_full_f64<0x128>(k);     // row_ror:8
  k += __shfl_xor(k, 16);
  k += __shfl_xor(k, 32);
  return k;
}

// Copies rows [0, nrow) x columns [0, ncol) of the table window whose
// top-left entry is (v0, u0) to LDS at `region` (row pitch `pitch` words),
// table rows clamped to N and columns to P - 1, with LDS-direct buffer loads
// (no registers, all in flight together), and waits for them.  Four waves.
__device__ __forceinline__ void stage_region(__amdgpu_buffer_rsrc_t rs, int P, int N, int v0,
                                             int u0, int nrow, int ncol, int pitch,
                                             uint32_t *region, int wave, int lane,
                                             int n_waves = 4) {
  for (int row = wave; row < nrow; row += n_waves) {
    const int gy = min(v0 + row, N);
    for (int c0 = 0; c0 < ncol; c0 += 64) {
      if (c0 + lane < ncol) {
        const int gx = min(u0 + c0 + lane, P - 1);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (__attribute__((address_space(3))) void *)(region + row * pitch + c0), 4,
            (gy * P + gx) * 4, 0, 0, 0);
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
}

// The staged region made relative in both directions (modulo 2^32): entry
// (r, c) becomes s(r, c) - s(r, 0) - s(0, c) + s(0, 0), the sum of f over the
// region's rows [0, r) and columns [0, c), below 255 x rows x pitch, so it is
// exact as an unsigned 32-bit value for any frame and the FP64 products W s
// stay small.  Box sums are unchanged, and so is a template's corner sum: its
// weights add to zero along every row and every column.  s(0, c) comes from
// the global table (the entries stage_region read), so a wave shifts the rows
// it staged as soon as its own loads have landed, without a barrier; four
// rows at a time, their first entries read before any row is written.
__device__ __forceinline__ void region_relative(__amdgpu_buffer_rsrc_t rs, int P, int N, int v0,
                                                int u0, uint32_t *region, int nrow, int ncol,
                                                int pitch, int wave, int lane, int n_waves) {
  constexpr int G = 4, ZK = 4;  // rows per group; column chunks whose s(0, c) stay in registers
  const int gy = min(v0, N) * P;  // the region's first row in the table
  auto row0_entry = [&](int c) {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, min(u0 + c, P - 1) * 4, gy * 4, 0);
  };
  const uint32_t s00 = __builtin_amdgcn_raw_buffer_load_b32(rs, 0, (gy + min(u0, P - 1)) * 4, 0);
  uint32_t zk[ZK];
#pragma unroll
  for (int k = 0; k < ZK; ++k) zk[k] = lane + 64 * k < ncol ? row0_entry(lane + 64 * k) : 0u;
  for (int row0 = wave; row0 < nrow; row0 += G * n_waves) {
    uint32_t b[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int row = row0 + g * n_waves;
      b[g] = row < nrow ? region[row * pitch] - s00 : 0u;
    }
    auto shift = [&](int c, uint32_t z) {
      uint32_t v[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int row = row0 + g * n_waves;
        v[g] = row < nrow ? region[row * pitch + c] : 0u;
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int row = row0 + g * n_waves;
        if (row < nrow) region[row * pitch + c] = v[g] - b[g] - z;
      }
    };
#pragma unroll
    for (int k = 0; k < ZK; ++k)
      if (lane + 64 * k < ncol) shift(lane + 64 * k, zk[k]);
    for (int c = lane + 64 * ZK; c < ncol; c += 64) shift(c, row0_entry(c));
  }
}

__device__ __forceinline__ uint32_t lds_at(const uint32_t *region, int byte_off) {
  return *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(region) + byte_off);
}

// rho from the numerator's segment sum and the window sums (Eqs. (12),
// (16)-(18)), FP64.
__device__ __forceinline__ double slow_rho(double acc, uint32_t sf, u64 sf2, const DevTmpl &td) {
  const long long V = (long long)((u64)(uint32_t)td.n * sf2 - (u64)sf * sf);
  const double num = acc - (double)sf / (double)td.n * td.r64;
  return V == 0 ? 0.0 : num / sqrt((double)V / (double)td.n * td.q_k);
}

// Whether four windows are consecutive offsets of one row (region byte
// offsets 4 apart); the answer is made wave-uniform.
__device__ __forceinline__ bool consecutive4(const int (&base)[4]) {
  const bool c = base[1] == base[0] + 4 && base[2] == base[0] + 8 && base[3] == base[0] + 12;
  return __builtin_amdgcn_readfirstlane((int)c) != 0;
}

// FP64 sum of c_i F_i over the segments (Eq. (12), first term) for four
// windows of one template whose table entries are staged in LDS (made
// relative by region_relative): base[j] is the region byte offset of window
// j's top-left entry.  Lanes run over the template's corner slots (see
// SlowTmpl), 64-slot blocks whose slot entries are requested ahead; per slot
// and window one LDS read gives the table entry s at the corner and W s is
// added to the lane's FP64 sum, which over all corners is the sum of c_i F_i.
// Lane l returns the sum of window l mod 4.  CONSEC: the four windows are consecutive offsets of one row
// (base[j] = base[0] + 4 j), so one address per slot serves all four reads,
// with immediate offsets.  DEEP: slot entries four blocks ahead in three
// register sets (more registers), else one step ahead.
template <bool CONSEC, bool DEEP>
__device__ __forceinline__ double staged_num4(const uint32_t *region, const int (&base)[4],
                                              __amdgpu_buffer_rsrc_t rso,
                                              __amdgpu_buffer_rsrc_t rsw, int n_iter, int lane) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  auto block = [&](uint32_t o, double w) {
    uint32_t D[4];
    if constexpr (CONSEC) {
      const uint32_t *pp =
          reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(region) + base[0] + o);
#pragma unroll
      for (int j = 0; j < 4; ++j) D[j] = pp[j];
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) D[j] = lds_at(region, base[j] + (int)o);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = __builtin_fma((double)D[j], w, acc[j]);
  };
  auto load_o = [&](int i) {
    return __builtin_amdgcn_raw_buffer_load_b32(rso, lane * 4, min(i, n_iter - 1) * 256, 0);
  };
  auto load_w = [&](int i) {
    return __builtin_bit_cast(
        double, __builtin_amdgcn_raw_buffer_load_b64(rsw, lane * 8, min(i, n_iter - 1) * 512, 0));
  };
  if constexpr (DEEP) {
    // slot entries in three register sets, each reloaded as soon as its two
    // blocks are scored and used four blocks later (no register copies, which
    // would wait for the loads)
    uint32_t oa0 = load_o(0), oa1 = load_o(1), ob0 = load_o(2), ob1 = load_o(3), oc0 = load_o(4),
             oc1 = load_o(5);
    double wa0 = load_w(0), wa1 = load_w(1), wb0 = load_w(2), wb1 = load_w(3), wc0 = load_w(4),
           wc1 = load_w(5);
    int it = 0;
    for (; it + 6 <= n_iter; it += 6) {
      block(oa0, wa0);
      block(oa1, wa1);
      oa0 = load_o(it + 6);
      oa1 = load_o(it + 7);
      wa0 = load_w(it + 6);
      wa1 = load_w(it + 7);
      // thirds one after another: interleaving all six blocks' LDS reads would
      // hold them live at once and cost occupancy
      __builtin_amdgcn_sched_barrier(0);
      block(ob0, wb0);
      block(ob1, wb1);
      ob0 = load_o(it + 8);
      ob1 = load_o(it + 9);
      wb0 = load_w(it + 8);
      wb1 = load_w(it + 9);
      __builtin_amdgcn_sched_barrier(0);
      block(oc0, wc0);
      block(oc1, wc1);
      oc0 = load_o(it + 10);
      oc1 = load_o(it + 11);
      wc0 = load_w(it + 10);
      wc1 = load_w(it + 11);
      __builtin_amdgcn_sched_barrier(0);
    }
    // the last n_iter - it < 6 blocks, held in the sets in order
    if (it < n_iter) block(oa0, wa0);
    if (it + 1 < n_iter) block(oa1, wa1);
    if (it + 2 < n_iter) block(ob0, wb0);
    if (it + 3 < n_iter) block(ob1, wb1);
    if (it + 4 < n_iter) block(oc0, wc0);
    if (it + 5 < n_iter) block(oc1, wc1);
  } else {
    // one step ahead (the copies into the current registers wait for the
    // loads): fewer registers, for kernels whose occupancy they limit
    uint32_t o0 = load_o(0), o1 = load_o(1);
    double w0 = load_w(0), w1 = load_w(1);
    int it = 0;
    for (; it + 2 <= n_iter; it += 2) {
      const uint32_t n0 = load_o(it + 2), n1 = load_o(it + 3);
      const double m0 = load_w(it + 2), m1 = load_w(it + 3);
      block(o0, w0);
      block(o1, w1);
      o0 = n0;
      o1 = n1;
      w0 = m0;
      w1 = m1;
    }
    if (it < n_iter) block(o0, w0);
  }
  return wave_sum4_f64(acc[0], acc[1], acc[2], acc[3], lane);
}

// FP64 rho (Eqs. (13), (15)-(18)) of the window whose top-left entry is at
// region byte offset q (row pitch `pitch` words) and global byte offset g,
// given its segment sum.
__device__ __forceinline__ double staged_rho(double sum, const uint32_t *region, int pitch, int q,
                                             int g, __amdgpu_buffer_rsrc_t rs2, int P4,
                                             const DevTmpl &td) {
  const int qh = q + td.H * pitch * 4, w4 = td.W * 4;
  const uint32_t sf = (lds_at(region, qh + w4) - lds_at(region, qh)) -
                      (lds_at(region, q + w4) - lds_at(region, q));  // Eq. (13)
  const u64 sf2 = window_sq(rs2, g, 0, w4, P4, td.H, td.sq_rows);  // Eq. (15)
  return slow_rho(sum, sf, sf2, td);
}

// rho of four windows (staged_num4, then staged_rho for lane l's window
// l mod 4; gof[j] is window j's byte offset in the global tables).
template <bool CONSEC>
__device__ __forceinline__ double staged_rho4(const uint32_t *region, int pitch,
                                              const int (&base)[4], const int (&gof)[4],
                                              __amdgpu_buffer_rsrc_t rso,
                                              __amdgpu_buffer_rsrc_t rsw, int n_iter,
                                              __amdgpu_buffer_rsrc_t rs2, int P4,
                                              const DevTmpl &td, int lane) {
  const double sum = staged_num4<CONSEC, true>(region, base, rso, rsw, n_iter, lane);
  const int jj = lane & 3;
  const int q = jj == 0 ? base[0] : jj == 1 ? base[1] : jj == 2 ? base[2] : base[3];
  const int g = jj == 0 ? gof[0] : jj == 1 ? gof[1] : jj == 2 ? gof[2] : gof[3];
  return staged_rho(sum, region, pitch, q, g, rs2, P4, td);
}


// Kernel arguments are restrict-qualified pointers (not an argument block)
// so that wave-uniform descriptor and segment reads become scalar loads.
__global__ __launch_bounds__(256) void slow_kernel(
    const uint32_t *__restrict__ s, const uint32_t *__restrict__ s2, long long frame_stride,
    int P, int N, const DevTmpl *__restrict__ tmpls, const int4 *__restrict__ geom,
    const double *__restrict__ c64, const SlowTmpl *__restrict__ stmpl,
    const uint32_t *__restrict__ slot_off, const double *__restrict__ slot_w,
    const PairDesc *__restrict__ pairs, const double *__restrict__ thrs,
    const sncc_hit *__restrict__ cand, const int *__restrict__ cand_count, int cand_cap,
    const RunDesc *__restrict__ runs, const int *__restrict__ run_count, int run_cap,
    int *__restrict__ work, sncc_hit *__restrict__ out, int out_cap,
    int *__restrict__ out_count) {
  extern __shared__ uint32_t region[];
  __shared__ int run_sh;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n_cand = min(*cand_count, cand_cap);
  const int n_runs = min(*run_count, run_cap);
  const int P4 = P * 4;
  const uint32_t bytes = (uint32_t)(frame_stride * 4);
  auto emit = [&](int pair, int u, int v, double rho) {
    const int pos = atomicAdd(out_count, 1);
    if (pos < out_cap) {
      sncc_hit o;
      o.pair = pair;
      o.u = u;
      o.v = v;
      o.reserved = 0;
      o.rho = rho;
      out[pos] = o;
    }
  };
  for (;;) {
    if (threadIdx.x == 0) run_sh = atomicAdd(work, 1);
    __syncthreads();
    const int r = __builtin_amdgcn_readfirstlane(run_sh);
    if (r >= n_runs) break;
    const RunDesc rd = runs[r];
    const int start = rd.start, end = min(rd.start + rd.count, n_cand);
    const PairDesc pd = pairs[rd.pair];
    const DevTmpl td = tmpls[pd.tmpl];
    const SlowTmpl st = stmpl[pd.tmpl];
    const double thr = thrs[pd.tmpl];
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(s + (long long)pd.frame * frame_stride, bytes);
    const __amdgpu_buffer_rsrc_t rs2 = make_rsrc(s2 + (long long)pd.frame * frame_stride, bytes);
    if (start < end && st.tbl >= 0) {
      // region rows [v0, v0 + rows), columns [u0, u0 + pitch), clamped to
      // the table (clamped entries are never read by a window of the run)
      stage_region(rs, P, N, rd.v0, rd.u0, st.rows, st.pitch, st.pitch, region, wave, lane);
      region_relative(rs, P, N, rd.v0, rd.u0, region, st.rows, st.pitch, st.pitch, wave, lane, 4);
      __syncthreads();
      const __amdgpu_buffer_rsrc_t rso = make_rsrc(slot_off + st.tbl, (uint32_t)st.n_iter * 256u);
      const __amdgpu_buffer_rsrc_t rsw = make_rsrc(slot_w + st.tbl, (uint32_t)st.n_iter * 512u);
      for (int b = start + wave * kSlowBatch; b < end; b += 4 * kSlowBatch) {
        int su[kSlowBatch], sv[kSlowBatch], base[kSlowBatch], gof[kSlowBatch];
#pragma unroll
        for (int j = 0; j < kSlowBatch; ++j) {
          const sncc_hit h = cand[min(b + j, end - 1)];
          su[j] = h.u;
          sv[j] = h.v;
          base[j] = ((h.v - rd.v0) * st.pitch + (h.u - rd.u0)) * 4;
          gof[j] = h.v * P4 + h.u * 4;
        }
        // lane j < kSlowBatch holds survivor b + j
        const double rho =
            consecutive4(base)
                ? staged_rho4<true>(region, st.pitch, base, gof, rso, rsw, st.n_iter, rs2, P4,
                                    td, lane)
                : staged_rho4<false>(region, st.pitch, base, gof, rso, rsw, st.n_iter, rs2, P4,
                                     td, lane);
        const int jj = lane & 3;
        const int uu = jj == 0 ? su[0] : jj == 1 ? su[1] : jj == 2 ? su[2] : su[3];
        const int vv = jj == 0 ? sv[0] : jj == 1 ? sv[1] : jj == 2 ? sv[2] : sv[3];
        if (lane < kSlowBatch && b + lane < end && rho >= thr) emit(rd.pair, uu, vv, rho);
      }
    } else if (start < end) {
      for (int b = start + wave * 64; b < end; b += 256) {
        const int c = b + lane;
        const sncc_hit h = cand[min(c, end - 1)];
        const int voff = h.v * P4 + h.u * 4;
        const double acc = slow_sum(rs, voff, P4, geom + td.seg_off, c64 + td.seg_off, td.K);
        const uint32_t sf = window_box(rs, voff, 0, td.W * 4, td.H * P4);  // Eq. (13)
        const u64 sf2 = window_sq(rs2, voff, 0, td.W * 4, P4, td.H, td.sq_rows);
        const double rho = slow_rho(acc, sf, sf2, td);
        if (c < end && rho >= thr) emit(rd.pair, h.u, h.v, rho);
      }
    }
    __syncthreads();  // region and run_sh are rewritten for the next run
  }
}

int slow_occupancy(int lds_bytes) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, slow_kernel, 256, lds_bytes) !=
      hipSuccess)
    return 1;
  return std::max(1, blocks);
}

int launch_slow(const SlowArgs &a, int grid, int lds_bytes, hipStream_t st) {
  hipLaunchKernelGGL(slow_kernel, dim3(grid), dim3(256), lds_bytes, st, a.s, a.s2,
                     a.frame_stride, a.P, a.N, a.tmpls, a.geom, a.c64, a.stmpl, a.slot_off,
                     a.slot_w, a.pairs, a.thr, a.cand, a.cand_count, a.cand_cap, a.runs,
                     a.run_count, a.run_cap, a.work, a.out, a.out_cap, a.out_count);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------------------------- FP64 refine
// Section 5, steps 7f-i with the coarse pass's top-k as candidates: rho in
// FP64 with the fine approximation at every offset within `radius` of a
// candidate, and the best of them (rho descending, then v, then u).  One
// workgroup per pair: the candidates are ordered by (column band of 16, v, u)
// in one wave, and their neighbourhoods are listed in LDS in that order, each
// offset once (by the first candidate whose neighbourhood holds it).  The
// unique offsets are then scored in chunks
// of at most kRefineChunk consecutive entries spanning at most the
// template's region spans (32 x 16 offsets where that region fits the LDS
// budget, else 16 x 8), each from a staged region of the frame's
// table: the segment sums four offsets per wave at a time (staged_num4),
// then rho one offset per thread (staged_rho); for templates whose region
// does not fit LDS, one offset per thread from the global tables
// (rho_plain).
constexpr int REFINE_CAP = 4096;
constexpr int kRefineChunk = 128;  // entries per chunk: up to four batches of four per wave
constexpr int kRefineWaves = 8;
constexpr int kRefineThreads = 64 * kRefineWaves;

__global__ __launch_bounds__(kRefineThreads) void refine_kernel(
    const uint32_t *__restrict__ s, const uint32_t *__restrict__ s2, long long frame_stride,
    int P, const DevTmpl *__restrict__ tmpls, const int4 *__restrict__ geom,
    const double *__restrict__ c64, const SlowTmpl *__restrict__ stmpl,
    const uint32_t *__restrict__ slot_off, const double *__restrict__ slot_w,
    const PairDesc *__restrict__ pairs, const int *__restrict__ order,
    const sncc_match *__restrict__ cand, int n_cand, int radius, int N,
    sncc_match64 *__restrict__ out, int *__restrict__ count) {
  __shared__ uint32_t first[REFINE_CAP / 32];  // bit i: entry i starts a chunk
  __shared__ int wsum[kRefineWaves];
  __shared__ double best_r[kRefineWaves];
  __shared__ int best_i[kRefineWaves];
  __shared__ int cand_u[64], cand_v[64];  // the candidates in (band, v, u) order
  // the chunk's segment sums (kRefineChunk doubles), the offset list (np
  // ints), then the region
  extern __shared__ __align__(16) uint32_t dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int p = order ? order[blockIdx.x] : (int)blockIdx.x;
  const PairDesc pd = pairs[p];
  const DevTmpl td = tmpls[pd.tmpl];
  const SlowTmpl st = stmpl[pd.tmpl];
  const int side = 2 * radius + 1, area = side * side;
  const int total = n_cand * area;
  const int band_keys = pd.nv * 16;  // keys per column band
  int np = 1;
  while (np < total) np <<= 1;
  double *const num = reinterpret_cast<double *>(dyn);
  int *const list = reinterpret_cast<int *>(dyn + 2 * kRefineChunk);
  uint32_t *const region = dyn + 2 * kRefineChunk + np;
  // entries are (v << 16 | u) when both fit 16 bits, else the row-major index
  const bool packed = pd.nu <= 65536 && pd.nv <= 65536;
  int L = 0;
  auto to_entry = [&](int u, int v) { return packed ? (v << 16) | u : v * pd.nu + u; };
  if (n_cand <= 64) {
    // the candidates, ordered by (column band of 16, v, u) with a bitonic sort
    // in wave 0's lanes (k <= 64); invalid candidates sort last
    if (wave == 0) {
      int key = 0x7fffffff;
      if (lane < n_cand) {
        const sncc_match c = cand[(long long)p * n_cand + lane];
        if (c.u >= 0) key = (c.u >> 4) * band_keys + c.v * 16 + (c.u & 15);
      }
      for (int size = 2; size <= 64; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
          const int other = __shfl_xor(key, stride);
          const bool up = (lane & size) == 0, low = (lane & stride) == 0;
          key = (low == up) ? min(key, other) : max(key, other);
        }
      int cu = -1, cv = -1;
      if (key != 0x7fffffff) {
        const int band = key / band_keys, rem = key - band * band_keys;
        cv = rem >> 4;
        cu = band * 16 + (rem & 15);
      }
      if (lane < n_cand) {
        cand_u[lane] = cu;
        cand_v[lane] = cv;
      }
    }
    __syncthreads();
    // the union of the neighbourhoods: an offset is listed by the first
    // candidate (in that order) whose neighbourhood holds it, so every offset
    // once; entries follow the candidates, each neighbourhood row by row
    for (int e0 = 0; e0 < total; e0 += kRefineThreads) {
      const int e = e0 + tid;
      int u = 0, v = 0;
      bool own = false;
      if (e < total) {
        const int j = e / area, d = e - j * area;
        const int cu = cand_u[j], cv = cand_v[j];
        u = cu + d % side - radius;
        v = cv + d / side - radius;
        own = cu >= 0 && u >= 0 && u < pd.nu && v >= 0 && v < pd.nv;
        for (int i = 0; own && i < j; ++i)
          own = !(abs(u - cand_u[i]) <= radius && abs(v - cand_v[i]) <= radius);
      }
      const uint32_t incl = wave_incl_scan(own ? 1u : 0u);
      if (lane == 63) wsum[wave] = (int)incl;
      __syncthreads();
      int pos = L + (int)incl - (own ? 1 : 0), add = 0;
      for (int w = 0; w < kRefineWaves; ++w) {
        pos += w < wave ? wsum[w] : 0;
        add += wsum[w];
      }
      if (own) list[pos] = to_entry(u, v);
      L += add;
      __syncthreads();  // wsum is rewritten by the next round
    }
  } else {
    // more candidates than a wave's lanes: the neighbourhoods' keys (band, v,
    // u) are sorted (bitonic, in LDS) and made unique, then rewritten as
    // entries in place
    for (int e = tid; e < np; e += kRefineThreads) {
      int val = 0x7fffffff;
      if (e < total) {
        const int j = e / area, d = e - j * area;
        const sncc_match c = cand[(long long)p * n_cand + j];
        const int u = c.u + d % side - radius, v = c.v + d / side - radius;
        if (c.u >= 0 && u >= 0 && u < pd.nu && v >= 0 && v < pd.nv)
          val = (u >> 4) * band_keys + v * 16 + (u & 15);
      }
      list[e] = val;
    }
    __syncthreads();
    for (int size = 2; size <= np; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = tid; i < np; i += kRefineThreads) {
          const int j = i ^ stride;
          if (j > i) {
            const int x = list[i], y = list[j];
            const bool up = (i & size) == 0;
            if ((x > y) == up) {
              list[i] = y;
              list[j] = x;
            }
          }
        }
        __syncthreads();
      }
    // unique keys: each thread owns a contiguous run of the sorted list (at
    // most 4096 / kRefineThreads = 8 entries)
    const int per = (np + kRefineThreads - 1) / kRefineThreads;
    const int r0 = min(np, tid * per), r1 = min(np, r0 + per);
    int mine[8];
    int m = 0;
    for (int i = r0; i < r1; ++i)
      if (list[i] != 0x7fffffff && (i == 0 || list[i] != list[i - 1])) {
        const int key = list[i];
        const int band = key / band_keys, rem = key - band * band_keys;
        mine[m++] = to_entry(band * 16 + (rem & 15), rem >> 4);
      }
    const uint32_t incl = wave_incl_scan((uint32_t)m);
    if (lane == 63) wsum[wave] = (int)incl;
    __syncthreads();
    int off = (int)incl - m;
    for (int w = 0; w < wave; ++w) off += wsum[w];
    for (int w = 0; w < kRefineWaves; ++w) L += wsum[w];
    __syncthreads();  // every run read before the list is compacted in place
    for (int q = 0; q < m; ++q) list[off + q] = mine[q];
    __syncthreads();
  }
  // FP64 scores with the fine approximation, chunk by chunk
  const uint32_t *S = s + (long long)pd.frame * frame_stride;
  const uint32_t *S2 = s2 + (long long)pd.frame * frame_stride;
  const uint32_t bytes = (uint32_t)(frame_stride * 4);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(S, bytes);
  const __amdgpu_buffer_rsrc_t rs2 = make_rsrc(S2, bytes);
  const int P4 = P * 4;
  auto entry = [&](int i, int &u, int &v) {
    const int x = list[i];
    if (packed) {
      u = x & 0xffff;
      v = (int)((uint32_t)x >> 16);
    } else {
      v = x / pd.nu;
      u = x - v * pd.nu;
    }
  };
  double br = -__builtin_inf();
  int bi = 0x7fffffff;
  auto offer = [&](double r, int idx) {
    if (r > br || (r == br && idx < bi)) {
      br = r;
      bi = idx;
    }
  };
  if (st.tbl < 0) {  // region too large for LDS: one offset per thread
    for (int i = tid; i < L; i += kRefineThreads) {
      int u, v;
      entry(i, u, v);
      bool flat;
      const double r = rho_plain(S, S2, P, u, v, td.W, td.H, td.K, td.sq_rows, td.q_k, td.r64,
                                 geom + td.seg_off, c64 + td.seg_off, flat);
      offer(r, v * pd.nu + u);
    }
  }
  // chunks: runs of at most kRefineChunk consecutive entries whose offsets
  // span at most the template's region spans (its pitch less W + 1 columns,
  // its rows less H), cut greedily in list order by wave 0, which reads the
  // entries 64 at a time into lanes and walks them with lane reads (the
  // serial walk waits on no LDS read)
  for (int i = tid; i < REFINE_CAP / 32; i += kRefineThreads) first[i] = 0;
  __syncthreads();
  const int span_u = st.pitch - td.W - 1, span_v = st.rows - td.H;
  if (wave == 0) {
    int c0 = 0, umin = 0, umax = 0, vmin = 0, vmax = 0;
    for (int i0 = 0; i0 < L; i0 += 64) {
      int lu = 0, lv = 0;
      if (i0 + lane < L) entry(i0 + lane, lu, lv);
      const int n64 = min(64, L - i0);
      uint64_t starts = 0;
      for (int q = 0; q < n64; ++q) {
        const int i = i0 + q;
        const int u = __builtin_amdgcn_readlane(lu, q), v = __builtin_amdgcn_readlane(lv, q);
        if (i == c0 || i - c0 == kRefineChunk || max(umax, u) - min(umin, u) >= span_u ||
            max(vmax, v) - min(vmin, v) >= span_v) {
          starts |= 1ull << q;
          c0 = i;
          umin = umax = u;
          vmin = vmax = v;
        } else {
          umin = min(umin, u);
          umax = max(umax, u);
          vmin = min(vmin, v);
          vmax = max(vmax, v);
        }
      }
      if (lane < 2) first[(i0 >> 5) + lane] = (uint32_t)(starts >> (32 * lane));
    }
  }
  __syncthreads();
  auto chunk_end = [&](int c0) {  // the next chunk's first entry, or L
    for (int i = c0 + 1; i < L;) {
      const uint32_t w = first[i >> 5] >> (i & 31);
      if (w) return min(L, i + __builtin_ctz(w));
      i = (i | 31) + 1;
    }
    return L;
  };
  for (int c0 = 0; st.tbl >= 0 && c0 < L;) {
    const int c1 = __builtin_amdgcn_readfirstlane(chunk_end(c0));
    const int n = c1 - c0;  // at most kRefineChunk = 128: lane i takes entries c0 + i, + 64
    // bounds by wave maxima (the minima as maxima of complements; absent
    // entries give 0 to every maximum)
    uint32_t mu = 0, mv = 0, nu_ = 0, nv_ = 0;
    for (int i = lane; i < n; i += 64) {
      int eu, ev;
      entry(c0 + i, eu, ev);
      mu = max(mu, (uint32_t)eu);
      mv = max(mv, (uint32_t)ev);
      nu_ = max(nu_, ~(uint32_t)eu);
      nv_ = max(nv_, ~(uint32_t)ev);
    }
    const int umax = (int)__builtin_amdgcn_readlane((int)wave_incl_max(mu), 63);
    const int vmax = (int)__builtin_amdgcn_readlane((int)wave_incl_max(mv), 63);
    const int umin = (int)~__builtin_amdgcn_readlane((int)wave_incl_max(nu_), 63);
    const int vmin = (int)~__builtin_amdgcn_readlane((int)wave_incl_max(nv_), 63);
    // the entries the chunk's windows read: rows [vmin, vmax + H], columns
    // [umin, umax + W] of the table, at the region's pitch
    const int nrow = vmax - vmin + td.H + 1, ncol = umax - umin + td.W + 1;
    stage_region(rs, P, N, vmin, umin, nrow, ncol, st.pitch, region, wave, lane, kRefineWaves);
    region_relative(rs, P, N, vmin, umin, region, nrow, ncol, st.pitch, wave, lane, kRefineWaves);
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rso = make_rsrc(slot_off + st.tbl, (uint32_t)st.n_iter * 256u);
    const __amdgpu_buffer_rsrc_t rsw = make_rsrc(slot_w + st.tbl, (uint32_t)st.n_iter * 512u);
    for (int e0 = wave * 4; e0 < n; e0 += 4 * kRefineWaves) {  // four entries per wave
      int base[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int su, sv;
        entry(c0 + min(e0 + j, n - 1), su, sv);
        base[j] = ((sv - vmin) * st.pitch + (su - umin)) * 4;
      }
      // lane j < 4 holds the sum of entry c0 + e0 + j
      const double sum = consecutive4(base)
                             ? staged_num4<true, false>(region, base, rso, rsw, st.n_iter, lane)
                             : staged_num4<false, false>(region, base, rso, rsw, st.n_iter, lane);
      if (lane < 4 && e0 + lane < n) num[e0 + lane] = sum;
    }
    __syncthreads();
    // rho of the chunk's entries, one per thread: the window sums and the
    // division are a lane's work, not a wave's per four windows
    for (int i = tid; i < n; i += kRefineThreads) {
      int u, v;
      entry(c0 + i, u, v);
      const int q = ((v - vmin) * st.pitch + (u - umin)) * 4;
      offer(staged_rho(num[i], region, st.pitch, q, v * P4 + u * 4, rs2, P4, td), v * pd.nu + u);
    }
    __syncthreads();  // the region and the sums are rewritten for the next chunk
    c0 = c1;
  }
  for (int msk = 32; msk >= 1; msk >>= 1) {
    const double orr = __shfl_xor(br, msk);
    const int oi = __shfl_xor(bi, msk);
    if (orr > br || (orr == br && oi < bi)) {
      br = orr;
      bi = oi;
    }
  }
  if (lane == 0) {
    best_r[wave] = br;
    best_i[wave] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < kRefineWaves; ++w)
      if (best_r[w] > br || (best_r[w] == br && best_i[w] < bi)) {
        br = best_r[w];
        bi = best_i[w];
      }
    sncc_match64 o;
    if (L == 0) {
      o.u = -1;
      o.v = -1;
      o.rho = -__builtin_inf();
    } else {
      o.v = bi / pd.nu;
      o.u = bi - o.v * pd.nu;
      o.rho = br;
    }
    out[p] = o;
    if (count) count[p] = L;
  }
}

int refine_region_budget(int np, int wgs) {
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, (const void *)refine_kernel) != hipSuccess) return 0;
  const long long left = (long long)kTileMaxLds / std::max(1, wgs) - (long long)fa.sharedSizeBytes -
                         kRefineChunk * 8 - (long long)np * 4;
  return left > 0 ? (int)left : 0;
}

int launch_refine(const uint32_t *s, const uint32_t *s2, long long frame_stride, int P,
                  const DevTmpl *tmpls, const int4 *geom, const double *c64,
                  const SlotTables &slots, const PairDesc *pairs, int n_pairs,
                  const sncc_match *cand, int n_cand, int radius, sncc_match64 *out, int *count,
                  hipStream_t st) {
  const int total = n_cand * (2 * radius + 1) * (2 * radius + 1);
  if (total > REFINE_CAP) return -1;
  int np = 1;
  while (np < total) np <<= 1;
  const int N = (int)(frame_stride / P) - 1;
  const int fixed = kRefineChunk * 8 + np * 4;
  auto go = [&](int first, int n, int region_bytes) {
    if (n <= 0) return;
    hipLaunchKernelGGL(refine_kernel, dim3(n), dim3(kRefineThreads), fixed + region_bytes, st, s,
                       s2, frame_stride, P, tmpls, geom, c64, slots.tmpl, slots.off, slots.w,
                       pairs, slots.order ? slots.order + first : nullptr, cand, n_cand, radius,
                       N, out, count);
  };
  if (slots.order) {
    go(0, slots.n_first, slots.lds_first);
    go(slots.n_first, n_pairs - slots.n_first, slots.lds_bytes);
  } else {
    go(0, n_pairs, slots.lds_bytes);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sncc
