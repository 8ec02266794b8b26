// The persistent scoring kernel (Eqs. (11)-(18)), templated on the tile
// shape: RU x RV offsets per lane, NW waves, LDS row pitch LP (words; 0 for
// the direct form that reads corners from the global table) and the sink
// (rho map, per-item top-k partials, or a compacted survivor list).  Each tile shape is compiled in
// its own translation unit (tile_entry.hip).
#pragma once

#include "device_util.hpp"

namespace sncc {

static_assert(kNumLpClasses == 11, "the LP-class switch in tile_kernel lists 11 cases");

// Stages the pass's row intervals of one frame's sum table into LDS with
// LDS-direct buffer loads: lane c4 of a wave moves 16 bytes of a row.  Rows
// below the table's last row (N) and 16-byte chunks past its pitch are not
// read: only offsets outside the valid range would use them, and those are
// masked, so every load stays inside the frame's table.
template <int LP, int NW>
__device__ __forceinline__ void stage_pass(__amdgpu_buffer_rsrc_t rs, int P, int N,
                                           const Interval *__restrict__ ivs, int iv_begin,
                                           int iv_end, int u0, int v0, int stage_w4,
                                           uint32_t *lds, int wave, int lane) {
  const int w4 = min(stage_w4, (P - u0) >> 2);  // P and u0 are multiples of 4
  for (int iv = iv_begin; iv < iv_end; ++iv) {
    const Interval I = ivs[iv];
    const int rows = min(I.n_rows, N + 1 - (v0 + I.rel_row));
    for (int j = wave; j < rows; j += NW) {
      const int src = ((v0 + I.rel_row + j) * P + u0) * 4;
      uint32_t *dst = lds + (I.lds_row + j) * LP;
#pragma unroll
      for (int c = 0; c < (LP / 4 + 63) / 64; ++c) {
        if (c * 64 + lane < w4)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rs, (__attribute__((address_space(3))) void *)(dst + c * 256), 16,
              lane * 16 + c * 1024, src, 0, 0);
      }
    }
  }
}

// NC horizontal chains of L segments each (records rp[c (L + 1) + j]) for
// the lane's RU x RV offsets.  Per boundary column the difference of the
// chain's bottom and top rows is read once (two LDS reads); a segment's box
// sum (Eq. (11), exact modulo 2^32) is the difference of its right and left
// columns' values, G_i = F_i - A_i b in integers, and the products G_i c_i of
// the block are summed in FP32 before one compensated (Kahan) addition per
// offset.  `base` is the lane's LDS origin.
template <int RU, int RV, int LP, int L, int NC>
__device__ __forceinline__ void chain_block(const TileRec *__restrict__ rp, const uint32_t *base,
                                            const int (&nb)[RU * RV], float (&acc)[RU * RV],
                                            float (&cmp)[RU * RV]) {
  constexpr int NI = L + 1;
  const uint32_t *tp[NC][NI], *bp[NC][NI];
  int A[NC][NI];
  float c[NC][NI];
#pragma unroll
  for (int ch = 0; ch < NC; ++ch)
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const TileRec e = rp[ch * NI + j];
      tp[ch][j] = base + e.off_tl;
      bp[ch][j] = base + e.off_bl;
      A[ch][j] = e.w_area;
      c[ch][j] = e.c;
    }
#pragma unroll
  for (int dv = 0; dv < RV; ++dv)
#pragma unroll
    for (int du = 0; du < RU; ++du) {
      const int o = dv * LP + du * 64;
      const int r = dv * RU + du;
      float y = -cmp[r];
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) {
        uint32_t prev = bp[ch][0][o] - tp[ch][0][o];
#pragma unroll
        for (int j = 1; j < NI; ++j) {
          const uint32_t cur = bp[ch][j][o] - tp[ch][j][o];
          const uint32_t F = cur - prev;
          const int G = (int)F + __mul24(A[ch][j], nb[r]);
          y = __builtin_fmaf((float)G, c[ch][j], y);
          prev = cur;
        }
      }
      const float t = acc[r] + y;
      cmp[r] = (t - acc[r]) - y;
      acc[r] = t;
    }
}

template <int RU, int RV, int NW, int LP, int SINK>
__device__ __forceinline__ void run_item(
    const uint32_t *__restrict__ s, const uint32_t *__restrict__ s2, long long frame_stride,
    int P, int N, const PassDesc *__restrict__ passes, const Interval *__restrict__ ivs,
    const TileRec *__restrict__ recs, const WorkItem &it, const PairDesc &pd,
    const DevTmpl &td, u64 &lkey, int k, float *__restrict__ rho_out, int rho_pitch,
    uint8_t *__restrict__ degen, uint32_t *lds, float *scl, uint32_t *thr_sh,
    const CompactOut &co, int wave, int lane) {
  constexpr int BU = 64 * RU, BV = NW * RV, R = RU * RV;
  // per-offset scales live in LDS (thread-private slots) from the prologue to
  // the epilogue, which keeps them out of registers during the segment loop
  float *const my_sc = scl + wave * 64 + lane;
  const uint32_t bytes = (uint32_t)(N + 1) * (uint32_t)P * 4u;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(s + (long long)pd.frame * frame_stride, bytes);
  const __amdgpu_buffer_rsrc_t rs2 = make_rsrc(s2 + (long long)pd.frame * frame_stride, bytes);
  const int W = td.W, H = td.H, n = td.n;
  const float inv_n = 1.0f / (float)n;
  const double qnd = td.q_k / (double)n;  // energy * q_k = V * q_k / n
  const bool one_box = n <= kMaxSqBoxArea;
  const int lbase = wave * RV * LP + lane;
  const int cW = W * 4, cH = H * P * 4;  // byte offsets of the window corners

  for (int tile = it.tile_begin; tile < it.tile_end; ++tile) {
    const int tv = tile / pd.ntu, tu = tile - tv * pd.ntu;
    const int u0 = pd.u_base + tu * BU, v0 = tv * BV;

    // the first pass's rows are requested before the prologue's loads so
    // that both latencies overlap
    if constexpr (LP != 0) {
      __syncthreads();
      const PassDesc ps = passes[td.pass_begin];
      stage_pass<LP, NW>(rs, P, N, ivs, ps.iv_begin, ps.iv_end, u0 + ps.col0, v0, ps.stage_w4,
                         lds, wave, lane);
    }

    // per offset: window sums of f and f^2 (Eqs. (13), (15)), the integer
    // bias, and the scale 1 / sqrt(V q_k / n) from the exact window energy
    // V = n * Eq. (16) in 64-bit integers (0 when V = 0).  The loads are
    // issued before the first staging wait so that their latency overlaps
    // it; offsets outside the valid range read the window of the nearest
    // valid offset (inside the table) and are masked in the epilogue
    // byte offsets of the lane's windows in the table: a wave-uniform row
    // part (scalar) and a per-lane column part, clamped to the valid range
    int rowo[RV], colo[RU];
#pragma unroll
    for (int dv = 0; dv < RV; ++dv) rowo[dv] = min(v0 + wave * RV + dv, pd.nv - 1) * P * 4;
#pragma unroll
    for (int du = 0; du < RU; ++du) colo[du] = min(u0 + lane + 64 * du, pd.nu - 1) * 4;
    int nb[R];
    float acc[R], cmp[R];
    if (one_box) {
      // one exact box per window: V = n * sum f^2 - (sum f)^2 as one FP64 fma
      // of integers below 2^53, hence exact.  The corner loads of two offsets
      // at a time are issued before any is used, so that their latencies
      // overlap; larger batches push a value live across the item into
      // scratch memory, a store per wave and item
      constexpr int RH = R > 2 ? 2 : R;  // offsets per batch of loads
#pragma unroll
      for (int h = 0; h < R; h += RH) {
        uint32_t c1[RH][4], c2[RH][4];
#pragma unroll
        for (int j = 0; j < RH; ++j) {
          const int r = h + j, dv = r / RU, du = r % RU;
          window_corners(rs, colo[du], rowo[dv], cW, cH, c1[j]);
          window_corners(rs2, colo[du], rowo[dv], cW, cH, c2[j]);
        }
#pragma unroll
        for (int j = 0; j < RH; ++j) {
          const int r = h + j;
          const uint32_t sf = (c1[j][3] - c1[j][2]) - (c1[j][1] - c1[j][0]);   // Eq. (13)
          const uint32_t sf2 = (c2[j][3] - c2[j][2]) - (c2[j][1] - c2[j][0]);  // Eq. (15)
          nb[r] = -(int)__builtin_rintf((float)sf * inv_n);
          const double fs = (double)sf;
          const double Vd = __builtin_fma((double)n, (double)sf2, -(fs * fs));
          my_sc[r * NW * 64] = Vd == 0.0 ? 0.f : __builtin_amdgcn_rsqf((float)(Vd * qnd));
          acc[r] = 0.f;
          cmp[r] = 0.f;
        }
      }
    } else {
      // banded sum of f^2; V in 64-bit integers
#pragma unroll
      for (int dv = 0; dv < RV; ++dv)
#pragma unroll
        for (int du = 0; du < RU; ++du) {
          const int r = dv * RU + du;
          const uint32_t sf = window_box(rs, colo[du], rowo[dv], cW, cH);
          const u64 sf2 = window_sq(rs2, colo[du], rowo[dv], cW, P * 4, H, td.sq_rows);
          nb[r] = -(int)__builtin_rintf((float)sf * inv_n);
          const u64 V = (u64)(uint32_t)n * sf2 - (u64)sf * sf;
          const float x = (float)((double)V * qnd);
          my_sc[r * NW * 64] = V == 0 ? 0.f : __builtin_amdgcn_rsqf(x);
          acc[r] = 0.f;
          cmp[r] = 0.f;
        }
    }

    if constexpr (LP == 0) {
      // direct form: the template's horizontal chains from the global table,
      // one record per boundary column (see plan_direct): buffer loads with
      // the column's top and bottom entries as scalar offsets give its
      // difference D; a segment's F_i (Eq. (11)) is D minus the previous
      // column's D, then the staged form's arithmetic, four records per
      // compensated step (first columns add A = c = 0; the list is padded
      // to whole groups with records that add zero).  The next record's
      // entries are requested before the current record's are used
      const PassDesc ps = passes[td.pass_begin];
      const DirectRec *dp = reinterpret_cast<const DirectRec *>(recs + ps.seg_begin);
      const int nrec = (ps.seg_end - ps.seg_begin) >> 1;
      int vb[R];
#pragma unroll
      for (int dv = 0; dv < RV; ++dv)
#pragma unroll
        for (int du = 0; du < RU; ++du) {
          vb[dv * RU + du] = rowo[dv] + colo[du];
        }
      uint32_t at[R], ab[R], nt[R], nbt[R], dprev[R];
#pragma unroll
      for (int r = 0; r < R; ++r) dprev[r] = 0;
      auto column = [&](const DirectRec &e, uint32_t(&ct)[R], uint32_t(&cb)[R]) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          ct[r] = __builtin_amdgcn_raw_buffer_load_b32(rs, vb[r], e.top, 0);
          cb[r] = __builtin_amdgcn_raw_buffer_load_b32(rs, vb[r], e.bot, 0);
        }
      };
      if (nrec > 0) column(dp[0], at, ab);
      for (int i = 0; i < nrec; i += 4) {
        float y[R];
#pragma unroll
        for (int r = 0; r < R; ++r) y[r] = -cmp[r];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const DirectRec e = dp[i + q];
          column(dp[min(i + q + 1, nrec - 1)], nt, nbt);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const uint32_t D = ab[r] - at[r];
            const uint32_t F = D - dprev[r];  // Eq. (11)
            dprev[r] = D;
            const int G = (int)F + __mul24(e.area, nb[r]);
            y[r] = __builtin_fmaf((float)G, e.c, y[r]);
            at[r] = nt[r];
            ab[r] = nbt[r];
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float t = acc[r] + y[r];
          cmp[r] = (t - acc[r]) - y[r];
          acc[r] = t;
        }
      }
    } else {
    // per-segment terms (Eqs. (11), (12)), pass by pass; the products of four
    // segments are added before one compensated (Kahan) step
    for (int p = td.pass_begin; p < td.pass_end; ++p) {
      const PassDesc ps = passes[p];
      if (p != td.pass_begin) {
        __syncthreads();
        stage_pass<LP, NW>(rs, P, N, ivs, ps.iv_begin, ps.iv_end, u0 + ps.col0, v0,
                           ps.stage_w4, lds, wave, lane);
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      // chains grouped by length, about four segments per compensated step
      const TileRec *rp = recs + ps.seg_begin;
      for (int q = ps.n_chain[3]; q > 0; --q, rp += 5)
        chain_block<RU, RV, LP, 4, 1>(rp, lds + lbase, nb, acc, cmp);
      for (int q = ps.n_chain[2]; q > 0; --q, rp += 4)
        chain_block<RU, RV, LP, 3, 1>(rp, lds + lbase, nb, acc, cmp);
      int q2 = ps.n_chain[1];
      for (; q2 >= 2; q2 -= 2, rp += 6) chain_block<RU, RV, LP, 2, 2>(rp, lds + lbase, nb, acc, cmp);
      if (q2) {
        chain_block<RU, RV, LP, 2, 1>(rp, lds + lbase, nb, acc, cmp);
        rp += 3;
      }
      int q1 = ps.n_chain[0];
      for (; q1 >= 4; q1 -= 4, rp += 8) chain_block<RU, RV, LP, 1, 4>(rp, lds + lbase, nb, acc, cmp);
      for (; q1 > 0; --q1, rp += 2) chain_block<RU, RV, LP, 1, 1>(rp, lds + lbase, nb, acc, cmp);
    }
    }  // staged form

    // epilogue: rho = num / sqrt(V q_k / n) (Eqs. (17), (18)) in FP32
    if (SINK == kSinkMap) {
#pragma unroll
      for (int dv = 0; dv < RV; ++dv)
#pragma unroll
        for (int du = 0; du < RU; ++du) {
          const int r = dv * RU + du;
          const int u = u0 + lane + 64 * du, v = v0 + wave * RV + dv;
          const float sc = my_sc[r * NW * 64];
          if (u < pd.nu && v < pd.nv) {
            rho_out[(long long)v * rho_pitch + u] = (acc[r] - cmp[r]) * sc;
            if (degen) degen[(long long)v * rho_pitch + u] = sc == 0.f ? 1 : 0;
          }
        }
    } else if (SINK == kSinkCompact) {
      // offsets whose rho reaches the template's threshold are appended to
      // the survivor list with one atomic per wave, ordered by column group
      // (du, then kRunCols lanes at a time), then dv, then lane, so that
      // neighbouring entries are neighbouring offsets of one row; the wave's
      // entries of each group of kRunCols columns form a run
      constexpr int G = 64 / kRunCols, NQ = G * RU;
      constexpr u64 kGroup = kRunCols == 64 ? ~0ull : (1ull << kRunCols) - 1ull;
      u64 m[R];
      int cnt[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) cnt[q] = 0;
#pragma unroll
      for (int dv = 0; dv < RV; ++dv)
#pragma unroll
        for (int du = 0; du < RU; ++du) {
          const int r = dv * RU + du;
          const int u = u0 + lane + 64 * du, v = v0 + wave * RV + dv;
          acc[r] = (acc[r] - cmp[r]) * my_sc[r * NW * 64];  // acc now holds rho
          m[r] = __ballot(u < pd.nu && v < pd.nv && acc[r] >= td.thr);
#pragma unroll
          for (int g = 0; g < G; ++g) cnt[G * du + g] += __popcll(m[r] & (kGroup << (kRunCols * g)));
        }
      int total = 0, n_runs = 0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        total += cnt[q];
        n_runs += cnt[q] > 0;
      }
      if (total > 0) {
        int base = 0;
        if (lane == 0) {
          base = atomicAdd(co.count, total);
          int ri = atomicAdd(co.run_count, n_runs);
          int start = base;
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            if (cnt[q] > 0 && ri < co.run_cap) {
              RunDesc rd;
              rd.start = start;
              rd.count = cnt[q];
              rd.pair = it.pair;
              rd.u0 = u0 + kRunCols * q;
              rd.v0 = v0 + wave * RV;
              rd.pad[0] = rd.pad[1] = rd.pad[2] = 0;
              co.runs[ri] = rd;
            }
            ri += cnt[q] > 0;
            start += cnt[q];
          }
        }
        int pos = __builtin_amdgcn_readfirstlane(base);
        const u64 below = (1ull << lane) - 1ull;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int dv = 0; dv < RV; ++dv) {
            const int du = q / G, r = dv * RU + du;
            const u64 mq = m[r] & (kGroup << (kRunCols * (q % G)));
            if ((mq >> lane) & 1ull) {
              const int at = pos + __popcll(mq & below);
              if (at < co.cap) {
                sncc_hit h;
                h.pair = it.pair;
                h.u = u0 + lane + 64 * du;
                h.v = v0 + wave * RV + dv;
                h.reserved = 0;
                h.rho = (double)acc[r];
                co.hits[at] = h;
              }
            }
            pos += __popcll(mq);
          }
      }
    } else {
      // waves publish the high word of their k-th key (a 32-bit store, so
      // readers see an old or a new value, never a mix); (largest, 0) is at
      // most some wave's k-th key and filters every wave.  A float test
      // against that high word (never stricter than the key test) skips key
      // building for tiles with no candidate
      uint32_t fh = (uint32_t)(lane_u64(lkey, k - 1) >> 32);
#pragma unroll
      for (int w = 0; w < NW; ++w) fh = max(fh, thr_sh[w]);
      const float fth = fh <= 0x007fffffu ? -__builtin_inff() : float_unorder(fh);
      float rho[R];
      bool any = false;
#pragma unroll
      for (int dv = 0; dv < RV; ++dv)
#pragma unroll
        for (int du = 0; du < RU; ++du) {
          const int r = dv * RU + du;
          const int u = u0 + lane + 64 * du, v = v0 + wave * RV + dv;
          rho[r] = (u < pd.nu && v < pd.nv) ? (acc[r] - cmp[r]) * my_sc[r * NW * 64]
                                            : -__builtin_inff();
          any |= rho[r] >= fth;
        }
      if (__ballot(any) != 0) {
        u64 cand[R];
#pragma unroll
        for (int dv = 0; dv < RV; ++dv)
#pragma unroll
          for (int du = 0; du < RU; ++du) {
            const int r = dv * RU + du;
            const int u = u0 + lane + 64 * du, v = v0 + wave * RV + dv;
            cand[r] = rho[r] >= fth && rho[r] != -__builtin_inff()
                          ? make_key(rho[r], v * pd.nu + u) : 0;
          }
        // a few keys go into the list one by one (best first, so at most k
        // insertions); a larger batch with a larger k (a wave's first tiles)
        // through the sort-and-merge buffer, which takes the
        // wave's scale slots (read above for this tile; the next prologue
        // rewrites them): low words in r = 0's, high words in r = 1's
        const u64 fl = (u64)fh << 32;
        const u64 thr = max(lane_u64(lkey, k - 1), fl);
        int n = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) n += __popcll(__ballot(cand[r] > thr));
        if (n <= 2 || k <= 2) {
          topk_offer<R>(lkey, cand, k, lane, fl);
        } else {
          float *slot0 = scl + wave * 64;
          topk_offer_batched<R>(lkey, cand, k, lane, fl, slot0, slot0 + NW * 64);
        }
        if (lane == 0) thr_sh[wave] = (uint32_t)(lane_u64(lkey, k - 1) >> 32);
      }
    }
  }
}

template <int RU, int RV, int NW, int SINK>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) void tile_kernel(
    const uint32_t *__restrict__ s, const uint32_t *__restrict__ s2, long long frame_stride,
    int P, int N, const DevTmpl *__restrict__ tmpls, const PassDesc *__restrict__ passes,
    const Interval *__restrict__ ivs, const TileRec *__restrict__ recs,
    const PairDesc *__restrict__ pairs, const WorkItem *__restrict__ items,
    const int *__restrict__ order, const int *__restrict__ qbeg, int nq,
    int *__restrict__ queue, int k, u64 *__restrict__ partial, u64 *__restrict__ pair_floor,
    float *__restrict__ rho_out, int rho_pitch, uint8_t *__restrict__ degen, CompactOut co) {
  // dynamic LDS: per-offset scales (R words per thread), then the staged rows
  extern __shared__ __align__(16) uint32_t lds[];
  constexpr int kScaleWords = 64 * NW * RU * RV;
  __shared__ int item_sh;
  __shared__ uint32_t thr_sh[NW];  // high words of the waves' k-th keys (current item)
  // the wave index is made a scalar, so that what derives from it is too
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  // Work queues: queue j holds order[qbeg[j] .. qbeg[j + 1]) and its counter
  // sits at queue[16 j].  A workgroup drains the queue of the chiplet (XCD)
  // it runs on, whose L2 then holds the frame rows that queue's items share,
  // and then the others in turn; every workgroup leaves once it has found
  // all queues empty.  nq == 0: the grid has one workgroup per item, and
  // workgroup b runs order[b] and leaves (no counters: a small launch would
  // otherwise end with each workgroup's round of atomics over every queue).
  const int home = (int)(__builtin_amdgcn_s_getreg(20 | (3 << 11)) & 15) % max(nq, 1);
  int tried = 0;  // queues found empty (thread 0)
  for (;;) {
    if (threadIdx.x == 0) {
      int got = -1;
      if (nq == 0 && tried++ == 0) got = order[blockIdx.x];
      while (tried < nq) {
        const int qq = (home + tried) % nq;
        const int i = atomicAdd(queue + 16 * qq, 1);
        if (i < qbeg[qq + 1] - qbeg[qq]) {
          got = order[qbeg[qq] + i];
          break;
        }
        ++tried;
      }
      item_sh = got;
      // a key below the k-th key of another item of the same pair cannot be
      // in the pair's top k; items publish theirs when they finish.  Every
      // wave's threshold word starts from that floor (no wave reads these
      // words any more: the previous item's merge passed a barrier).  With
      // one workgroup per item (nq == 0) the items run at once and the floors
      // are neither read nor published, so they need no reset
      uint32_t fl = 0;
      if (SINK == kSinkTopk && got >= 0 && nq != 0)
        fl = (uint32_t)(__hip_atomic_load(pair_floor + items[got].pair, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) >> 32);
      for (int w = 0; w < NW; ++w) thr_sh[w] = fl;
    }
    __syncthreads();
    const int item = item_sh;
    __syncthreads();
    if (item < 0) break;
    const WorkItem it = items[item];
    const PairDesc pd = pairs[it.pair];
    const DevTmpl td = tmpls[pd.tmpl];
    u64 lkey = 0;
#define SNCC_RUN(LPV)                                                                    \
  run_item<RU, RV, NW, LPV, SINK>(s, s2, frame_stride, P, N, passes, ivs, recs, it, pd, td, \
                                 lkey, k, rho_out, rho_pitch, degen, lds + kScaleWords,      \
                                 reinterpret_cast<float *>(lds), thr_sh, co, wave, lane)
    switch (td.lp_class) {
      case 0: SNCC_RUN(kLpClasses[0]); break;
      case 1: SNCC_RUN(kLpClasses[1]); break;
      case 2: SNCC_RUN(kLpClasses[2]); break;
      case 3: SNCC_RUN(kLpClasses[3]); break;
      case 4: SNCC_RUN(kLpClasses[4]); break;
      case 5: SNCC_RUN(kLpClasses[5]); break;
      case 6: SNCC_RUN(kLpClasses[6]); break;
      case 7: SNCC_RUN(kLpClasses[7]); break;
      case 8: SNCC_RUN(kLpClasses[8]); break;
      case 9: SNCC_RUN(kLpClasses[9]); break;
      case 10: SNCC_RUN(kLpClasses[10]); break;
      default: SNCC_RUN(0); break;  // direct form
    }
#undef SNCC_RUN
    if (SINK == kSinkTopk) {
      // merge the waves' lists into wave 0's and write the item's partial
      u64 *buf = reinterpret_cast<u64 *>(lds);
      __syncthreads();
      if (lane < k) buf[wave * k + lane] = lkey;
      __syncthreads();
      if (wave == 0) {
        // each wave's list is sorted: one bitonic merge per wave, or for a
        // small k insertions until a wave's next key falls short
        if (k >= 8) {
          for (int w = 1; w < NW; ++w)
            topk_merge_sorted(lkey, lane < k ? buf[w * k + lane] : 0ull, k, lane);
        } else {
          u64 thr = lane_u64(lkey, k - 1);
          for (int w = 1; w < NW; ++w)
            for (int j = 0; j < k; ++j) {
              const u64 key = buf[w * k + j];
              if (key <= thr) break;
              topk_insert(lkey, key, k, lane);
              thr = lane_u64(lkey, k - 1);
            }
        }
        if (lane < k) partial[(long long)item * k + lane] = lkey;
        const u64 kth = lane_u64(lkey, k - 1);
        if (lane == 0 && kth != 0 && nq != 0) atomicMax(pair_floor + it.pair, kth);
      }
    }
  }
}

}  // namespace sncc
