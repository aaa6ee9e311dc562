// Column-parallel interpolative decomposition of the segments of one level
// (Sections 4.1-4.2, stacked form of eq. (4.12)).
//
// One workgroup of NW wave64 handles one segment.  Lane j owns column j of
// the stacked coupling matrix [A_{n,c}; A_{c,n}^T] (NCOL columns per lane,
// so n <= 64 * NCOL), and the waves share its rows (row i belongs to wave
// i mod NW).  Column norms, Householder dot products and updates are then
// per-lane loops over rows with no cross-lane reduction; the pivot search is
// one wave reduction.  Pivoting never moves data: lane j keeps original
// column j, and a position -> column table records the order.
//
// Four tiers cover the segment sizes of a level:
//   A  NW = 1,  Y and row table in LDS (fine levels: thousands of segments)
//   B  NW = 4,  Y and row table in LDS (middle levels), two groups per CU
//   B2 the same kernel with up to 152 KB of LDS, one group per CU
//   C  NW = 8,  152 KB of LDS, for segments whose coupling rows exceed it:
//      the far rows and the row table in LDS when they leave room for
//      enough of Y, else in the segment's global scratch; Y, the
//      m = |N| + h rows of a pass, split: its first rows (at least min(m,
//      n), all that fit) in LDS, the rest in global scratch
// Segments wider than 128 columns take the block-cooperative kernel
// k_seg_id.  Every tier computes the same tier function, so each segment is
// handled by exactly one launch; tier A also writes the identity result of
// segments without an ID.
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "kernels_factor.hpp"
#include "layout.hpp"

namespace spalu {

constexpr int ID_MAXPROBES = 8;

// One row of the stacked coupling matrix.
struct IdRow {
  int64_t base;    // value-arena offset of the entry in column 0
  int32_t stride;  // value-arena step between columns
  int32_t vh;      // 2 * vertex + half (half 1: a row of A_{c,d}^T)
};

// Gaussian tile of one wave: the entries of a pair of sample rows for 64 far
// rows (one Philox draw per lane).
constexpr int ID_GTILE = 128;

// Bytes of one entry of the stacked matrix Y for factors stored with st
// bytes per value: FP32 storage keeps Y in FP32 (all arithmetic on it in
// FP64), FP64 storage in FP64.
__host__ __device__ inline int idc_ye(int st) { return st == 4 ? 4 : 8; }

// LDS bytes of one workgroup of a tier (rows_in_lds: Y, the far rows B_F in
// the storage type (st bytes) and the row table).
__host__ __device__ inline size_t idc_lds_bytes(int nw, int ncol, int n, int R, int st, bool rows_in_lds) {
  size_t b = 0;
  if (rows_in_lds) b += size_t(R) * n * (idc_ye(st) + st) + size_t(R) * (sizeof(IdRow) + 4);
  b += size_t(ID_MAXPROBES) * n * 8;              // probe rows
  b += size_t(nw) * ID_GTILE * 8;                 // Gaussian tiles
  b += size_t(2) * nw * 64 * ncol * 8;            // norm and dot partials
  b += size_t(2) * n * 4 + 16;                    // position <-> column
  return (b + 15) & ~size_t(15);
}

// LDS bytes of the far rows B_F (storage type), row table and row order of a
// segment with R coupling rows.
__host__ __device__ inline size_t idc_table_bytes(int n, int R, int st) {
  return ((size_t(R) * n * st + 15) & ~size_t(15)) + size_t(R) * sizeof(IdRow) + ((size_t(R) * 4 + 15) & ~size_t(15));
}

// Doubles of global scratch a tier-C segment uses (Y, B_F, then the row table
// and the row order).
__host__ __device__ inline size_t idc_scratch_doubles(int n, int R) {
  return 2 * size_t(R) * n + (size_t(R) * (sizeof(IdRow) + 4) + 7) / 8;
}

// Waves of a tier-B workgroup (two per CU) and of a tier-B2 workgroup (one
// per CU).
constexpr int ID_B_WAVES = 4;
constexpr int ID_B2_WAVES = 8;

struct IdTiers {
  int budget_a;   // LDS bytes of the tier-A launch
  int budget_b;   // LDS bytes of the tier-B launch (two groups per CU)
  int budget_b2;  // LDS bytes of the tier-B2 launch (one group per CU)
  int st;         // bytes of the storage type
  int lds_c;      // LDS bytes of the tier-C launch (Y of the passes that fit)
  int c_ydiv;     // tier C keeps its far rows and tables in LDS when they
                  // leave room for max(n, R / c_ydiv) rows of Y
};

// Tier of a segment that gets an ID, from its sizes (n columns, R rows):
// 1: tier A, 2: B, 3: B2, 4: C with the far rows and row tables in LDS
// (when they leave room there for max(n, R / c_ydiv) rows of Y), 6: C with
// them in global scratch, 5: block-cooperative kernel.
__host__ __device__ inline int id_tier_of_size(int n, int R, IdTiers t) {
  if (n <= 64 && idc_lds_bytes(1, 1, n, R, t.st, true) <= size_t(t.budget_a)) return 1;
  if (n <= 128 && idc_lds_bytes(ID_B_WAVES, 2, n, R, t.st, true) <= size_t(t.budget_b)) return 2;
  if (n <= 128 && idc_lds_bytes(ID_B2_WAVES, 2, n, R, t.st, true) <= size_t(t.budget_b2)) return 3;
  const int ry = R / t.c_ydiv;
  const size_t yrows = size_t(n > ry ? n : ry);
  if (n <= 128 && idc_lds_bytes(ID_B2_WAVES, 2, n, 0, t.st, false) + idc_table_bytes(n, R, t.st) +
                      yrows * n * idc_ye(t.st) <= size_t(t.lds_c))
    return 4;
  if (n <= 128) return 6;
  return 5;
}

// 0: no ID (identity: no coupling rows, compression off, or a start sample
// count below zero, which keeps the segment whole), else the tier of the
// sizes.
__device__ inline int id_tier(const DSeg& S, int n, int R, const IdParams& prm, int c, IdTiers t) {
  const bool do_id = (S.flags & SEG_REGULAR) && (S.flags & SEG_HAS_NBR) && prm.eps > 0.0 && n > 0;
  if (!do_id || R == 0) return 0;
  if (prm.h_init && prm.h_init[prm.seg_base + c] < 0) return 0;
  return id_tier_of_size(n, R, t);
}

// 64-bit value of lane src (two 32-bit shuffles).
__device__ inline int64_t shfl_i64(int64_t v, int src) {
  const int lo = __shfl(int(uint32_t(uint64_t(v))), src, 64);
  const int hi = __shfl(int(uint32_t(uint64_t(v) >> 32)), src, 64);
  return int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}

template <int NW>
__device__ inline void grp_sync() {
  if constexpr (NW == 1)
    wave_sync();
  else
    __syncthreads();
}

// Fetches rows [0, cnt) of the list (near rows order[p], then far rows
// order[R - 1 - f]): near row p goes to row p of Y (Ya below row yl, Yb from
// there on), far row f to BF[f * n + j].  One (row, column) entry per thread
// and step, so every load of a step is independent and in flight at once.
template <typename T, int NT, typename YE>
__device__ inline void idc_fetch(const T* __restrict__ varena, const IdRow* rows, const int* order, int R, int nN,
                                 int cnt, YE* Ya, YE* Yb, int yl, T* BF, int n) {
#pragma unroll 4
  for (int t = threadIdx.x; t < cnt * n; t += NT) {
    const int p = t / n, j = t - p * n;
    const bool near = p < nN;
    const IdRow m = rows[near ? order[p] : order[R - 1 - (p - nN)]];
    const T v = varena[m.base + int64_t(j) * m.stride];
    if (near)
      (p < yl ? Ya : Yb)[t] = YE(v);
    else
      BF[size_t(p - nN) * n + j] = v;
  }
}

// First row at or after lo that belongs to the same wave as row i0 (rows
// i0, i0 + NW, ...).
template <int NW>
__device__ inline int idc_next_row(int i0, int lo) {
  return i0 >= lo ? i0 : i0 + (lo - i0 + NW - 1) / NW * NW;
}

// Sum over this wave's rows i = i0, i0 + NW, ... < m of Y[i][a] * Y[i][b]
// (row-major, ld n); UR rows are loaded before their products are summed, so
// that many loads are in flight.
template <int NW, int UR, typename YE>
__device__ inline double idc_rowdot(const YE* Y, int n, int i0, int m, int a, int b) {
  double acc[UR];
#pragma unroll
  for (int u = 0; u < UR; ++u) acc[u] = 0.0;
  int i = i0;
  for (; i + (UR - 1) * NW < m; i += UR * NW) {
    double ya[UR], yb[UR];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      ya[u] = double(Y[size_t(i + u * NW) * n + a]);
      yb[u] = double(Y[size_t(i + u * NW) * n + b]);
    }
#pragma unroll
    for (int u = 0; u < UR; ++u) acc[u] += ya[u] * yb[u];
  }
  for (; i < m; i += NW) acc[0] += double(Y[size_t(i) * n + a]) * double(Y[size_t(i) * n + b]);
  double t = 0.0;
#pragma unroll
  for (int u = 0; u < UR; ++u) t += acc[u];
  return t;
}

// Y[i][col] -= f * Y[i][q] over this wave's rows i = i0, i0 + NW, ... < m
// (in FP64, stored in Y's type); returns the sum of the squares of the
// updated entries as stored.
template <int NW, int UR, typename YE>
__device__ inline double idc_rowaxpy(YE* Y, int n, int i0, int m, int col, int q, double f) {
  double acc[UR];
#pragma unroll
  for (int u = 0; u < UR; ++u) acc[u] = 0.0;
  int i = i0;
  for (; i + (UR - 1) * NW < m; i += UR * NW) {
    double yc[UR], yq[UR];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      yc[u] = double(Y[size_t(i + u * NW) * n + col]);
      yq[u] = double(Y[size_t(i + u * NW) * n + q]);
    }
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const YE y = YE(yc[u] - f * yq[u]);
      Y[size_t(i + u * NW) * n + col] = y;
      acc[u] += double(y) * double(y);
    }
  }
  for (; i < m; i += NW) {
    const YE y = YE(double(Y[size_t(i) * n + col]) - f * double(Y[size_t(i) * n + q]));
    Y[size_t(i) * n + col] = y;
    acc[0] += double(y) * double(y);
  }
  double t = 0.0;
#pragma unroll
  for (int u = 0; u < UR; ++u) t += acc[u];
  return t;
}

// Row table of the stacked coupling matrix of segment c, built by one wave:
// rows[r] (block offset, column stride, vertex and half) for r < R, and
// order[]: the near rows from the front, the far rows from the back (far row
// f is order[R - 1 - f]); s_cnt receives (|N|, |F|).  The near field is the
// neighbour DOFs within Chebyshev distance S.thr of the segment's box.  hm
// is the number of halves per neighbour: 2 (rows of A_{d,c} and of
// A_{c,d}^T), or 1 in the symmetric form (rows of A_{d,c} only).
__device__ inline void idc_row_table(const DSeg& S, const DSeg* segs, const DNbr* nbrs, const DBlk* blks,
                                     GridGeom g, const int32_t* iarena, const DLevelDyn& dyn, int n, int R,
                                     int hm, IdRow* rows, int* order, int* s_cnt) {
  const int lane = threadIdx.x & 63;
  int nN = 0, nF = 0, r0 = 0;
  const int nnb = S.nbr_end - S.nbr_begin;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  if (nnb <= 64) {
    // neighbour e = lane: its size, DOF list and block offsets, loaded
    // together; its rows start at rs (exclusive prefix sum of hm n_d).
    // Row r of the table (neighbour, half, index) is then found by each
    // lane from these, so the whole table costs one more trip to memory
    int nd_l = 0;
    int64_t io_l = 0, o0_l = 0, o1_l = 0;
    if (lane < nnb) {
      const DNbr nb = nbrs[S.nbr_begin + lane];
      nd_l = dyn.n[nb.d];
      io_l = segs[nb.d].ioff;
      o0_l = blks[nb.blk_dc].off;
      o1_l = blks[nb.blk_cd].off;
    }
    int rs = hm * nd_l;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(rs, o, 64);
      if (lane >= o) rs += t;
    }
    rs -= hm * nd_l;
    for (int rb = 0; rb < R; rb += 64) {
      const int r = rb + lane;
      const bool valid = r < R;
      int owner = 0;  // the last neighbour whose rows start at or before r
      for (int q = 1; q < nnb; ++q)
        if (r >= __shfl(rs, q, 64)) owner = q;
      const int nd = __shfl(nd_l, owner, 64), rr = r - __shfl(rs, owner, 64);
      const int half = rr >= nd ? 1 : 0, i = rr - half * nd;
      const int64_t io = shfl_i64(io_l, owner), off0 = shfl_i64(o0_l, owner), off1 = shfl_i64(o1_l, owner);
      int v = 0;
      bool near = false;
      if (valid) {
        v = iarena[io + i];
        int cv[3];
        vcoords(g, v, cv);
        int dist = 0;
        for (int a = 0; a < 3; ++a) {
          int da = S.lo[a] - cv[a];
          if (cv[a] - S.hi[a] > da) da = cv[a] - S.hi[a];
          if (da > dist) dist = da;
        }
        near = dist <= S.thr;
      }
      const uint64_t mn = __ballot(valid && near), mf = __ballot(valid && !near);
      if (valid) {
        IdRow m;
        m.base = half == 0 ? off0 + int64_t(i) * n : off1 + i;
        m.stride = half == 0 ? 1 : nd;
        m.vh = 2 * v + half;
        rows[r] = m;
        if (near)
          order[nN + __popcll(mn & below)] = r;
        else
          order[R - 1 - (nF + __popcll(mf & below))] = r;
      }
      nN += __popcll(mn);
      nF += __popcll(mf);
    }
  } else {
    for (int e = S.nbr_begin; e < S.nbr_end; ++e) {
      const DNbr nb = nbrs[e];
      const int nd = dyn.n[nb.d];
      const int32_t* dd = iarena + segs[nb.d].ioff;
      const int64_t off0 = blks[nb.blk_dc].off, off1 = blks[nb.blk_cd].off;
      for (int half = 0; half < hm; ++half) {
        for (int i0 = 0; i0 < nd; i0 += 64) {
          const int i = i0 + lane;
          const bool valid = i < nd;
          int v = 0;
          bool near = false;
          if (valid) {
            v = dd[i];
            int cv[3];
            vcoords(g, v, cv);
            int dist = 0;
            for (int a = 0; a < 3; ++a) {
              int da = S.lo[a] - cv[a];
              if (cv[a] - S.hi[a] > da) da = cv[a] - S.hi[a];
              if (da > dist) dist = da;
            }
            near = dist <= S.thr;
          }
          const uint64_t mn = __ballot(valid && near), mf = __ballot(valid && !near);
          if (valid) {
            const int r = r0 + half * nd + i;
            IdRow m;
            m.base = half == 0 ? off0 + int64_t(i) * n : off1 + i;
            m.stride = half == 0 ? 1 : nd;
            m.vh = 2 * v + half;
            rows[r] = m;
            if (near)
              order[nN + __popcll(mn & below)] = r;
            else
              order[R - 1 - (nF + __popcll(mf & below))] = r;
          }
          nN += __popcll(mn);
          nF += __popcll(mf);
        }
      }
      r0 += hm * nd;
    }
  }
  if (lane == 0) {
    s_cnt[0] = nN;
    s_cnt[1] = nF;
  }
}

template <typename T, int NW, int NCOL, bool YG, int TIER, bool TABS = false>
__global__ __launch_bounds__(64 * NW) void k_seg_id_cols(const DSeg* segs, int nseg, const DNbr* nbrs,
                                                         const DBlk* blks, GridGeom g, int32_t* iarena,
                                                         T* __restrict__ varena, double* __restrict__ scratch,
                                                         DLevelDyn dyn, IdParams prm, IdTiers tiers) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_cnt[2];
  __shared__ int s_acc;
  constexpr int NT = 64 * NW;
  constexpr int UR = YG ? 8 : 4;  // rows in flight per lane in the CPQR passes
  const int c = blockIdx.x;
  if (c >= nseg) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const DSeg S = segs[c];
  const int n = dyn.n[c];
  int R = 0;
  const int hm = prm.sym ? 1 : 2;  // halves of the coupling rows per neighbour
  for (int e = S.nbr_begin; e < S.nbr_end; ++e) R += hm * dyn.n[nbrs[e].d];
  const int tier = id_tier(S, n, R, prm, c, tiers);
  int32_t* dofs = iarena + S.ioff;
  int32_t* perm_out = dofs + S.cap;
  if (TIER == 1 && tier == 0) {
    for (int i = tid; i < n; i += NT) perm_out[i] = i;
    if (tid == 0) {
      dyn.k[c] = n;
      dyn.nr[c] = 0;
      dyn.h[c] = 0;
      dyn.passes[c] = 0;
      dyn.nfar[c] = 0;
    }
    return;
  }
  if (tier != TIER) return;

  // ---- memory carve-up ----
  // Y's entries: FP32 for FP32 storage, FP64 otherwise (arithmetic in FP64)
  using YE = typename std::conditional<sizeof(T) == 4, float, double>::type;
  char* sp = smem;
  YE* Y;
  YE* Yg = nullptr;  // tier C: room for all R rows of Y in global scratch
  IdRow* rows;
  int* order;
  T* BF;  // far rows, row-major (ld n), in the storage type
  if constexpr (YG && TABS) {
    // far rows, row table and order in LDS; Y in LDS when a pass fits
    Yg = reinterpret_cast<YE*>(scratch + S.scr_off);
    Y = Yg;
    BF = reinterpret_cast<T*>(sp);
    sp += (size_t(R) * n * sizeof(T) + 15) & ~size_t(15);
    rows = reinterpret_cast<IdRow*>(sp);
    sp += size_t(R) * sizeof(IdRow);
    order = reinterpret_cast<int*>(sp);
    sp += (size_t(R) * 4 + 15) & ~size_t(15);
  } else if constexpr (YG) {
    // scratch: Y, B_F and the tables at the offsets of R n doubles each
    Yg = reinterpret_cast<YE*>(scratch + S.scr_off);
    Y = Yg;
    BF = reinterpret_cast<T*>(scratch + S.scr_off + size_t(R) * n);
    rows = reinterpret_cast<IdRow*>(scratch + S.scr_off + 2 * size_t(R) * n);
    order = reinterpret_cast<int*>(rows + R);
  } else {
    Y = reinterpret_cast<YE*>(sp);
    sp += size_t(R) * n * sizeof(YE);
    BF = reinterpret_cast<T*>(sp);
    sp += size_t(R) * n * sizeof(T);
    rows = reinterpret_cast<IdRow*>(sp);
    sp += size_t(R) * sizeof(IdRow);
  }
  double* P = reinterpret_cast<double*>(sp);  // probe rows, row-major (probes x n)
  sp += size_t(ID_MAXPROBES) * n * 8;
  double* Gt = reinterpret_cast<double*>(sp) + size_t(w) * ID_GTILE;  // this wave's Gaussian tile
  sp += size_t(NW) * ID_GTILE * 8;
  double* pn = reinterpret_cast<double*>(sp);  // norm partials [NW][NCOL][64]
  sp += size_t(NW) * 64 * NCOL * 8;
  double* pd = reinterpret_cast<double*>(sp);  // dot partials [NW][NCOL][64]
  sp += size_t(NW) * 64 * NCOL * 8;
  if constexpr (!YG) {
    order = reinterpret_cast<int*>(sp);
    sp += size_t(R) * 4;
  }
  int* pos2col = reinterpret_cast<int*>(sp);
  int* col2pos = pos2col + n;
  // tier C: the rest of the launch's LDS holds the first ylds_rows rows of
  // Y, the rows after them go to Yg
  YE* Ylds = nullptr;
  int ylds_rows = 0;
  if constexpr (YG) {
    const size_t used = (size_t(reinterpret_cast<char*>(col2pos + n) - smem) + 15) & ~size_t(15);
    if (size_t(tiers.lds_c) > used + size_t(n) * sizeof(YE)) {
      Ylds = reinterpret_cast<YE*>(smem + used);
      ylds_rows = int((size_t(tiers.lds_c) - used) / (size_t(n) * sizeof(YE)));
    }
  }

  // ---- 1. row table: near rows listed from the front, far rows from the back ----
  if (w == 0) idc_row_table(S, segs, nbrs, blks, g, iarena, dyn, n, R, hm, rows, order, s_cnt);
  __syncthreads();
  const int nN = s_cnt[0], nF = s_cnt[1];

  int h = prm.h0;
  if (prm.h_init) {
    const int hi = prm.h_init[prm.seg_base + c];
    if (hi > 0) h = hi;
  }
  const int probes = prm.probes;
  int passes = 0, k = 0;
  double r11 = 0.0;
  while (true) {
    ++passes;
    const bool sampled = h < nF;
    const int m = nN + (sampled ? h : nF);
    // one pass on the stacked rows: rows below yl at Y (in LDS; for tier C
    // in global scratch when not even the first min(m, n) rows fit there),
    // tier C's rows from yl on at Yb (global scratch, row i at Yb + i n).
    // Every row the pivot steps, T and the check touch lies below
    // min(m, n) <= yl.  Called at one site per memory layout so that each
    // inlined copy uses its spaces' own instructions.  True when the ID is
    // accepted.
    auto pass = [&](YE* Y, YE* Yb, int yl) -> bool {
      const int mi = m < yl ? m : yl;
      // ---- 2. Y = [B_N; G B_F / sqrt(h)] or the exact far rows; B_F is
      //         fetched once and kept for later passes ----
      idc_fetch<T, NT>(varena, rows, order, R, nN, passes == 1 ? R : nN, Y, Yb, yl, BF, n);
      __syncthreads();
      if (!sampled) {
        for (int t = tid; t < nF * n; t += NT) (nN + t / n < yl ? Y : Yb)[size_t(nN) * n + t] = YE(BF[t]);
      } else {
        // rows of the sketch (stream 0, scaled by 1 / sqrt(h)) and of the
        // probes (stream 1) in pairs, one Philox draw per pair and far row:
        // pair p by wave p mod NW, over all far rows in order (the wave's
        // Gaussian tile holds the entries of 64 far rows), written by that
        // wave alone (no barrier)
        const double sc = 1.0 / sqrt(double(h));
        const int hp = (h + 1) / 2, pp = (probes + 1) / 2;
        double* Gw = Gt;  // this wave's tile: 64 far rows x 2 rows
        for (int p = w; p < hp + pp; p += NW) {
          const int stream = p < hp ? 0 : 1;
          const int pair = stream == 0 ? p : p - hp;
          const int nrows = stream == 0 ? h : probes;
          const int r0 = 2 * pair;
          double a0[NCOL], a1[NCOL];
  #pragma unroll
          for (int s2 = 0; s2 < NCOL; ++s2) a0[s2] = a1[s2] = 0.0;
          for (int f0 = 0; f0 < nF; f0 += 64) {
            const int ff = f0 + lane;
            double ev = 0.0, od = 0.0;
            if (ff < nF) {
              const int vh = rows[order[R - 1 - ff]].vh;
              if constexpr (sizeof(T) == 4) {
                float e32, o32;
                gauss_pair_f32(prm.seed, prm.level, stream, pair, vh >> 1, c, vh & 1, &e32, &o32);
                ev = e32;
                od = o32;
              } else {
                gauss_pair(prm.seed, prm.level, stream, pair, vh >> 1, c, vh & 1, &ev, &od);
              }
            }
            Gw[2 * lane] = ev;
            Gw[2 * lane + 1] = od;
            wave_sync();
            const int fw = nF - f0 < 64 ? nF - f0 : 64;
            // columns past n read column n - 1 (their sums are never
            // stored): no branch around the loads, so they go out together
            const T* bf = BF + size_t(f0) * n;
            int jc[NCOL];
  #pragma unroll
            for (int s2 = 0; s2 < NCOL; ++s2) jc[s2] = lane + 64 * s2 < n ? lane + 64 * s2 : n - 1;
            // FB far rows per batch, all loads first, then the products
            // (tier C in FP64 keeps one row per step: the batch's registers
            // would not fit beside its CPQR's)
            constexpr bool BATCH = sizeof(T) == 4 || !YG;
            constexpr int FB = sizeof(T) == 4 ? 8 : 4;
            int t = 0;
            if constexpr (BATCH)
            for (; t + FB <= fw; t += FB) {
              T bv[FB][NCOL];
              double gv[2 * FB];
  #pragma unroll
              for (int u = 0; u < FB; ++u)
  #pragma unroll
                for (int s2 = 0; s2 < NCOL; ++s2) bv[u][s2] = bf[size_t(t + u) * n + jc[s2]];
  #pragma unroll
              for (int u = 0; u < 2 * FB; ++u) gv[u] = Gw[2 * t + u];
  #pragma unroll
              for (int u = 0; u < FB; ++u) {
                const double g0 = gv[2 * u], g1 = gv[2 * u + 1];
  #pragma unroll
                for (int s2 = 0; s2 < NCOL; ++s2) {
                  a0[s2] += g0 * double(bv[u][s2]);
                  a1[s2] += g1 * double(bv[u][s2]);
                }
              }
            }
            if constexpr (BATCH) {
              for (; t < fw; ++t) {
                const double g0 = Gw[2 * t], g1 = Gw[2 * t + 1];
  #pragma unroll
                for (int s2 = 0; s2 < NCOL; ++s2) {
                  const double b = double(bf[size_t(t) * n + jc[s2]]);
                  a0[s2] += g0 * b;
                  a1[s2] += g1 * b;
                }
              }
            } else {
  #pragma unroll 4
              for (; t < fw; ++t) {
                const double g0 = Gw[2 * t], g1 = Gw[2 * t + 1];
  #pragma unroll
                for (int s2 = 0; s2 < NCOL; ++s2) {
                  const int j = lane + 64 * s2;
                  const double b = j < n ? double(bf[size_t(t) * n + j]) : 0.0;
                  a0[s2] += g0 * b;
                  a1[s2] += g1 * b;
                }
              }
            }
            wave_sync();
          }
  #pragma unroll
          for (int s2 = 0; s2 < NCOL; ++s2) {
            const int j = lane + 64 * s2;
            if (j < n) {
              if (stream == 0) {
                (nN + r0 < yl ? Y : Yb)[size_t(nN + r0) * n + j] = YE(a0[s2] * sc);
                if (r0 + 1 < nrows) (nN + r0 + 1 < yl ? Y : Yb)[size_t(nN + r0 + 1) * n + j] = YE(a1[s2] * sc);
              } else {
                P[size_t(r0) * n + j] = a0[s2];
                if (r0 + 1 < nrows) P[size_t(r0 + 1) * n + j] = a1[s2];
              }
            }
          }
        }
      }
      __syncthreads();

      // ---- 3. CPQR (fresh norms, tie rule: smallest original column) ----
      // The position <-> column tables live in registers during the pivot
      // steps: every wave keeps the same copy, lane l holding the entries
      // l + 64 s, so no step waits on a single thread's LDS updates.
      uint64_t done[NCOL];
      int p2c[NCOL], c2p[NCOL];
  #pragma unroll
      for (int s = 0; s < NCOL; ++s) {
        done[s] = 0ull;
        p2c[s] = c2p[s] = lane + 64 * s;
      }
  #pragma unroll
      for (int s = 0; s < NCOL; ++s) {
        const int j = lane + 64 * s;
        double t = 0.0;
        if (j < n) {
          t = idc_rowdot<NW, UR>(Y, n, w, mi, j, j);
          if constexpr (YG) t += idc_rowdot<NW, UR>(Yb, n, idc_next_row<NW>(w, yl), m, j, j);
        }
        pn[(w * NCOL + s) * 64 + lane] = t;
      }
      __syncthreads();
      const int kmax = m < n ? m : n;
      k = kmax;
      for (int j = 0; j < kmax; ++j) {
        double nv[NCOL];
        bool act[NCOL];
        double mxl = 0.0;
  #pragma unroll
        for (int s = 0; s < NCOL; ++s) {
          const int col = lane + 64 * s;
          act[s] = col < n && !((done[s] >> lane) & 1ull);
          double pv[NW];
  #pragma unroll
          for (int ww = 0; ww < NW; ++ww) pv[ww] = pn[(ww * NCOL + s) * 64 + lane];
          double t = 0.0;
  #pragma unroll
          for (int ww = 0; ww < NW; ++ww) t += pv[ww];
          nv[s] = sqrt(t);
          if (act[s]) mxl = fmax(mxl, nv[s]);
        }
        const double mx = wave_max(mxl);
        int q = -1;
  #pragma unroll
        for (int s = 0; s < NCOL; ++s) {
          const uint64_t cm = __ballot(act[s] && nv[s] >= mx * (1.0 - 1e-12));
          if (q < 0 && cm) q = 64 * s + __ffsll((unsigned long long)cm) - 1;
        }
        if (j == 0) r11 = mx;
        if (mx == 0.0 || mx <= prm.eps * r11 || q < 0) {
          k = j;
          break;
        }
        const int qs = q >> 6, ql = q & 63;
        double nq = nv[0];
  #pragma unroll
        for (int s = 1; s < NCOL; ++s)
          if (qs == s) nq = nv[s];
        const double alpha = __shfl(nq, ql, 64);
        const double x0 = double(Y[size_t(j) * n + q]);
        const double sg = x0 >= 0.0 ? 1.0 : -1.0;
        const double v0 = x0 + sg * alpha;
        const double vv = 2.0 * alpha * (alpha + fabs(x0));
        const int jown = j % NW;
        const int i1 = j + 1 + ((w - (j + 1) % NW) + NW) % NW;  // this wave's first row below j
        // dot products of the reflector with every live column
  #pragma unroll
        for (int s = 0; s < NCOL; ++s) {
          const int col = lane + 64 * s;
          double d = 0.0;
          if (act[s] && col != q) {
            if (w == jown) d = v0 * double(Y[size_t(j) * n + col]);
            d += idc_rowdot<NW, UR>(Y, n, i1, mi, q, col);
            if constexpr (YG) d += idc_rowdot<NW, UR>(Yb, n, idc_next_row<NW>(i1, yl), m, q, col);
          }
          pd[(w * NCOL + s) * 64 + lane] = d;
        }
        __syncthreads();
        // apply the reflector; accumulate the fresh norms of rows > j
  #pragma unroll
        for (int s = 0; s < NCOL; ++s) {
          const int col = lane + 64 * s;
          double a = 0.0;
          if (act[s] && col != q) {
            double pv[NW];
  #pragma unroll
            for (int ww = 0; ww < NW; ++ww) pv[ww] = pd[(ww * NCOL + s) * 64 + lane];
            double t = 0.0;
  #pragma unroll
            for (int ww = 0; ww < NW; ++ww) t += pv[ww];
            const double f = 2.0 * t / vv;
            if (w == jown) Y[size_t(j) * n + col] = YE(double(Y[size_t(j) * n + col]) - f * v0);
            a = idc_rowaxpy<NW, UR>(Y, n, i1, mi, col, q, f);
            if constexpr (YG) a += idc_rowaxpy<NW, UR>(Yb, n, idc_next_row<NW>(i1, yl), m, col, q, f);
          }
          pn[(w * NCOL + s) * 64 + lane] = a;
        }
        if (w == jown && lane == ql) Y[size_t(j) * n + q] = YE(-sg * alpha);
        done[qs] |= 1ull << ql;
        {
          // position j takes column q; the column there moves to q's old position
          int c2pq = c2p[0], p2cj = p2c[0];
  #pragma unroll
          for (int s = 1; s < NCOL; ++s) {
            if (qs == s) c2pq = c2p[s];
            if ((j >> 6) == s) p2cj = p2c[s];
          }
          const int qp = __shfl(c2pq, ql, 64), cj = __shfl(p2cj, j & 63, 64);
  #pragma unroll
          for (int s = 0; s < NCOL; ++s) {
            const int idx = lane + 64 * s;
            if (idx == qp) p2c[s] = cj;
            if (idx == cj) c2p[s] = qp;
            if (idx == j) p2c[s] = q;
            if (idx == q) c2p[s] = j;
          }
        }
        __syncthreads();
      }
      if (w == 0)
  #pragma unroll
        for (int s = 0; s < NCOL; ++s)
          if (lane + 64 * s < n) pos2col[lane + 64 * s] = p2c[s];
      __syncthreads();

      // ---- 4. T = R11^{-1} R12, in place in rows < k of the remaining columns ----
      const int nr = n - k;
      for (int i = k - 1; i >= 0; --i) {
        const int ci = pos2col[i];
        const double rii = double(Y[size_t(i) * n + ci]);
        double tq[NCOL];
  #pragma unroll
        for (int s = 0; s < NCOL; ++s) {
          const int qq = lane + 64 * s;
          tq[s] = qq < nr ? double(Y[size_t(i) * n + pos2col[k + qq]]) / rii : 0.0;
        }
        grp_sync<NW>();
  #pragma unroll
        for (int s = 0; s < NCOL; ++s) {
          const int qq = lane + 64 * s;
          if (qq < nr) {
            const int cq = pos2col[k + qq];
            if (w == i % NW) Y[size_t(i) * n + cq] = YE(tq[s]);
            for (int t = w; t < i; t += NW)
              Y[size_t(t) * n + cq] = YE(double(Y[size_t(t) * n + cq]) - double(Y[size_t(t) * n + ci]) * tq[s]);
          }
        }
        grp_sync<NW>();
      }
      __syncthreads();

      // ---- 5. a-posteriori check with the probe rows: E = P_r - P_s T
      //         (one probe per wave, the columns of T over the lanes) ----
      bool accept = true;
      if (sampled) {
        for (int pr = w; pr < probes; pr += NW) {
          double sv = 0.0;
  #pragma unroll
          for (int s = 0; s < NCOL; ++s) {
            const int qq = lane + 64 * s;
            if (qq < nr) {
              const int cq = pos2col[k + qq];
              const double* Pr = P + size_t(pr) * n;
              double e = Pr[cq];
              int t = 0;
              for (; t + UR <= k; t += UR) {
                double yv[UR], pv[UR];
  #pragma unroll
                for (int u = 0; u < UR; ++u) {
                  yv[u] = double(Y[size_t(t + u) * n + cq]);
                  pv[u] = Pr[pos2col[t + u]];
                }
  #pragma unroll
                for (int u = 0; u < UR; ++u) e -= pv[u] * yv[u];
              }
              for (; t < k; ++t) e -= Pr[pos2col[t]] * double(Y[size_t(t) * n + cq]);
              sv += e * e;
            }
          }
          sv = wave_sum(sv);
          if (lane == 0) pn[pr] = sqrt(sv);
        }
        __syncthreads();
        if (tid == 0) {
          double worst = 0.0;
          for (int pr = 0; pr < probes; ++pr) worst = fmax(worst, pn[pr]);
          s_acc = worst <= prm.tau * sqrt(double(nr)) * prm.eps * r11 ? 1 : 0;
        }
        __syncthreads();
        accept = s_acc != 0;
      }
      if (accept) {
        T* Tm = varena + S.t_off;
        for (int t = tid; t < k * nr; t += NT) {
          const int i = t / nr, qq = t % nr;
          Tm[t] = T(Y[size_t(i) * n + pos2col[k + qq]]);
        }
        for (int i = tid; i < n; i += NT) perm_out[i] = pos2col[i];
        return true;
      }
      return false;
    };
    bool accepted;
    if constexpr (YG)
      accepted = ylds_rows >= (m < n ? m : n) ? pass(Ylds, Yg, ylds_rows) : pass(Yg, Yg, m);
    else
      accepted = pass(Y, Y, m);
    if (accepted) break;
    h *= 2;
    __syncthreads();
  }
  if (tid == 0) {
    dyn.k[c] = k;
    dyn.nr[c] = n - k;
    dyn.h[c] = h < nF ? h : nF;
    dyn.passes[c] = passes;
    dyn.nfar[c] = nF;
  }
}

// ---------------------------------------------------------------------------
// Block-cooperative ID for segments wider than 128 columns: the stacked rows
// are staged in the segment's global scratch, the CPQR runs on NT threads.
// ---------------------------------------------------------------------------

// CPQR of Y (m x n, column-major, ld) with fresh column norms each step and
// the tie rule of the oracle; returns k and writes |R_11| to *r11.  perm[]
// (original column index per position) is permuted alongside.
//
// Each step makes one pass over the trailing columns: a wave takes a column,
// forms its Householder dot, updates it and sums the squares of the updated
// entries below the pivot row, which are the fresh norms the next step
// pivots on (recomputed from the entries, not downdated).  When the rows
// below the pivot fit CPQR_RB entries per lane (32, or 16 for groups of 16
// waves, which have half the registers), the Householder vector stays in
// registers for the whole step and each column is read once.
template <int NW>
__device__ int block_cpqr(double* Y, int ld, int m, int n, int* perm, double eps, double* nrm,
                          double* s_scal, int* s_int, double* r11_out) {
  constexpr int NT = 64 * NW;
  constexpr int CPQR_RB = NW >= 16 ? 16 : 32;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int kk = m < n ? m : n;
  int k = kk;
  double r11 = 0.0;
  // norms of the first step (rows 0..m-1)
  for (int col = wv; col < n; col += NW) {
    double s = 0.0;
    for (int i = lane; i < m; i += 64) {
      const double y = Y[size_t(col) * ld + i];
      s += y * y;
    }
    s = wave_sum(s);
    if (lane == 0) nrm[col] = sqrt(s);
  }
  __syncthreads();
  for (int j = 0; j < kk; ++j) {
    if (wv == 0) {
      double mx = 0.0;
      for (int col = j + lane; col < n; col += 64) mx = fmax(mx, nrm[col]);
      mx = wave_max(mx);
      int key = 1 << 30, q = 1 << 30;
      for (int col = j + lane; col < n; col += 64)
        if (nrm[col] >= mx * (1.0 - 1e-12)) {
          const int pk = perm[col];
          if (pk < key) {
            key = pk;
            q = col;
          }
        }
      wave_argmin_int(key, q);
      if (lane == 0) {
        s_scal[0] = mx;
        s_int[0] = q;
        s_scal[2] = nrm[q];
      }
    }
    __syncthreads();
    const double mx = s_scal[0];
    const int q = s_int[0];
    const double alpha = s_scal[2];
    if (j == 0) r11 = mx;
    if (mx == 0.0 || mx <= eps * r11) {
      k = j;
      break;
    }
    if (q != j) {
      for (int i = tid; i < m; i += NT) {
        const double t = Y[size_t(j) * ld + i];
        Y[size_t(j) * ld + i] = Y[size_t(q) * ld + i];
        Y[size_t(q) * ld + i] = t;
      }
      if (tid == 0) {
        const int t = perm[j];
        perm[j] = perm[q];
        perm[q] = t;
        nrm[q] = nrm[j];  // the column moved to position q keeps its norm
      }
    }
    __syncthreads();
    const double x0 = Y[size_t(j) * ld + j];
    const double sg = x0 >= 0.0 ? 1.0 : -1.0;
    const double v0 = x0 + sg * alpha;
    if (wv == 0) {
      double s = 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) {
        const double y = Y[size_t(j) * ld + i];
        s += y * y;
      }
      s = wave_sum(s);
      if (lane == 0) s_scal[1] = s + v0 * v0;
    }
    __syncthreads();
    const double vv = s_scal[1];
    const int i0 = j + 1 + lane;
    if (m - (j + 1) <= 64 * CPQR_RB) {
      // Householder vector in registers, one read and one write per column
      double vr[CPQR_RB];
#pragma unroll
      for (int u = 0; u < CPQR_RB; ++u) {
        const int i = i0 + 64 * u;
        vr[u] = i < m ? Y[size_t(j) * ld + i] : 0.0;
      }
      for (int col = j + 1 + wv; col < n; col += NW) {
        double* yc = Y + size_t(col) * ld;
        double yr[CPQR_RB];
        double w = 0.0;
#pragma unroll
        for (int u = 0; u < CPQR_RB; ++u) {
          const int i = i0 + 64 * u;
          yr[u] = i < m ? yc[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < CPQR_RB; ++u) w += vr[u] * yr[u];
        w = wave_sum(w) + v0 * yc[j];
        const double f = 2.0 * w / vv;
        if (lane == 0) yc[j] -= f * v0;
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < CPQR_RB; ++u) {
          const int i = i0 + 64 * u;
          const double y = yr[u] - f * vr[u];
          if (i < m) {
            yc[i] = y;
            s += y * y;
          }
        }
        s = wave_sum(s);
        if (lane == 0) nrm[col] = sqrt(s);
      }
    } else {
      // taller: the same in chunks of CPQR_RB rows per lane, the loads of a
      // chunk issued together (the sums keep the row order of the lanes)
      const double* vj = Y + size_t(j) * ld;
      for (int col = j + 1 + wv; col < n; col += NW) {
        double* yc = Y + size_t(col) * ld;
        double w = 0.0;
        for (int c0 = i0; c0 < m; c0 += 64 * CPQR_RB) {
          double vr[CPQR_RB], yr[CPQR_RB];
#pragma unroll
          for (int u = 0; u < CPQR_RB; ++u) {
            const int i = c0 + 64 * u;
            vr[u] = i < m ? vj[i] : 0.0;
            yr[u] = i < m ? yc[i] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < CPQR_RB; ++u) w += vr[u] * yr[u];
        }
        w = wave_sum(w) + v0 * yc[j];
        const double f = 2.0 * w / vv;
        if (lane == 0) yc[j] -= f * v0;
        double s = 0.0;
        for (int c0 = i0; c0 < m; c0 += 64 * CPQR_RB) {
          double vr[CPQR_RB], yr[CPQR_RB];
#pragma unroll
          for (int u = 0; u < CPQR_RB; ++u) {
            const int i = c0 + 64 * u;
            vr[u] = i < m ? vj[i] : 0.0;
            yr[u] = i < m ? yc[i] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < CPQR_RB; ++u) {
            const int i = c0 + 64 * u;
            const double y = yr[u] - f * vr[u];
            if (i < m) {
              yc[i] = y;
              s += y * y;
            }
          }
        }
        s = wave_sum(s);
        if (lane == 0) nrm[col] = sqrt(s);
      }
    }
    __syncthreads();
    if (tid == 0) Y[size_t(j) * ld + j] = -sg * alpha;
    __syncthreads();
  }
  *r11_out = r11;
  return k;
}


template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_seg_id(const DSeg* segs, int nseg, const DNbr* nbrs,
                                               const DBlk* blks, GridGeom g, int32_t* iarena,
                                               T* varena, double* scratch, DLevelDyn dyn,
                                               IdParams prm, IdTiers tiers) {
  constexpr int NW = NT / 64;
  extern __shared__ double lds[];
  __shared__ double s_nrm[512];
  __shared__ double s_scal[NW > 4 ? NW : 4];
  __shared__ int s_int[4];
  __shared__ int s_w[NW];
  __shared__ int s_cnt[2];
  const int c = blockIdx.x;
  if (c >= nseg) return;
  const int tid = threadIdx.x;
  const DSeg S = segs[c];
  const int n = dyn.n[c];
  int R = 0;
  const int hm = prm.sym ? 1 : 2;  // halves of the coupling rows per neighbour
  for (int e = S.nbr_begin; e < S.nbr_end; ++e) R += hm * dyn.n[nbrs[e].d];
  if (id_tier(S, n, R, prm, c, tiers) != 5) return;
  int32_t* dofs = iarena + S.ioff;
  int32_t* perm = dofs + S.cap;
  int32_t* tag = perm + 2 * S.cap;  // after piv
  for (int i = tid; i < n; i += NT) perm[i] = i;
  const size_t rc = size_t(S.rcap);
  double* BN = scratch + S.scr_off;  // near rows, column-major (ld rcap)
  double* BF = BN + rc * S.cap;      // far rows, row-major (ld n)
  double* Yg = BF + rc * S.cap;      // work matrix, column-major (ld rcap)
  double* P = Yg + rc * S.cap;       // probe rows, row-major (8 x n)
  if (tid == 0) {
    s_cnt[0] = 0;
    s_cnt[1] = 0;
  }
  __syncthreads();
  // 1. stack [A_{n,c}; A_{c,n}^T] (A_{n,c} alone in the symmetric form) row
  // by row, split near / far
  for (int e = S.nbr_begin; e < S.nbr_end; ++e) {
    const DNbr nb = nbrs[e];
    const int nd = dyn.n[nb.d];
    const int32_t* dd = iarena + segs[nb.d].ioff;
    for (int half = 0; half < hm; ++half) {
      const T* blk = varena + blks[half == 0 ? nb.blk_dc : nb.blk_cd].off;
      for (int base = 0; base < nd; base += NT) {
        const int i = base + tid;
        const bool valid = i < nd;
        int v = 0;
        bool near = false;
        if (valid) {
          v = dd[i];
          int cv[3];
          vcoords(g, v, cv);
          int dist = 0;
          for (int a = 0; a < 3; ++a) {
            int da = S.lo[a] - cv[a];
            if (cv[a] - S.hi[a] > da) da = cv[a] - S.hi[a];
            if (da > dist) dist = da;
          }
          near = dist <= S.thr;
        }
        int tn, tf;
        const int pn = block_scan_flag<NW>(valid && near, s_w, &tn);
        const int pf = block_scan_flag<NW>(valid && !near, s_w, &tf);
        const int bn = s_cnt[0], bf = s_cnt[1];
        if (valid) {
          if (near) {
            const int r = bn + pn;
            for (int j = 0; j < n; ++j)
              BN[size_t(j) * rc + r] = double(half == 0 ? blk[size_t(i) * n + j] : blk[size_t(j) * nd + i]);
          } else {
            const int r = bf + pf;
            for (int j = 0; j < n; ++j)
              BF[size_t(r) * n + j] = double(half == 0 ? blk[size_t(i) * n + j] : blk[size_t(j) * nd + i]);
            tag[2 * r] = v;
            tag[2 * r + 1] = half;
          }
        }
        __syncthreads();
        if (tid == 0) {
          s_cnt[0] = bn + tn;
          s_cnt[1] = bf + tf;
        }
        __syncthreads();
      }
    }
  }
  const int nN = s_cnt[0], nF = s_cnt[1];
  if (nN + nF == 0) {  // no coupling rows left: nothing to compress against
    if (tid == 0) {
      dyn.k[c] = n;
      dyn.nr[c] = 0;
      dyn.h[c] = 0;
      dyn.passes[c] = 0;
      dyn.nfar[c] = 0;
    }
    return;
  }
  int h = prm.h0;
  if (prm.h_init) {
    const int hi = prm.h_init[prm.seg_base + c];
    if (hi > 0) h = hi;
  }
  int passes = 0, k = 0;
  double r11 = 0.0;
  T* Tm = varena + S.t_off;
  while (true) {
    ++passes;
    const bool sampled = h < nF;
    const int m = nN + (sampled ? h : nF);
    // 2. Y = [B_N; G B_F / sqrt(h)] (or the exact far rows)
    for (int t = tid; t < nN * n; t += NT) {
      const int j = t / nN, i = t % nN;
      Yg[size_t(j) * rc + i] = BN[size_t(j) * rc + i];
    }
    if (!sampled) {
      for (int t = tid; t < nF * n; t += NT) {
        const int f = t / n, j = t % n;
        Yg[size_t(j) * rc + nN + f] = BF[size_t(f) * n + j];
      }
    } else {
      const double sc = 1.0 / sqrt(double(h));
      for (int t = tid; t < h * n; t += NT) {
        const int i = t % h, j = t / h;
        Yg[size_t(j) * rc + nN + i] = 0.0;
      }
      for (int t = tid; t < prm.probes * n; t += NT) P[t] = 0.0;
      const int hp = h + prm.probes;  // sample rows, then probe rows
      for (int i0 = 0; i0 < hp; i0 += 32) {
        const int ih = hp - i0 < 32 ? hp - i0 : 32;
        for (int f0 = 0; f0 < nF; f0 += 64) {
          const int fw = nF - f0 < 64 ? nF - f0 : 64;
          __syncthreads();
          for (int t = tid; t < ih * fw; t += NT) {
            const int ii = t / fw, f = t % fw;
            const int row = i0 + ii;
            const int stream = row < h ? 0 : 1;
            const int r = row < h ? row : row - h;
            lds[ii * 64 + f] = gauss_entry(prm.seed, prm.level, stream, r, tag[2 * (f0 + f)], c,
                                           tag[2 * (f0 + f) + 1]);
          }
          __syncthreads();
          for (int t = tid; t < ih * n; t += NT) {
            const int ii = t / n, j = t % n;
            double acc = 0.0;
            for (int f = 0; f < fw; ++f) acc += lds[ii * 64 + f] * BF[size_t(f0 + f) * n + j];
            const int row = i0 + ii;
            if (row < h)
              Yg[size_t(j) * rc + nN + row] += acc;
            else
              P[(row - h) * n + j] += acc;
          }
        }
      }
      __syncthreads();
      for (int t = tid; t < h * n; t += NT) {
        const int i = t % h, j = t / h;
        Yg[size_t(j) * rc + nN + i] *= sc;
      }
    }
    for (int i = tid; i < n; i += NT) perm[i] = i;
    __syncthreads();
    // 3. CPQR (staged in LDS when it fits)
    const bool inlds = size_t(m) * n <= LDS_DOUBLES;
    double* Y = inlds ? lds : Yg;
    const int ld = inlds ? m : int(rc);
    if (inlds) {
      for (int t = tid; t < m * n; t += NT) {
        const int j = t / m, i = t % m;
        lds[t] = Yg[size_t(j) * rc + i];
      }
    }
    double* nrm = n <= 512 ? s_nrm : P + 8 * n;
    __syncthreads();
    k = block_cpqr<NW>(Y, ld, m, n, perm, prm.eps, nrm, s_scal, s_int, &r11);
    __syncthreads();
    // 4. T = R11^{-1} R12 (back substitution in FP64, in place in Y)
    const int nr = n - k;
    for (int q = tid; q < nr; q += NT) {
      double* col = Y + size_t(k + q) * ld;
      for (int i = k - 1; i >= 0; --i) {
        double s = col[i];
        for (int t = i + 1; t < k; ++t) s -= Y[size_t(t) * ld + i] * col[t];
        col[i] = s / Y[size_t(i) * ld + i];
      }
    }
    __syncthreads();
    bool accept = true;
    if (sampled) {
      // 5. a-posteriori check with the probe rows: E = P_r - P_s T
      double worst = 0.0;
      for (int pr = 0; pr < prm.probes; ++pr) {
        double s = 0.0;
        for (int q = tid; q < nr; q += NT) {
          double e = P[pr * n + perm[k + q]];
          for (int t = 0; t < k; ++t) e -= P[pr * n + perm[t]] * Y[size_t(k + q) * ld + t];
          s += e * e;
        }
        s = block_sum<NW>(s, s_scal);
        worst = fmax(worst, sqrt(s));
      }
      accept = worst <= prm.tau * sqrt(double(nr)) * prm.eps * r11;
    }
    if (accept) {
      for (int t = tid; t < k * nr; t += NT) {
        const int i = t / nr, q = t % nr;
        Tm[t] = T(Y[size_t(k + q) * ld + i]);
      }
      break;
    }
    h *= 2;
    __syncthreads();
  }
  if (tid == 0) {
    dyn.k[c] = k;
    dyn.nr[c] = n - k;
    dyn.h[c] = h < nF ? h : nF;
    dyn.passes[c] = passes;
    dyn.nfar[c] = nF;
  }
}



}  // namespace spalu
