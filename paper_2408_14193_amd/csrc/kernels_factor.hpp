// Factorization kernels (Algorithm 2).  One workgroup per leaf, segment or
// block of a level; all segments of a level go in one launch.  T is the
// storage type of blocks and factors (double for the plain form, float for
// the mixed form); pivoted LUs of diagonal blocks and the ID's triangular
// solve always run in FP64.
#pragma once

#include "device_common.hpp"
#include "layout.hpp"
#include "mfma_tile.hpp"

namespace spalu {

// store(t, load(t)) for t in [0, count), t = lane + stride * m: the loads
// of a batch of NB are issued together, so a staging loop costs one trip to
// memory per batch instead of one per load; a last batch of one row loads
// that row only.
template <int NB, typename L, typename F>
__device__ inline void load_batched(int count, int lane, int stride, L load, F store) {
  using V = decltype(load(0));
  int t0 = 0;
  for (; t0 + NB * stride <= count; t0 += NB * stride) {
    V v[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) v[b] = load(t0 + b * stride + lane);
#pragma unroll
    for (int b = 0; b < NB; ++b) store(t0 + b * stride + lane, v[b]);
  }
  if (t0 < count) {
    // the last, partial batch: only the rows of the range are loaded
    // when they fit in one row, else all NB with clamped indices
    if (count - t0 <= stride) {
      const int t = t0 + lane;
      if (t < count) store(t, load(t));
    } else {
      V v[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int t = t0 + b * stride + lane;
        v[b] = load(t < count ? t : count - 1);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int t = t0 + b * stride + lane;
        if (t < count) store(t, v[b]);
      }
    }
  }
}

// store(t, src[t]) for t in [0, count), in batches as above.
template <int NB, typename S, typename F>
__device__ inline void stage_batched(const S* src, int count, int lane, int stride, F store) {
  load_batched<NB>(count, lane, stride, [&](int t) { return src[t]; }, store);
}

struct GridGeom {
  int nx, ny, nz;
};

__device__ inline void vcoords(const GridGeom& g, int v, int c[3]) {
  c[0] = v % g.nx;
  c[1] = (v / g.nx) % g.ny;
  c[2] = v / (g.nx * g.ny);
}

// CSR entry A(u, w) (0 if absent); columns ascending in each row.
__device__ inline double csr_at(const int64_t* rowptr, const int32_t* colind, const double* vals, int u,
                                int w) {
  for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e)
    if (colind[e] == w) return vals[e];
  return 0.0;
}

// Local index in a leaf box of grid vertex w, a stencil neighbour of the box
// vertex u with local coordinates (ix, iy, iz) and local index i; -1 when w
// lies outside the box.  The box is w0 x w1 x w2 and its local index runs x
// fastest; the direction of w follows from w - u alone.
__device__ inline int box_nbr(const GridGeom& g, int w0, int w1, int w2, int ix, int iy, int iz, int i, int u,
                              int w) {
  const int d = w - u, sxy = g.nx * g.ny;
  if (d == 0) return i;
  if (g.nx > 1 && d == 1) return ix + 1 < w0 ? i + 1 : -1;
  if (g.nx > 1 && d == -1) return ix > 0 ? i - 1 : -1;
  if (g.ny > 1 && d == g.nx) return iy + 1 < w1 ? i + w0 : -1;
  if (g.ny > 1 && d == -g.nx) return iy > 0 ? i - w0 : -1;
  if (g.nz > 1 && d == sxy) return iz + 1 < w2 ? i + w0 * w1 : -1;
  if (g.nz > 1 && d == -sxy) return iz > 0 ? i - w0 * w1 : -1;
  return -1;
}

// Zeroes n ints (a kernel, not a memset, so that it can sit in a captured
// graph).
__global__ void k_zero_i32(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Every CSR entry must lie on the stencil (|dx|+|dy|+|dz| <= 1) and columns
// must ascend; flags bit 1 otherwise.
__global__ void k_check_pattern(GridGeom g, int64_t n, const int64_t* rowptr, const int32_t* colind,
                                int* status) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int cv[3];
  vcoords(g, int(v), cv);
  int last = -1;
  for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
    const int w = colind[e];
    bool ok = w > last && w >= 0 && w < n;
    if (ok) {
      int cw[3];
      vcoords(g, w, cw);
      const int d = abs(cw[0] - cv[0]) + abs(cw[1] - cv[1]) + abs(cw[2] - cv[2]);
      ok = d <= 1;
    }
    if (!ok) atomicOr(status, 2);
    last = w;
  }
}

// Symmetric form: every CSR entry (v, w) must have its mirror (w, v) with the
// same value (the rows are short, so the mirror is found by a scan); flags
// bit 2 otherwise.
__global__ void k_check_symmetric(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* vals,
                                  int* status) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
    const int w = colind[e];
    if (w < 0 || w >= n) continue;  // reported by the pattern check
    bool ok = false;
    for (int64_t f = rowptr[w]; f < rowptr[w + 1]; ++f)
      if (colind[f] == int(v)) ok = vals[f] == vals[e];
    if (!ok) atomicOr(status, 4);
  }
}

// ---------------------------------------------------------------------------
// Leaf elimination (eq. (4.8)): A_II^{-1} by Gauss-Jordan elimination with
// partial pivoting (in place; the row interchanges become column
// interchanges of the inverse), X = A_II^{-1} A_IB and S = A_BI X.  Three
// barriers per pivot step.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(WG) void k_leaf_factor(const DLeaf* leaves, int nleaf, GridGeom g,
                                                    const int64_t* rowptr, const int32_t* colind,
                                                    const double* vals, int32_t* iarena, T* varena,
                                                    double* gscratch, int64_t gscr_stride, int* status,
                                                    int level, int lds_doubles, int defer) {
  extern __shared__ double lds[];
  __shared__ int s_piv;
  __shared__ double s_d;
  __shared__ int s_pv[LEAF_MAX_NI];
  const int lf = blockIdx.x;
  if (lf >= nleaf) return;
  const DLeaf L = leaves[lf];
  const int ni = L.ni, nb = L.nb, tid = threadIdx.x;
  const int w0 = L.hi[0] - L.lo[0] + 1, w1 = L.hi[1] - L.lo[1] + 1;
  const int32_t* bverts = iarena + L.ioff;
  int32_t* piv = iarena + L.ioff + nb;
  const bool fits = leaf_lds_need(ni, nb) <= lds_doubles;       // staging in LDS (lds_doubles given)
  double* A = fits ? lds : gscratch + size_t(lf) * gscr_stride;  // A_II, then its inverse
  double* B = A + ni * ni;                                        // A_IB
  double* X = B + ni * nb;                                        // A_II^{-1} A_IB
  double* f = X + ni * nb;                                        // column k before step k
  int* bv = reinterpret_cast<int*>(f + ni);                       // boundary vertices
  for (int t = tid; t < ni * ni + ni * nb; t += WG) A[t] = 0.0;
  for (int b = tid; b < nb; b += WG) bv[b] = bverts[b];
  __syncthreads();
  // interior rows: A_II and A_IB
  for (int i = tid; i < ni; i += WG) {
    const int ix = i % w0, iy = (i / w0) % w1, iz = i / (w0 * w1);
    const int u = (L.lo[0] + ix) + g.nx * ((L.lo[1] + iy) + g.ny * (L.lo[2] + iz));
    for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
      const int w = colind[e];
      int cw[3];
      vcoords(g, w, cw);
      if (cw[0] >= L.lo[0] && cw[0] <= L.hi[0] && cw[1] >= L.lo[1] && cw[1] <= L.hi[1] &&
          cw[2] >= L.lo[2] && cw[2] <= L.hi[2]) {
        const int j = (cw[0] - L.lo[0]) + w0 * ((cw[1] - L.lo[1]) + w1 * (cw[2] - L.lo[2]));
        A[i * ni + j] = vals[e];
      } else {
        for (int b = 0; b < nb; ++b)
          if (bv[b] == w) {
            B[i * nb + b] = vals[e];
            break;
          }
      }
    }
  }
  __syncthreads();
  bool singular = false;
  for (int k = 0; k < ni; ++k) {
    // pivot: largest |a_ik|, i >= k (ties to the smaller row); keep column k
    for (int i = tid; i < ni; i += WG) f[i] = A[i * ni + k];
    if (tid < 64) {
      double bv = -1.0;
      int bi = 1 << 30;
      for (int i = k + tid; i < ni; i += 64) {
        const double a = fabs(A[i * ni + k]);
        if (a > bv) {
          bv = a;
          bi = i;
        }
      }
      wave_argmax(bv, bi);
      if (tid == 0) {
        const int pp = bi < ni ? bi : k;
        s_piv = pp;
        s_d = A[pp * ni + k];
        s_pv[k] = pp;
      }
    }
    __syncthreads();
    const int p = s_piv;
    const double d = s_d;
    if (d == 0.0) {  // uniform: every thread read the same d
      singular = true;
      __syncthreads();
      continue;
    }
    // swap rows k and p, scale the new row k (its entry k becomes 1/d)
    for (int j = tid; j < ni; j += WG) {
      const double ak = A[k * ni + j], ap = A[p * ni + j];
      if (p != k) A[p * ni + j] = ak;
      A[k * ni + j] = j == k ? 1.0 / d : ap / d;
    }
    __syncthreads();
    // eliminate column k from every other row; the multiplier of row i is
    // its entry in column k after the interchange.  Thread (r, j) = (tid /
    // 64, tid % 64) updates column j (and j + 64, ...) of rows r, r + 4, ...
    for (int j = tid & 63; j < ni; j += 64) {
      const double akj = A[k * ni + j];
      for (int i = tid >> 6; i < ni; i += WG / 64) {
        if (i == k) continue;
        const double mi = i == p ? f[k] : f[i];
        if (j == k)
          A[i * ni + j] = -mi * akj;
        else
          A[i * ni + j] -= mi * akj;
      }
    }
    __syncthreads();
  }
  if (singular && tid == 0) flag_singular(status, level);
  for (int k = tid; k < ni; k += WG) piv[k] = s_pv[k];
  // undo the row interchanges on the columns of the inverse, last first
  for (int k = ni - 1; k >= 0; --k) {
    const int p = s_pv[k];
    if (p == k) continue;
    for (int i = tid; i < ni; i += WG) {
      const double t = A[i * ni + k];
      A[i * ni + k] = A[i * ni + p];
      A[i * ni + p] = t;
    }
    __syncthreads();
  }
  // A_II^{-1}, stored transposed (entry (i, q) at q * ni + i) so that the
  // solve's lanes, one per row, read consecutive addresses
  T* LUo = varena + L.lu_off;
  for (int t = tid; t < ni * ni; t += WG) LUo[t] = T(A[(t % ni) * ni + t / ni]);
  // defer: X and S are left to k_leaf_x_mfma (staging in scratch)
  if (defer) return;
  // X = A_II^{-1} A_IB
  for (int t = tid; t < ni * nb; t += WG) {
    const int i = t / nb, c = t - i * nb;
    double acc = 0.0;
    for (int q = 0; q < ni; ++q) acc += A[i * ni + q] * B[q * nb + c];
    X[t] = acc;
  }
  __syncthreads();
  // S = A_BI X (boundary rows, sparse)
  T* S = varena + L.s_off;
  for (int t = tid; t < nb * nb; t += WG) {
    const int b = t / nb, c = t % nb;
    const int u = bv[b];
    double acc = 0.0;
    for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
      const int w = colind[e];
      int cw[3];
      vcoords(g, w, cw);
      if (cw[0] >= L.lo[0] && cw[0] <= L.hi[0] && cw[1] >= L.lo[1] && cw[1] <= L.hi[1] &&
          cw[2] >= L.lo[2] && cw[2] <= L.hi[2]) {
        const int j = (cw[0] - L.lo[0]) + w0 * ((cw[1] - L.lo[1]) + w1 * (cw[2] - L.lo[2]));
        acc += vals[e] * X[j * nb + c];
      }
    }
    S[t] = T(acc);
  }
}

// Second half of k_leaf_factor for leaves staged in scratch (3D), launched
// after it with defer set: X = A_II^{-1} A_IB on the matrix cores (FP64
// 16 x 64 output tiles, one wave per tile, operands read from the leaf's
// scratch), then S = A_BI X.  A launch of its own keeps the tiles' registers
// out of the Gauss-Jordan sweep, whose occupancy matters when many leaves
// share a CU.
template <typename T>
__global__ __launch_bounds__(WG) void k_leaf_x_mfma(const DLeaf* leaves, int nleaf, GridGeom g,
                                                    const int64_t* rowptr, const int32_t* colind,
                                                    const double* vals, T* varena, double* gscratch,
                                                    int64_t gscr_stride) {
  const int lf = blockIdx.x;
  if (lf >= nleaf) return;
  const DLeaf L = leaves[lf];
  const int ni = L.ni, nb = L.nb, tid = threadIdx.x;
  const int w0 = L.hi[0] - L.lo[0] + 1, w1 = L.hi[1] - L.lo[1] + 1;
  const double* A = gscratch + size_t(lf) * gscr_stride;  // A_II^{-1}
  const double* B = A + ni * ni;                           // A_IB
  double* X = const_cast<double*>(B) + ni * nb;            // A_II^{-1} A_IB
  const int* bv = reinterpret_cast<const int*>(X + ni * nb + ni);
  {
    const int w = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int nti = (ni + 15) >> 4, ncg = (nb + 63) >> 6;
    for (int unit = w; unit < nti * ncg; unit += NWAVE) {
      const int ti = unit / ncg, cg = unit - ti * ncg, i0 = 16 * ti, j0 = 64 * cg;
      const int nct = ((nb - j0 < 64 ? nb - j0 : 64) + 15) >> 4;
      gg_v4 acc[4] = {};
      wave_tile_mfma(
          [&](int i, int q) {
            const double v = A[(i < ni ? i : ni - 1) * ni + (q < ni ? q : ni - 1)];
            return i < ni && q < ni ? v : 0.0;
          },
          [&](int q, int col) {
            const int c = j0 + col;
            return B[(q < ni ? q : ni - 1) * nb + (c < nb ? c : nb - 1)];
          },
          i0, 0, ni, nct, acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + lk + 4 * r;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int c = j0 + 16 * cc + li;
          if (i < ni && c < nb && cc < nct) X[i * nb + c] = acc[cc][r];
        }
      }
    }
  }
  __syncthreads();
  // S = A_BI X (boundary rows, sparse)
  T* S = varena + L.s_off;
  for (int t = tid; t < nb * nb; t += WG) {
    const int b = t / nb, c = t % nb;
    const int u = bv[b];
    double acc = 0.0;
    for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
      const int w = colind[e];
      int cw[3];
      vcoords(g, w, cw);
      if (cw[0] >= L.lo[0] && cw[0] <= L.hi[0] && cw[1] >= L.lo[1] && cw[1] <= L.hi[1] &&
          cw[2] >= L.lo[2] && cw[2] <= L.hi[2]) {
        const int j = (cw[0] - L.lo[0]) + w0 * ((cw[1] - L.lo[1]) + w1 * (cw[2] - L.lo[2]));
        acc += vals[e] * X[j * nb + c];
      }
    }
    S[t] = T(acc);
  }
}

// One wave per leaf of at most 64 interior vertices: Gauss-Jordan
// elimination with partial pivoting of [A_II | A_IB], lane i holding row i
// in registers, so that the sweep needs no barriers.  Rows are never
// swapped and the pivot row of step k is not divided by its pivot d_k during
// the sweep (the multipliers carry 1/d_k); each row is divided by the pivot
// of the step that chose it at the end.  The pivot column of every step sits
// in register slot 0: after the update the row moves down one slot and the
// new column of the inverse enters at the last one, so after ni steps slots
// [0, nb) hold A_II^{-1} A_IB and slots [WC - ni, WC) the columns of the
// inverse in pivot order.  Row r of the results sits in the lane chosen at
// step r, and column k of the inverse there belongs to vertex piv[k].
constexpr int LEAF_WAVE_MAX_NI = 64;

// Register slots per lane for a leaf (0: the leaf needs the block kernel).
__host__ __device__ inline int leaf_wave_slots(int ni, int nb) {
  const int w = ni + nb;
  if (ni > LEAF_WAVE_MAX_NI) return 0;
  return w <= 48 ? 48 : w <= 80 ? 80 : w <= 96 ? 96 : 0;
}

// Dynamic LDS bytes of the one-wave kernel: the broadcast pivot row, X, the
// boundary couplings, the pivot order and the boundary list.
__host__ __device__ inline int leaf_wave_lds_bytes(int wc, int ni, int nb) {
  return 8 * (wc + ni * nb + nb) + 4 * (ni + 2 * nb);
}

template <typename T, int WC>
__global__ __launch_bounds__(64) void k_leaf_factor_wave(const DLeaf* leaves, int nleaf, GridGeom g,
                                                         const int64_t* rowptr, const int32_t* colind,
                                                         const double* vals, int32_t* iarena, T* varena,
                                                         int* status, int level) {
  extern __shared__ double lds[];
  const int lf = blockIdx.x;
  if (lf >= nleaf) return;
  const DLeaf L = leaves[lf];
  const int ni = L.ni, nb = L.nb, lane = threadIdx.x;
  const int w0 = L.hi[0] - L.lo[0] + 1, w1 = L.hi[1] - L.lo[1] + 1, w2 = L.hi[2] - L.lo[2] + 1;
  double* prow = lds;                                  // pivot row of the step
  double* X = lds + WC;                                // A_II^{-1} A_IB, ni x nb
  double* ba = X + ni * nb;                            // a_bi of boundary vertex b
  int* pord = reinterpret_cast<int*>(ba + nb);         // pivot vertex of step k
  int* bvl = pord + ni;                                // boundary vertices
  int* bi = bvl + nb;                                  // its interior neighbour i (-1: none)
  const int32_t* bverts = iarena + L.ioff;
  int32_t* piv = iarena + L.ioff + nb;
  // boundary vertex b: its coupling a_bi into the box (a vertex outside a
  // box is a stencil neighbour of at most one box vertex)
  for (int b = lane; b < nb; b += 64) {
    const int ub = bverts[b];
    bvl[b] = ub;
    int cb[3];
    vcoords(g, ub, cb);
    const int bx = cb[0] - L.lo[0], by = cb[1] - L.lo[1], bz = cb[2] - L.lo[2];
    int ib = -1;
    double a = 0.0;
    for (int64_t e = rowptr[ub]; e < rowptr[ub + 1]; ++e) {
      const int d = colind[e] - ub;
      int jx = bx, jy = by, jz = bz;
      if (g.nx > 1 && (d == 1 || d == -1)) jx += d;
      else if (g.ny > 1 && (d == g.nx || d == -g.nx)) jy += d / g.nx;
      else if (g.nz > 1 && (d == g.nx * g.ny || d == -g.nx * g.ny)) jz += d / (g.nx * g.ny);
      else continue;
      if (jx >= 0 && jx < w0 && jy >= 0 && jy < w1 && jz >= 0 && jz < w2) {
        ib = jx + w0 * (jy + w1 * jz);
        a = vals[e];
      }
    }
    bi[b] = ib;
    ba[b] = a;
  }
  wave_sync();
  // lane i assembles row i of [A_II | A_IB]
  double r[WC];
#pragma unroll
  for (int s = 0; s < WC; ++s) r[s] = 0.0;
  if (lane < ni) {
    const int ix = lane % w0, iy = (lane / w0) % w1, iz = lane / (w0 * w1);
    const int u = (L.lo[0] + ix) + g.nx * ((L.lo[1] + iy) + g.ny * (L.lo[2] + iz));
    const int64_t e0 = rowptr[u], e1 = rowptr[u + 1];
    for (int64_t e = e0; e < e1; ++e) {
      const int w = colind[e];
      int slot = box_nbr(g, w0, w1, w2, ix, iy, iz, lane, u, w);
      if (slot < 0) {
        for (int b = 0; b < nb; ++b)
          if (bvl[b] == w) {
            slot = ni + b;
            break;
          }
      }
      const double v = vals[e];
#pragma unroll
      for (int s = 0; s < WC; ++s) r[s] = s == slot ? v : r[s];
    }
  }
  bool used = lane >= ni, singular = false;
  int my_step = 0;
  double my_d = 1.0;
  for (int k = 0; k < ni; ++k) {
    double a = used ? -1.0 : fabs(r[0]);
    int ia = used ? (1 << 30) : lane;
    wave_argmax(a, ia);
    int p = __builtin_amdgcn_readfirstlane(ia);
    if (p >= ni) {  // no comparable entry (NaN): take the first unused row
      p = __ffsll((unsigned long long)__ballot(!used)) - 1;
      singular = true;
    }
    wave_sync();
    if (lane == p) {
#pragma unroll
      for (int s = 0; s < WC; ++s) prow[s] = r[s];
    }
    wave_sync();
    const double d = prow[0];
    if (!(d != 0.0)) singular = true;
    const double inv_d = d != 0.0 ? 1.0 / d : 0.0;
    const bool is_p = lane == p;
    const double m = is_p ? 0.0 : r[0] * inv_d;
    // in chunks of 16 slots; the empty asm statements pin each chunk's
    // results before the next chunk's loads, so that the pivot row is never
    // held in registers whole
#pragma unroll
    for (int s0 = 1; s0 < WC; s0 += 16) {
#pragma unroll
      for (int s = s0; s < s0 + 16 && s < WC; ++s) r[s - 1] = fma(-m, prow[s], r[s]);
#pragma unroll
      for (int s = s0; s < s0 + 16 && s < WC; ++s) asm volatile("" : "+v"(r[s - 1])::"memory");
    }
    r[WC - 1] = is_p ? 1.0 : -m;
    if (is_p) {
      used = true;
      my_step = k;
      my_d = d;
    }
    if (lane == 0) pord[k] = p;
  }
  wave_sync();
  if (singular && lane == 0) flag_singular(status, level);
  for (int k = lane; k < ni; k += 64) piv[k] = pord[k];
  if (lane < ni) {
    const double sc = 1.0 / my_d;
#pragma unroll
    for (int s = 0; s < WC; ++s) r[s] *= sc;
  }
  // the inverse, transposed (entry (i, q) at q * ni + i), and X to LDS and,
  // transposed the same way, to memory for the backward solve
  T* Ainv = varena + L.lu_off;
  T* Xo = varena + L.x_off;
#pragma unroll
  for (int s = 0; s < WC; ++s) {
    const int k = s - (WC - ni);
    if (k >= 0) {
      const int q = pord[k];
      if (lane < ni) Ainv[size_t(q) * ni + my_step] = T(r[s]);
    } else if (s < nb) {
      if (lane < ni) {
        X[my_step * nb + s] = r[s];
        Xo[size_t(s) * ni + my_step] = T(r[s]);
      }
    }
  }
  wave_sync();
  // S = A_BI X, one boundary row at a time, lane = column
  T* S = varena + L.s_off;
  for (int b = 0; b < nb; ++b) {
    const int ib = bi[b];
    const double a = ba[b];
    for (int c = lane; c < nb; c += 64) S[size_t(b) * nb + c] = T(ib >= 0 ? a * X[ib * nb + c] : 0.0);
  }
}

// Level-L setup: sizes and DOF lists of the level-L segments.
__global__ void k_init_level(const DSeg* segs, int nseg, const int32_t* verts_ptr,
                             const int32_t* verts, int32_t* iarena, DLevelDyn dyn) {
  const int c = blockIdx.x;
  if (c >= nseg) return;
  const DSeg S = segs[c];
  const int n = verts_ptr[c + 1] - verts_ptr[c];
  int32_t* dofs = iarena + S.ioff;
  for (int i = threadIdx.x; i < n; i += blockDim.x) dofs[i] = verts[verts_ptr[c] + i];
  if (threadIdx.x == 0) {
    dyn.n[c] = n;
    dyn.k[c] = n;
    dyn.nr[c] = 0;
    dyn.h[c] = 0;
    dyn.passes[c] = 0;
    dyn.off[c] = 0;
    dyn.nfar[c] = 0;
  }
}

// Level-L blocks: A restricted to (c, d) minus the leaf Schur contributions.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_assemble_leafL(const DBlk* blks, int nblk, const DSeg* segs,
                                                       const int32_t* iarena_c, const DLevelDyn dyn,
                                                       const int32_t* lc_ptr, const DLeafContrib* lc,
                                                       const DLeaf* leaves, const int64_t* rowptr,
                                                       const int32_t* colind, const double* vals,
                                                       T* varena) {
  const int b = blockIdx.x;
  if (b >= nblk) return;
  const DBlk B = blks[b];
  const int nc = dyn.n[B.c], nd = dyn.n[B.d];
  const int32_t* dc = iarena_c + segs[B.c].ioff;
  const int32_t* dd = iarena_c + segs[B.d].ioff;
  T* out = varena + B.off;
  for (int t = threadIdx.x; t < nc * nd; t += NT) {
    const int i = t / nd, j = t % nd;
    double v = csr_at(rowptr, colind, vals, dc[i], dd[j]);
    for (int q = lc_ptr[b]; q < lc_ptr[b + 1]; ++q) {
      const DLeafContrib C = lc[q];
      const DLeaf Lf = leaves[C.leaf];
      v -= double(varena[Lf.s_off + size_t(C.oc + i) * Lf.nb + C.od + j]);
    }
    out[t] = T(v);
  }
}

// ---------------------------------------------------------------------------
// Per-segment interpolative decomposition (Sections 4.1-4.2).
// ---------------------------------------------------------------------------
struct IdParams {
  double eps;
  double tau;
  uint32_t seed;
  int h0;
  int probes;
  int level;
  int seg_base;           // index of this level's segments in h_init
  const int32_t* h_init;  // optional start samples (learned form)
  int sym;                // symmetric form: one-sided coupling rows (A_{n,c} only)
};

// LU with partial pivoting of the row-major n x n A (in place) by one block,
// three barriers per step and no division per trailing element: the update
// scales the pivot row by 1 / A[j][j] and reads column j unscaled, and
// column j is divided by its pivot in the next step, by all threads, while
// wave 0 searches the next pivot.  Steps j < split search rows [j, split),
// later steps rows [j, n); ties go to the smaller row.  piv[j] = row swapped
// with row j.  Returns 1 if a pivot was zero (that step is skipped).  With
// sym (symmetric form) no rows are interchanged: the LU of the symmetric
// block is then L D L^T, U = D L^T, and a pivot that is not positive is
// reported as well.
template <int NT>
__device__ inline int seg_block_lu(double* A, int n, int split, int* piv, int* s_piv, bool sym) {
  const int tid = threadIdx.x;
  int singular = 0;
  double dprev = 0.0;  // pivot of the previous step (0: nothing to scale)
  for (int j = 0; j < n; ++j) {
    if (tid < 64) {
      const int hi = sym ? j + 1 : (j < split ? split : n);
      double bv = -1.0;
      int bi = 1 << 30;
      for (int i = j + tid; i < hi; i += 64) {
        const double a = fabs(A[i * n + j]);
        if (a > bv) {
          bv = a;
          bi = i;
        }
      }
      wave_argmax(bv, bi);
      if (tid == 0) *s_piv = bi < n ? bi : j;
    }
    if (dprev != 0.0)
      for (int i = j + tid; i < n; i += NT) A[i * n + j - 1] /= dprev;
    __syncthreads();
    const int p = *s_piv;
    if (p != j)
      for (int c = tid; c < n; c += NT) {
        const double t = A[j * n + c];
        A[j * n + c] = A[p * n + c];
        A[p * n + c] = t;
      }
    if (tid == 0) piv[j] = p;
    __syncthreads();
    const double d = A[j * n + j];
    dprev = d;
    if (sym && !(d > 0.0)) singular = 1;
    if (d == 0.0) {
      singular = 1;
      continue;  // uniform; column j stays unscaled
    }
    const int m = n - j - 1;
    if (m > 0 && m <= NT) {
      const int rstep = NT / m, r0 = tid / m, col = j + 1 + (tid - r0 * m);
      if (r0 < rstep) {
        const double u = A[j * n + col] / d;
        for (int i = j + 1 + r0; i < n; i += rstep) A[i * n + col] -= A[i * n + j] * u;
      }
    } else if (m > NT) {
      for (int col = j + 1 + tid; col < n; col += NT) {
        const double u = A[j * n + col] / d;
        for (int i = j + 1; i < n; ++i) A[i * n + col] -= A[i * n + j] * u;
      }
    }
    __syncthreads();
  }
  // column n-1 has no rows below its pivot
  return singular;
}

// The LU without interchanges of the symmetric form (L D L^T, U = D L^T) by
// panels of 16 columns, for wide segments staged in scratch: each panel is
// factored by rows (one barrier per column), its rows of U are solved with
// the unit-lower panel triangle (one column per thread), and the trailing
// matrix takes the panel's rank-16 update on the matrix cores (FP64 16 x 64
// tiles, one wave per tile, operands read from memory), so the trailing
// matrix is read once per panel instead of once per column.  A pivot that is
// not positive is reported (returns 1); piv receives the identity.
template <int NT>
__device__ inline int seg_block_ldl_panels(double* A, int n, int* piv) {
  constexpr int NB = 16, NW = NT / 64;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  int singular = 0;
  for (int i = tid; i < n; i += NT) piv[i] = i;
  for (int jb = 0; jb < n; jb += NB) {
    const int je = jb + NB < n ? jb + NB : n, nb = je - jb;
    // 1. the panel: columns jb..je-1, rows below each pivot
    for (int j = jb; j < je; ++j) {
      const double d = A[size_t(j) * n + j];
      if (!(d > 0.0)) singular = 1;
      for (int i = j + 1 + tid; i < n; i += NT) {
        const double l = A[size_t(i) * n + j] / d;
        A[size_t(i) * n + j] = l;
        for (int c = j + 1; c < je; ++c) A[size_t(i) * n + c] -= l * A[size_t(j) * n + c];
      }
      __syncthreads();
    }
    if (je == n) break;
    // 2. rows jb..je-1 of U right of the panel: L11^{-1} A12
    for (int c = je + tid; c < n; c += NT)
      for (int j = jb; j < je; ++j) {
        const double u = A[size_t(j) * n + c];
        for (int i = j + 1; i < je; ++i) A[size_t(i) * n + c] -= A[size_t(i) * n + j] * u;
      }
    __syncthreads();
    // 3. trailing matrix: A22 -= L21 U12
    const int m = n - je, nti = (m + 15) >> 4, ncg = (m + 63) >> 6;
    for (int unit = w; unit < nti * ncg; unit += NW) {
      const int ti = unit / ncg, cg = unit - ti * ncg, i0 = je + 16 * ti, j0 = je + 64 * cg;
      const int nct = ((n - j0 < 64 ? n - j0 : 64) + 15) >> 4;
      gg_v4 acc[4] = {};
      wave_tile_mfma(
          [&](int i, int u) {
            const double v = A[size_t(i < n ? i : n - 1) * n + jb + (u < nb ? u : nb - 1)];
            return i < n && u < nb ? v : 0.0;
          },
          [&](int u, int col) {
            const int c = j0 + col;
            return A[size_t(jb + (u < nb ? u : nb - 1)) * n + (c < n ? c : n - 1)];
          },
          i0, 0, nb, nct, acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + lk + 4 * r;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int c = j0 + 16 * cc + li;
          if (i < n && c < n && cc < nct) A[size_t(i) * n + c] -= acc[cc][r];
        }
      }
    }
    __syncthreads();
  }
  return singular;
}

// Packed inverses of the unit-lower L and upper U held in W (row-major
// n x n): out[i][c] = (L^{-1})[i][c] for i > c, (U^{-1})[i][c] for i <= c.
// L^{-1} by forward elimination of the identity and U^{-1} = (D^{-1} U)^{-1}
// D^{-1} by back elimination, both in X (n x n): step s eliminates column s
// of L and column n-1-s of U (disjoint triangles of X, one barrier per
// step).  The diagonal of X holds 1 / U[i][i]; the unit diagonals are
// implied.
//
// With sym (the L D L^T of the symmetric form, U = D L^T) the stored pair is
// balanced by Delta = D^{1/2}: R = Delta^{-1} L^{-1} (lower, its strict part
// stored, its diagonal 1 / Delta the same as that of the stored upper part)
// and C = U^{-1} Delta = R^T, so the row scaling R and the column scaling C
// are the Cholesky ones, C_ch^{-1} and C_ch^{-T} with C_ch = L Delta, and
// every scaled coupling keeps the level's matrix symmetric.  Row operations
// with the stored form then multiply row i's own entry by the stored
// diagonal instead of taking a unit diagonal.
__device__ inline double balance_entry(double v, int i, int c, double xii, double xcc) {
  // xii, xcc: 1 / U_ii and 1 / U_cc; Delta_i = 1 / sqrt(xii)
  return i > c ? v * sqrt(xii) : v / sqrt(xcc);
}

// The same packed inverses by panels of 16 rows, for wide segments staged
// in scratch: X holds L^{-1} (strict lower part, unit diagonal implied) and
// U^{-1} (upper part with its diagonal) directly.  L^{-1} by row panels from
// the top: the panel rows' products with the finished rows above (FP64
// 16 x 64 matrix-core tiles, operands read from memory), then a forward
// substitution inside the panel, one barrier per row; U^{-1} likewise by row
// panels from the bottom with a backward substitution.  The stored form is
// that of seg_block_inverse, balanced in the symmetric form.
template <int NT, typename TO>
__device__ inline void seg_block_inverse_panels(const double* W, int n, double* X, TO* out, bool sym) {
  constexpr int NB = 16, NW = NT / 64;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  // L^{-1}: row i, column c < i is -(sum over c <= u < i of L[i][u] Linv[u][c]), Linv[c][c] = 1
  auto linv = [&](int u, int c) { return u > c ? X[size_t(u) * n + c] : (u == c ? 1.0 : 0.0); };
  for (int ib = 0; ib < n; ib += NB) {
    const int ie = ib + NB < n ? ib + NB : n;
    // columns c < ib: the rows above the panel
    const int ncg = (ib + 63) >> 6;
    for (int cg = w; cg < ncg; cg += NW) {
      const int j0 = 64 * cg;
      const int nct = ((ib - j0 < 64 ? ib - j0 : 64) + 15) >> 4;
      gg_v4 acc[4] = {};
      wave_tile_mfma(
          [&](int i, int u) {
            const double l = W[size_t(i < ie ? i : ie - 1) * n + (u < ib ? u : ib - 1)];
            return i < ie && u < ib ? l : 0.0;
          },
          [&](int u, int col) {
            const int c = j0 + col;
            return u < ib && c < ib ? linv(u, c) : 0.0;
          },
          ib, j0, ib, nct, acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ib + lk + 4 * r;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int c = j0 + 16 * cc + li;
          if (i < ie && c < ib && cc < nct) X[size_t(i) * n + c] = -acc[cc][r];
        }
      }
    }
    __syncthreads();
    // inside the panel, row by row
    for (int i = ib; i < ie; ++i) {
      for (int c = tid; c < i; c += NT) {
        double v = c < ib ? X[size_t(i) * n + c] : 0.0;
        for (int u = c > ib ? c : ib; u < i; ++u) v -= W[size_t(i) * n + u] * linv(u, c);
        X[size_t(i) * n + c] = v;
      }
      __syncthreads();
    }
  }
  // U^{-1}: row i, column c >= i is (delta_ic - sum over i < u <= c of U[i][u] Uinv[u][c]) / U[i][i]
  auto uinv = [&](int u, int c) { return u <= c ? X[size_t(u) * n + c] : 0.0; };
  for (int ie = n; ie > 0; ie -= NB) {
    const int ib = ie - NB > 0 ? ie - NB : 0;
    // columns c >= ie: the rows below the panel
    const int m = n - ie, ncg = (m + 63) >> 6;
    for (int cg = w; cg < ncg; cg += NW) {
      const int j0 = ie + 64 * cg;
      const int nct = ((n - j0 < 64 ? n - j0 : 64) + 15) >> 4;
      const int u1 = j0 + 64 < n ? j0 + 64 : n;  // rows u <= c of the group's columns
      gg_v4 acc[4] = {};
      wave_tile_mfma(
          [&](int i, int u) {
            const double v = W[size_t(i < ie ? i : ie - 1) * n + (u < n ? u : n - 1)];
            return i < ie && u >= ie && u < u1 ? v : 0.0;
          },
          [&](int u, int col) {
            const int c = j0 + col;
            return u >= ie && u < n && c < n ? uinv(u, c) : 0.0;
          },
          ib, ie, u1, nct, acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ib + lk + 4 * r;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int c = j0 + 16 * cc + li;
          if (i < ie && c < n && cc < nct) X[size_t(i) * n + c] = -acc[cc][r];
        }
      }
    }
    __syncthreads();
    for (int i = ie - 1; i >= ib; --i) {
      const double d = W[size_t(i) * n + i];
      for (int c = i + tid; c < n; c += NT) {
        double v = (c == i ? 1.0 : 0.0) + (c >= ie ? X[size_t(i) * n + c] : 0.0);
        const int ue = c + 1 < ie ? c + 1 : ie;
        for (int u = i + 1; u < ue; ++u) v -= W[size_t(i) * n + u] * uinv(u, c);
        X[size_t(i) * n + c] = v / d;
      }
      __syncthreads();
    }
  }
  for (int t = tid; t < n * n; t += NT) {
    const int i = t / n, c = t - i * n;
    const double v = X[t];
    out[t] = TO(sym ? balance_entry(v, i, c, X[size_t(i) * n + i], X[size_t(c) * n + c]) : v);
  }
  __syncthreads();
}

template <int NT, typename TO>
__device__ inline void seg_block_inverse(const double* W, int n, double* X, TO* out, bool sym) {
  const int tid = threadIdx.x;
  for (int t = tid; t < n * n; t += NT) {
    const int i = t / n, c = t - i * n;
    X[t] = i == c ? 1.0 / W[t] : 0.0;
  }
  __syncthreads();
  for (int s = 0; s < n - 1; ++s) {
    const int jl = s, ju = n - 1 - s;
    const int R = n - 1 - s, C = s + 1;  // rows and columns of both updates
    for (int c0 = 0; c0 < C; c0 += NT) {
      const int cw = C - c0 < NT ? C - c0 : NT;
      const int rstep = NT / cw, r0 = tid / cw, cq = c0 + tid - r0 * cw;
      if (r0 < rstep) {
        // L: X[jl+1+r][cq] -= L[jl+1+r][jl] X[jl][cq]  (X[jl][jl] = 1)
        const double xl = cq == jl ? 1.0 : X[jl * n + cq];
        // U: X[r][ju+cq] -= (U[r][ju] / U[r][r]) X[ju][ju+cq]  (X[ju][ju] = 1)
        const int cu = ju + cq;
        const double xu = cq == 0 ? 1.0 : X[ju * n + cu];
        for (int r = r0; r < R; r += rstep) {
          const int il = jl + 1 + r;
          X[il * n + cq] -= W[il * n + jl] * xl;
          X[r * n + cu] -= W[r * n + ju] * X[r * n + r] * xu;
        }
      }
    }
    __syncthreads();
  }
  for (int t = tid; t < n * n; t += NT) {
    const int i = t / n, c = t - i * n;
    const double v = i > c ? X[t] : (i == c ? 1.0 : X[t]) * X[c * n + c];
    out[t] = TO(sym ? balance_entry(v, i, c, X[i * n + i], X[c * n + c]) : v);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Transform U_t A L_t of the diagonal block and two-stage LU (eqs. (2.7),
// (4.10)); the DOF list is reordered to [remainder; skeleton].
// ---------------------------------------------------------------------------
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_seg_lu(const DSeg* segs, int nseg, const DBlk* blks,
                                               int32_t* iarena, T* varena, double* scratch,
                                               DLevelDyn dyn, int* status, int need_lo, int need_hi,
                                               int lds_doubles, int level, int sym) {
  extern __shared__ double lds[];
  __shared__ int s_piv;
  const int c = blockIdx.x;
  if (c >= nseg) return;
  const int tid = threadIdx.x;
  const DSeg S = segs[c];
  const int n = dyn.n[c];
  if (n == 0) return;
  // this launch takes the segments whose staging need 2 n^2 (doubles) lies
  // in (need_lo, need_hi]; they work in LDS if it fits, else in scratch
  const int need = 2 * n * n;
  if (need <= need_lo || need > need_hi) return;
  const int k = dyn.k[c], nr = dyn.nr[c];
  const bool sp = dyn.passes[c] > 0;
  int32_t* dofs = iarena + S.ioff;
  int32_t* perm = dofs + S.cap;
  int32_t* piv = perm + S.cap;
  int32_t* tmp = piv + S.cap;  // tag region, >= cap ints
  const T* M = varena + blks[S.diag_blk].off;
  const bool inlds = need <= lds_doubles;
  double* W = inlds ? lds : scratch + S.scr_off;
  double* X = W + size_t(n) * n;  // gather map, then T, then the inverse workspace
  int* om = reinterpret_cast<int*>(X);
  // gather in [r; s] order: row/column p of W is om[p] = perm[k + p]
  // (p < nr), perm[p - nr] (p >= nr) of the block; the block's entries are
  // loaded in batches
  for (int p = tid; p < n; p += NT) om[p] = sp ? (p < nr ? perm[k + p] : perm[p - nr]) : p;
  __syncthreads();
  load_batched<8>(
      n * n, tid, NT,
      [&](int t) {
        const int p = t / n, q = t - p * n;
        return M[size_t(om[p]) * n + om[q]];
      },
      [&](int t, T v) { W[t] = double(v); });
  __syncthreads();
  if (sp && nr > 0 && k > 0) {
    // T (k x nr) staged next to W
    stage_batched<8>(varena + S.t_off, k * nr, tid, NT, [&](int t, T v) { X[t] = double(v); });
    __syncthreads();
    // columns: W[:, q] -= W[:, nr:] T[:, q]
    for (int t = tid; t < n * nr; t += NT) {
      const int p = t / nr, q = t - p * nr;
      double s = 0.0;
      for (int i = 0; i < k; ++i) s += W[size_t(p) * n + nr + i] * X[i * nr + q];
      W[size_t(p) * n + q] -= s;
    }
    __syncthreads();
    // rows: W[p, :] -= T[:, p]^T W[nr:, :]
    for (int t = tid; t < nr * n; t += NT) {
      const int p = t / n, q = t - p * n;
      double s = 0.0;
      for (int i = 0; i < k; ++i) s += X[i * nr + p] * W[size_t(nr + i) * n + q];
      W[size_t(p) * n + q] -= s;
    }
    __syncthreads();
  }
  // pivots in LDS while the LU runs (a global store before every barrier
  // would stall each step), copied out afterwards
  const bool pv_lds = inlds && need + (n + 1) / 2 <= lds_doubles;
  int* pv = pv_lds ? reinterpret_cast<int*>(lds + need) : piv;
  // wide symmetric-form segments (in scratch) by panels, the others step by step
  const bool panels = NT >= 1024 && sym && !inlds;
  if (panels ? seg_block_ldl_panels<NT>(W, n, pv) : seg_block_lu<NT>(W, n, sp ? nr : 0, pv, &s_piv, sym != 0))
    flag_singular(status, level);
  __syncthreads();
  // stored form of the interchanges: the composed row map (row i of P X is
  // row piv[i] of X), each entry traced back through the interchanges
  for (int i = tid; i < n; i += NT) {
    int pos = i;
    for (int r = n - 1; r >= 0; --r) {
      const int p = pv[r];
      pos = pos == r ? p : pos == p ? r : pos;
    }
    tmp[i] = pos;
  }
  __syncthreads();
  for (int i = tid; i < n; i += NT) piv[i] = tmp[i];
  __syncthreads();
  // packed inverses: strictly lower part of L^{-1} (unit diagonal implied)
  // and upper part of U^{-1}, so every later application is a product
  T* LU = varena + S.lu_off;
  if (NT >= 1024 && !inlds)
    seg_block_inverse_panels<NT>(W, n, X, LU, sym != 0);
  else
    seg_block_inverse<NT>(W, n, X, LU, sym != 0);
  if (sp) {
    for (int p = tid; p < n; p += NT) tmp[p] = dofs[p < nr ? perm[k + p] : perm[p - nr]];
    __syncthreads();
    for (int p = tid; p < n; p += NT) dofs[p] = tmp[p];
  }
}

// One wave per segment of at most 64 * CPL DOFs, lane l owning columns (and
// rows) l, l + 64, ...: the transform and the two-stage LU of k_seg_lu with
// wave-level synchronisation only, then the packed inverses formed in place.
// LDS: W (n x n, row-major), then T (k x nr), which first holds the gather
// map.  Segments with nmin < n <= nmax take part.  The factorization launches
// it with one column per lane for segments of up to 32 DOFs; wider ones go to
// the 256-thread k_seg_lu, which is faster there.
__host__ __device__ inline int seglu_wave_lds_doubles(int nw) { return nw * nw + (nw * nw + 3) / 4 + 1; }

template <typename T, int CPL>
__global__ __launch_bounds__(64) void k_seg_lu_wave(const DSeg* segs, int nseg, const DBlk* blks,
                                                    int32_t* iarena, T* varena, DLevelDyn dyn, int* status,
                                                    int nmin, int nmax, int level, int sym) {
  extern __shared__ double lds[];
  const int c = blockIdx.x;
  if (c >= nseg) return;
  const int lane = threadIdx.x;
  const DSeg S = segs[c];
  const int n = dyn.n[c];
  if (n == 0 || n <= nmin || n > nmax) return;
  const int k = dyn.k[c], nr = dyn.nr[c];
  const bool sp = dyn.passes[c] > 0;
  int32_t* dofs = iarena + S.ioff;
  int32_t* perm = dofs + S.cap;
  int32_t* piv = perm + S.cap;
  const T* M = varena + blks[S.diag_blk].off;
  double* W = lds;
  double* X = lds + size_t(n) * n;
  int* om = reinterpret_cast<int*>(X);
  // gather in [r; s] order: row/column p of W is om[p] = perm[k + p]
  // (p < nr), perm[p - nr] (p >= nr) of the block
  {
    int ov[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int p = lane + 64 * u < n ? lane + 64 * u : n - 1;
      ov[u] = sp ? (p < nr ? perm[k + p] : perm[p - nr]) : p;
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u)
      if (lane + 64 * u < n) om[lane + 64 * u] = ov[u];
  }
  wave_sync();
  load_batched<8>(
      n * n, lane, 64,
      [&](int t) {
        const int p = t / n, q = t - p * n;
        return M[size_t(om[p]) * n + om[q]];
      },
      [&](int t, T v) { W[t] = double(v); });
  wave_sync();
  if (sp && nr > 0 && k > 0) {
    const T* Tm = varena + S.t_off;
    load_batched<8>(k * nr, lane, 64, [&](int t) { return Tm[t]; }, [&](int t, T v) { X[t] = double(v); });
    wave_sync();
    // columns: W[:, q] -= W[:, nr:] T[:, q]  (q < nr)
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int q = lane + 64 * u;
      if (q < nr)
        for (int p = 0; p < n; ++p) {
          double s = 0.0;
          for (int i = 0; i < k; ++i) s += W[p * n + nr + i] * X[i * nr + q];
          W[p * n + q] -= s;
        }
    }
    wave_sync();
    // rows: W[p, :] -= T[:, p]^T W[nr:, :]  (p < nr)
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int q = lane + 64 * u;
      if (q < n)
        for (int p = 0; p < nr; ++p) {
          double s = 0.0;
          for (int i = 0; i < k; ++i) s += X[i * nr + p] * W[(nr + i) * n + q];
          W[p * n + q] -= s;
        }
    }
    wave_sync();
  }
  // LU with partial pivoting; steps j < nr search rows [j, nr), later steps
  // [j, n); ties go to the smaller row
  const int split = sp ? nr : 0;
  bool singular = false;
  int rm[CPL];  // composed row map of the interchanges so far, rows l + 64 u
#pragma unroll
  for (int u = 0; u < CPL; ++u) rm[u] = lane + 64 * u;
  for (int j = 0; j < n; ++j) {
    const int hi = sym ? j + 1 : (j < split ? split : n);  // symmetric form: no interchanges
    double bv = -1.0;
    int bi = 1 << 30;
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int r = lane + 64 * u;
      if (r >= j && r < hi) {
        const double a = fabs(W[r * n + j]);
        if (a > bv) {
          bv = a;
          bi = r;
        }
      }
    }
    wave_argmax(bv, bi);
    const int p = __builtin_amdgcn_readfirstlane(bi < n ? bi : j);
    if (p != j) {
      int a = 0, b = 0;
#pragma unroll
      for (int u = 0; u < CPL; ++u) {
        const int va = __builtin_amdgcn_readlane(rm[u], j & 63), vb = __builtin_amdgcn_readlane(rm[u], p & 63);
        if ((j >> 6) == u) a = va;
        if ((p >> 6) == u) b = vb;
      }
#pragma unroll
      for (int u = 0; u < CPL; ++u) {
        const int r = lane + 64 * u;
        rm[u] = r == j ? b : r == p ? a : rm[u];
        if (r < n) {
          const double t = W[j * n + r];
          W[j * n + r] = W[p * n + r];
          W[p * n + r] = t;
        }
      }
    }
    wave_sync();
    const double d = W[j * n + j];
    if (sym && !(d > 0.0)) singular = true;
    if (d == 0.0) {
      singular = true;
      continue;
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int r = lane + 64 * u;
      if (r > j && r < n) W[r * n + j] /= d;
    }
    wave_sync();
    // trailing update of the columns owned by this lane; inactive columns
    // read a valid column and do not store
    bool act[CPL], any = false;
    int cc[CPL];
    double ujc[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int col = lane + 64 * u;
      act[u] = col > j && col < n;
      any = any || act[u];
      cc[u] = act[u] ? col : j;
      ujc[u] = W[j * n + cc[u]];
    }
    if (any) {
      int i = j + 1;
      for (; i + 7 < n; i += 8) {
        double l[8], w[8][CPL];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          l[v] = W[(i + v) * n + j];
#pragma unroll
          for (int u = 0; u < CPL; ++u) w[v][u] = W[(i + v) * n + cc[u]];
        }
#pragma unroll
        for (int v = 0; v < 8; ++v)
#pragma unroll
          for (int u = 0; u < CPL; ++u)
            if (act[u]) W[(i + v) * n + cc[u]] = w[v][u] - l[v] * ujc[u];
      }
      for (; i < n; ++i) {
        const double lv = W[i * n + j];
#pragma unroll
        for (int u = 0; u < CPL; ++u)
          if (act[u]) W[i * n + cc[u]] -= lv * ujc[u];
      }
    }
    wave_sync();
  }
  if (singular && lane == 0) flag_singular(status, level);
#pragma unroll
  for (int u = 0; u < CPL; ++u)
    if (lane + 64 * u < n) piv[lane + 64 * u] = rm[u];
  // packed inverses in place: step s forms row s of L^{-1} (columns < s,
  // from the finished rows above it) and row n-1-s of U^{-1} (columns
  // >= n-1-s, from the finished rows below it); the two touch disjoint
  // triangles, and each row is written only after every lane has read it
  for (int s = 0; s < n; ++s) {
    const int il = s, iu = n - 1 - s;
    const double du = W[iu * n + iu];
    double sl[CPL], su[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int col = lane + 64 * u;
      const bool al = col < il, au = col >= iu && col < n;
      const int cl = al ? col : 0, cu = au ? col : iu;
      // L: X[il][col] = -(L[il][col] + sum_{col < m < il} L[il][m] X[m][col])
      // U: Y[iu][col] = (delta - sum_{iu < m <= col} U[iu][m] Y[m][col]) / U[iu][iu]
      const int nl = al ? il - 1 - cl : 0, nu = au ? cu - iu : 0;
      const int len = nl > nu ? nl : nu;
      double accl = al ? W[il * n + cl] : 0.0, accu = 0.0;
      for (int t = 0; t < len; t += 4) {
        double a[4], b[4], e[4], f[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ml = t + v < nl ? cl + 1 + t + v : cl;
          const int mu = t + v < nu ? iu + 1 + t + v : iu;
          a[v] = W[il * n + ml];
          b[v] = W[ml * n + cl];
          e[v] = W[iu * n + mu];
          f[v] = W[mu * n + cu];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          accl += t + v < nl ? a[v] * b[v] : 0.0;
          accu += t + v < nu ? e[v] * f[v] : 0.0;
        }
      }
      sl[u] = -accl;
      su[u] = ((col == iu ? 1.0 : 0.0) - accu) / du;
    }
    wave_sync();
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int col = lane + 64 * u;
      if (col < il) W[il * n + col] = sl[u];
      if (col >= iu && col < n) W[iu * n + col] = su[u];
    }
    wave_sync();
  }
  T* LU = varena + S.lu_off;
  for (int t = lane; t < n * n; t += 64) {
    const int i = t / n, c = t - i * n;
    LU[t] = T(sym ? balance_entry(W[t], i, c, W[i * n + i], W[c * n + c]) : W[t]);
  }
  if (sp) {
    int nd[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int p = lane + 64 * u < n ? lane + 64 * u : n - 1;
      nd[u] = dofs[p < nr ? perm[k + p] : perm[p - nr]];
    }
    wave_sync();
#pragma unroll
    for (int u = 0; u < CPL; ++u)
      if (lane + 64 * u < n) dofs[lane + 64 * u] = nd[u];
  }
}

// LDS doubles of the one-wave coupling scaling of a kc x kd block: the block
// in FP64, the two triangles in the storage type (vs bytes each), the maps.
__host__ __device__ inline int blk_scale_wave_need(int kc, int kd, int vs) {
  return kc * kd + ((kc * kc + kd * kd) * vs + 7) / 8 + (kc + kd + 1) / 2;
}
template <typename T>
__host__ __device__ inline bool blk_scale_wave_fits(int kc, int kd, int lds_doubles) {
  return kc <= 64 && kd <= 64 && blk_scale_wave_need(kc, kd, int(sizeof(T))) <= lds_doubles;
}
// LDS bytes of the matrix-core coupling scaling of a kc x kd block (the
// gathered block and L^{-1} times it in FP64, the row and column maps).
constexpr int SCALE_MFMA_MAX = 155648;
__host__ __device__ inline size_t blk_scale_mfma_bytes(int kc, int kd) {
  return size_t(2) * kc * kd * 8 + size_t(kc + kd) * 4 + 16;
}
__host__ __device__ inline bool blk_scale_mfma_fits(int kc, int kd, int lds_bytes) {
  return kc <= 128 && kd <= 128 && blk_scale_mfma_bytes(kc, kd) <= size_t(lds_bytes);
}

// Coupling scaling: A'_{cd} = L_ss,c^{-1} P_s,c A_cd[s_c, s_d] U_ss,d^{-1},
// with the skeleton blocks of the packed inverses of c and d (the inverse of
// a block triangular matrix has the inverse of its trailing diagonal block as
// its trailing diagonal block).  In the symmetric form (sym) the row
// operator's diagonal is the stored diagonal (the balanced pair R, C of
// seg_block_inverse) and P is the identity.
template <typename T>
__global__ __launch_bounds__(WG) void k_blk_scale(const DBlk* blks, const int32_t* blk_list, int nlist,
                                                  const DSeg* segs, const int32_t* iarena, T* varena,
                                                  DLevelDyn dyn, int wave_lds_doubles, int mfma_lds, int sym) {
  extern __shared__ double lds[];
  const int bi = blockIdx.x;
  if (bi >= nlist) return;
  const int tid = threadIdx.x;
  const DBlk B = blks[blk_list[bi]];
  const int c = B.c, d = B.d;
  const int nc = dyn.n[c], nd = dyn.n[d];
  const int kc = dyn.k[c], kd = dyn.k[d];
  const int nrc = dyn.nr[c], nrd = dyn.nr[d];
  if (kc == 0 || kd == 0) return;
  if (blk_scale_wave_fits<T>(kc, kd, wave_lds_doubles)) return;  // taken by k_blk_scale_wave
  if (blk_scale_mfma_fits(kc, kd, mfma_lds)) return;          // taken by k_blk_scale_mfma
  const bool spc = dyn.passes[c] > 0, spd = dyn.passes[d] > 0;
  const int32_t* permc = iarena + segs[c].ioff + segs[c].cap;
  const int32_t* permd = iarena + segs[d].ioff + segs[d].cap;
  const int32_t* pivc = permc + segs[c].cap;
  const T* A = varena + B.off;
  T* out = varena + B.soff;
  const T* Lc = varena + segs[c].lu_off;  // packed inverse of c
  const T* Ud = varena + segs[d].lu_off;  // packed inverse of d
  // block row of row i of P_s A_cd[s_c, s_d] and block column of column j,
  // in the dynamic LDS (LDS_DOUBLES * 2 ints)
  int* rs = reinterpret_cast<int*>(lds);
  int* cs = rs + kc;
  if (kc + kd > 2 * LDS_DOUBLES) {
    // (beyond every layout this library builds) poison the block so the
    // residual check reports it
    for (int t = tid; t < kc * kd; t += WG) out[t] = T(NAN);
    return;
  }
  for (int i = tid; i < kc; i += WG) {
    const int r = pivc[nrc + i] - nrc;
    rs[i] = spc ? permc[r] : r;
  }
  for (int j = tid; j < kd; j += WG) cs[j] = spd ? permd[j] : j;
  __syncthreads();
  // products on the matrix cores (FP64) in 16 x 64 tiles, operator entries
  // read from memory: first Y = L^{-1} X into the output region (the stored
  // diagonal in the symmetric form), then out = Y U^{-1} in place, each wave
  // owning whole 16-row stripes and taking their column groups from the
  // right, so a tile only reads columns that no tile has overwritten yet
  const int w = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int nti = (kc + 15) >> 4, ncg = (kd + 63) >> 6;
  for (int unit = w; unit < nti * ncg; unit += NWAVE) {
    const int ti = unit / ncg, cg = unit - ti * ncg, i0 = 16 * ti, j0 = 64 * cg;
    const int nct = ((kd - j0 < 64 ? kd - j0 : 64) + 15) >> 4;
    gg_v4 acc[4] = {};
    wave_tile_mfma(
        [&](int i, int u) {
          const double l = double(Lc[size_t(nrc + (i < kc ? i : kc - 1)) * nc + nrc + (u < kc ? u : kc - 1)]);
          return i < kc && u < i ? l : (i < kc && u == i ? (sym ? l : 1.0) : 0.0);
        },
        [&](int u, int col) {
          const int j = j0 + col;
          return double(A[size_t(rs[u < kc ? u : kc - 1]) * nd + cs[j < kd ? j : kd - 1]]);
        },
        i0, 0, i0 + 16 < kc ? i0 + 16 : kc, nct, acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + lk + 4 * r;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const int j = j0 + 16 * cc + li;
        if (i < kc && j < kd && cc < nct) out[size_t(i) * kd + j] = T(acc[cc][r]);
      }
    }
  }
  __syncthreads();
  for (int ti = w; ti < nti; ti += NWAVE) {
    const int i0 = 16 * ti;
    for (int cg = ncg - 1; cg >= 0; --cg) {
      const int j0 = 64 * cg;
      const int nct = ((kd - j0 < 64 ? kd - j0 : 64) + 15) >> 4;
      const int u1 = j0 + 64 < kd ? j0 + 64 : kd;
      gg_v4 acc[4] = {};
      wave_tile_mfma(
          [&](int i, int u) {
            const double y = double(out[size_t(i < kc ? i : kc - 1) * kd + (u < u1 ? u : u1 - 1)]);
            return i < kc && u < u1 ? y : 0.0;
          },
          [&](int u, int col) {
            const int j = j0 + col;
            const double uv = double(Ud[size_t(nrd + (u < kd ? u : kd - 1)) * nd + nrd + (j < kd ? j : kd - 1)]);
            return u <= j && j < kd ? uv : 0.0;
          },
          i0, 0, u1, nct, acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + lk + 4 * r;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int j = j0 + 16 * cc + li;
          if (i < kc && j < kd && cc < nct) out[size_t(i) * kd + j] = T(acc[cc][r]);
        }
      }
    }
  }
}

// The same coupling scaling on the matrix cores, four waves per block, for
// blocks beyond the one-wave kernel whose skeletons hold at most 128 DOFs:
// the gathered block X and Y = L_c^{-1} X stay in LDS in FP64; Y is formed
// in 16 x 64 tiles with the entries of the packed inverse of c read from
// memory, then out = Y U_d^{-1} is formed transposed, out^T = U_d^{-T} Y^T,
// so that the entries of U_d^{-1} are the ones read from memory too.
template <typename T>
__global__ __launch_bounds__(WG) void k_blk_scale_mfma(const DBlk* blks, const int32_t* blk_list, int nlist,
                                                       const DSeg* segs, const int32_t* iarena, T* varena,
                                                       DLevelDyn dyn, int wave_lds_doubles, int mfma_lds, int sym) {
  extern __shared__ double lds[];
  const int bi = blockIdx.x;
  if (bi >= nlist) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const DBlk B = blks[blk_list[bi]];
  const int c = B.c, d = B.d;
  const int kc = dyn.k[c], kd = dyn.k[d];
  if (kc == 0 || kd == 0) return;
  if (blk_scale_wave_fits<T>(kc, kd, wave_lds_doubles) || !blk_scale_mfma_fits(kc, kd, mfma_lds)) return;
  const int nc = dyn.n[c], nd = dyn.n[d];
  const int nrc = dyn.nr[c], nrd = dyn.nr[d];
  const bool spc = dyn.passes[c] > 0, spd = dyn.passes[d] > 0;
  const int32_t* permc = iarena + segs[c].ioff + segs[c].cap;
  const int32_t* permd = iarena + segs[d].ioff + segs[d].cap;
  const int32_t* pivc = permc + segs[c].cap;
  const T* A = varena + B.off;
  T* out = varena + B.soff;
  const T* Lc = varena + segs[c].lu_off;
  const T* Ud = varena + segs[d].lu_off;
  double* X = lds;            // kc x kd: P_s A_cd[s_c, s_d]
  double* Y = X + kc * kd;    // kc x kd: L^{-1} X
  int* rs = reinterpret_cast<int*>(Y + kc * kd);  // kc: block row of row i of P_s X
  int* cs = rs + kc;                              // kd: block column of column j
  for (int i = tid; i < kc; i += WG) {
    const int r = pivc[nrc + i] - nrc;
    rs[i] = spc ? permc[r] : r;
  }
  for (int j = tid; j < kd; j += WG) cs[j] = spd ? permd[j] : j;
  __syncthreads();
  load_batched<8>(
      kc * kd, tid, WG,
      [&](int t) {
        const int i = t / kd, j = t - i * kd;
        return A[size_t(rs[i]) * nd + cs[j]];
      },
      [&](int t, T v) { X[t] = double(v); });
  __syncthreads();
  // Y = L^{-1} X (unit lower; the stored diagonal in the symmetric form):
  // row tile i0 needs columns u <= i of L^{-1}
  const int nti = (kc + 15) >> 4, ncg = (kd + 63) >> 6;
  for (int unit = w; unit < nti * ncg; unit += NWAVE) {
    const int ti = unit / ncg, cg = unit - ti * ncg, i0 = 16 * ti, j0 = 64 * cg;
    const int nct = ((kd - j0 < 64 ? kd - j0 : 64) + 15) >> 4;
    gg_v4 acc[4] = {};
    wave_tile_mfma(
        [&](int i, int u) {
          const double l = double(Lc[size_t(nrc + (i < kc ? i : kc - 1)) * nc + nrc + (u < kc ? u : kc - 1)]);
          return i < kc && u < i ? l : (i < kc && u == i ? (sym ? l : 1.0) : 0.0);
        },
        [&](int u, int col) {
          const int j = j0 + col;
          return X[(u < kc ? u : kc - 1) * kd + (j < kd ? j : kd - 1)];
        },
        i0, 0, i0 + 16 < kc ? i0 + 16 : kc, nct, acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + lk + 4 * r;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const int j = j0 + 16 * cc + li;
        if (i < kc && j < kd && cc < nct) Y[i * kd + j] = acc[cc][r];
      }
    }
  }
  __syncthreads();
  // out^T = U^{-T} Y^T: row tile j0 of out^T (columns j of out) needs rows
  // u <= j of U^{-1}
  const int ntj = (kd + 15) >> 4, ncgi = (kc + 63) >> 6;
  for (int unit = w; unit < ntj * ncgi; unit += NWAVE) {
    const int tj = unit / ncgi, cg = unit - tj * ncgi, j0 = 16 * tj, i0 = 64 * cg;
    const int nct = ((kc - i0 < 64 ? kc - i0 : 64) + 15) >> 4;
    gg_v4 acc[4] = {};
    wave_tile_mfma(
        [&](int j, int u) {
          const double uv = double(Ud[size_t(nrd + (u < kd ? u : kd - 1)) * nd + nrd + (j < kd ? j : kd - 1)]);
          return j < kd && u <= j ? uv : 0.0;
        },
        [&](int u, int col) {
          const int i = i0 + col;
          return Y[(i < kc ? i : kc - 1) * kd + (u < kd ? u : kd - 1)];
        },
        j0, 0, j0 + 16 < kd ? j0 + 16 : kd, nct, acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = j0 + lk + 4 * r;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const int i = i0 + 16 * cc + li;
        if (j < kd && i < kc && cc < nct) out[size_t(i) * kd + j] = T(acc[cc][r]);
      }
    }
  }
}

// The same coupling scaling with one wave per block (skeletons of at most
// 64 DOFs, staging within lds_doubles): the block, the skeleton part of
// L_c^{-1} and of U_d^{-1} are fetched into LDS with independent loads; lane
// j then owns column j of the block.
template <typename T>
__global__ __launch_bounds__(64) void k_blk_scale_wave(const DBlk* blks, const int32_t* blk_list, int nlist,
                                                       const DSeg* segs, const int32_t* iarena, T* varena,
                                                       DLevelDyn dyn, int lds_doubles, int sym) {
  extern __shared__ double lds[];
  const int bi = blockIdx.x;
  if (bi >= nlist) return;
  const int lane = threadIdx.x;
  const DBlk B = blks[blk_list[bi]];
  const int c = B.c, d = B.d;
  const int kc = dyn.k[c], kd = dyn.k[d];
  if (!blk_scale_wave_fits<T>(kc, kd, lds_doubles)) return;
  const int nc = dyn.n[c], nd = dyn.n[d];
  const int nrc = dyn.nr[c], nrd = dyn.nr[d];
  if (kc == 0 || kd == 0) return;
  const bool spc = dyn.passes[c] > 0, spd = dyn.passes[d] > 0;
  const int32_t* permc = iarena + segs[c].ioff + segs[c].cap;
  const int32_t* permd = iarena + segs[d].ioff + segs[d].cap;
  const int32_t* pivc = permc + segs[c].cap;
  const T* A = varena + B.off;
  T* out = varena + B.soff;
  const T* Lc = varena + segs[c].lu_off;
  const T* Ud = varena + segs[d].lu_off;
  double* X = lds;                              // kc x kd
  T* Lb = reinterpret_cast<T*>(X + kc * kd);    // kc x kc (strict lower part used; diagonal too if sym)
  T* Ub = Lb + kc * kc;                         // kd x kd (upper part used)
  int* rs = reinterpret_cast<int*>(Ub + kd * kd);  // kc: block row of row i of P_s X
  int* cs = rs + kc;                               // kd: block column of column j
  // row map of the skeleton-part pivots of c (row i of P_s X is row
  // pivc[nrc + i] - nrc of X), composed with the skeleton DOF positions
  {
    const int i = lane < kc ? lane : kc - 1, j = lane < kd ? lane : kd - 1;
    const int r = pivc[nrc + i] - nrc;
    const int si = spc ? permc[r] : r, sj = spd ? permd[j] : j;
    if (lane < kc) rs[lane] = si;
    if (lane < kd) cs[lane] = sj;
  }
  // triangles of the packed inverses: every load issued (clamped rows and
  // columns), zeros stored outside the triangle
  load_batched<8>(
      kc * kc, lane, 64,
      [&](int t) {
        const int i = t / kc, u = t - i * kc;
        return Lc[size_t(nrc + i) * nc + nrc + u];
      },
      [&](int t, T v) {
        const int i = t / kc, u = t - i * kc;
        Lb[t] = u < i || (sym && u == i) ? v : T(0);
      });
  load_batched<8>(
      kd * kd, lane, 64,
      [&](int t) {
        const int u = t / kd, j = t - u * kd;
        return Ud[size_t(nrd + u) * nd + nrd + j];
      },
      [&](int t, T v) {
        const int u = t / kd, j = t - u * kd;
        Ub[t] = u <= j ? v : T(0);
      });
  wave_sync();
  load_batched<8>(
      kc * kd, lane, 64,
      [&](int t) {
        const int i = t / kd, j = t - i * kd;
        return A[size_t(rs[i]) * nd + cs[j]];
      },
      [&](int t, T v) { X[t] = double(v); });
  wave_sync();
  if (lane < kd) {
    const int j = lane;
    // Y = L^{-1} X (unit lower, or the stored diagonal in the symmetric
    // form), rows descending so X[u] (u < i) is still X
    for (int i = kc - 1; i >= 0; --i) {
      double v = sym ? double(Lb[i * kc + i]) * X[i * kd + j] : X[i * kd + j];
      for (int u = 0; u < i; ++u) v += double(Lb[i * kc + u]) * X[u * kd + j];
      X[i * kd + j] = v;
    }
  }
  wave_sync();
  // out = Y U^{-1}
  for (int t = lane; t < kc * kd; t += 64) {
    const int i = t / kd, j = t - i * kd;
    double v = 0.0;
    for (int u = 0; u <= j; ++u) v += X[i * kd + u] * double(Ub[u * kd + j]);
    out[t] = T(v);
  }
}

// Merge sizes: offsets of constituents inside each level-(l-1) segment, and
// the merged DOF list (constituent skeletons one after another).
__global__ void k_merge_sizes(const DSeg* useg, int nuseg, const int32_t* cons_ptr, const int32_t* cons,
                              const DSeg* segs, int32_t* iarena, DLevelDyn dyn, DLevelDyn udyn) {
  const int C = blockIdx.x;
  if (C >= nuseg) return;
  __shared__ int s_off;
  if (threadIdx.x == 0) s_off = 0;
  __syncthreads();
  int32_t* udofs = iarena + useg[C].ioff;
  for (int q = cons_ptr[C]; q < cons_ptr[C + 1]; ++q) {
    const int c = cons[q];
    const int k = dyn.k[c], nr = dyn.nr[c];
    const int o = s_off;
    const int32_t* dofs = iarena + segs[c].ioff;
    for (int i = threadIdx.x; i < k; i += blockDim.x) udofs[o + i] = dofs[nr + i];
    __syncthreads();
    if (threadIdx.x == 0) {
      dyn.off[c] = o;
      s_off = o + k;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    udyn.n[C] = s_off;
    udyn.k[C] = s_off;
    udyn.nr[C] = 0;
    udyn.h[C] = 0;
    udyn.passes[C] = 0;
    udyn.off[C] = 0;
    udyn.nfar[C] = 0;
  }
}

// Separator elimination fused with the merge: every level-(l-1) block is
// assembled from identity / scaled level-l blocks minus A'_{c,s} A'_{s,d}
// for the level-l separators s next to both c and d (Z_l, Z_u, E_(l)).
// With lds_bytes > 0, a task whose blocks fit keeps its kc x kd result in
// LDS and stages both factors of every term there with batched loads;
// otherwise the products read the factors from memory.
// acc (kc x kd, row-major, FP64) -= A (kc x ks) B (ks x kd), A and B
// row-major in LDS in the storage type: one separator term of the Schur
// update (A_{c,s} U_s^{-1}) (L_s^{-1} A_{s,d}) on the matrix cores, in 16 x 16
// output tiles dealt round-robin to the NW waves (a tile, and so each acc
// element, always belongs to the same wave).  FP64 storage: FP64 16x16x4
// MFMA.  FP32 storage (mixed form): FP32 16x16x4 MFMA with FP32
// accumulation inside a term.  Lane l supplies A[i0 + l%16][k0 + l/16] and
// B[k0 + l/16][j0 + l%16] (zero outside the matrices); its four results are
// column j0 + l%16 of rows i0 + l/16 + 4r (FP64) or i0 + 4(l/16) + r (FP32).
// Merge tasks whose skeletons exceed this size take the matrix-core tiles
// read from memory when they do not fit the LDS; smaller ones, with too few
// output tiles to occupy the waves, the per-thread dot products.
constexpr int MELIM_TILE_MIN = 128;

template <typename T, int NW>
__device__ inline void schur_term_mfma(double* acc, const T* A, const T* B, int kc, int ks, int kd) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ntj = (kd + 15) >> 4, nt = ((kc + 15) >> 4) * ntj;
  for (int tile = w; tile < nt; tile += NW) {
    const int i0 = (tile / ntj) * 16, j0 = (tile % ntj) * 16;
    const int ar = i0 + li, bc = j0 + li;
    const bool arow = ar < kc, bcol = bc < kd;
    if constexpr (sizeof(T) == 8) {
      typedef double v4 __attribute__((ext_vector_type(4)));
      v4 d;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + lk + 4 * r;
        d[r] = row < kc && bcol ? acc[row * kd + bc] : 0.0;
      }
      for (int k0 = 0; k0 < ks; k0 += 4) {
        const int k = k0 + lk;
        const double a = arow && k < ks ? -double(A[ar * ks + k]) : 0.0;
        const double b = bcol && k < ks ? double(B[k * kd + bc]) : 0.0;
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + lk + 4 * r;
        if (row < kc && bcol) acc[row * kd + bc] = d[r];
      }
    } else {
      typedef float v4 __attribute__((ext_vector_type(4)));
      v4 d;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + 4 * lk + r;
        d[r] = row < kc && bcol ? float(acc[row * kd + bc]) : 0.0f;
      }
      for (int k0 = 0; k0 < ks; k0 += 4) {
        const int k = k0 + lk;
        const float a = arow && k < ks ? -float(A[ar * ks + k]) : 0.0f;
        const float b = bcol && k < ks ? float(B[k * kd + bc]) : 0.0f;
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + 4 * lk + r;
        if (row < kc && bcol) acc[row * kd + bc] = double(d[r]);
      }
    }
  }
}

// WIDE = false: zero the level-(l-1) block, then every task except the wide
// ones (skeletons over MELIM_TILE_MIN that do not fit the LDS); WIDE = true,
// launched after it: the wide tasks only, on the matrix-core tiles (a kernel
// of its own, so their registers do not lower the occupancy of the others).
template <typename T, int NT, bool WIDE = false>
__global__ __launch_bounds__(NT) void k_merge_elim(const DBlk* ublks, int nublk, const int32_t* task_ptr,
                                                   const DTask* tasks, const DSepTerm* terms,
                                                   const DBlk* blks, T* varena, DLevelDyn dyn,
                                                   DLevelDyn udyn, int lds_bytes) {
  extern __shared__ double lds[];
  const int b = blockIdx.x;
  if (b >= nublk) return;
  const int tid = threadIdx.x;
  const DBlk U = ublks[b];
  const int nC = udyn.n[U.c], nD = udyn.n[U.d];
  T* out = varena + U.off;
  if (!WIDE) {
    for (int t = tid; t < nC * nD; t += NT) out[t] = T(0);
    __syncthreads();
  }
  for (int q = task_ptr[b]; q < task_ptr[b + 1]; ++q) {
    const DTask tk = tasks[q];
    const int kc = dyn.k[tk.c], kd = dyn.k[tk.d];
    const int oc = dyn.off[tk.c], od = dyn.off[tk.d];
    const T* src = tk.src >= 0 ? varena + blks[tk.src].soff : nullptr;
    int ksmax = 0;
    for (int e = tk.sep_begin; e < tk.sep_end; ++e) {
      const int ks = dyn.k[terms[e].s];
      ksmax = ks > ksmax ? ks : ksmax;
    }
    const int acc_bytes = (kc * kd * 8 + 15) & ~15;
    const bool staged = lds_bytes > 0 && tk.sep_end > tk.sep_begin &&
                        acc_bytes + (kc + kd) * ksmax * int(sizeof(T)) <= lds_bytes;
    const bool wide = !staged && (kc > MELIM_TILE_MIN || kd > MELIM_TILE_MIN);
    if (wide != WIDE) continue;
    if (staged) {
      double* acc = lds;  // kc x kd
      T* sA = reinterpret_cast<T*>(reinterpret_cast<char*>(lds) + acc_bytes);
      if (tk.src == -2 || !src)
        for (int t = tid; t < kc * kd; t += NT) acc[t] = tk.src == -2 && t / kd == t % kd ? 1.0 : 0.0;
      else
        stage_batched<8>(src, kc * kd, tid, NT, [&](int t, T v) { acc[t] = double(v); });
      for (int e = tk.sep_begin; e < tk.sep_end; ++e) {
        const DSepTerm st = terms[e];
        const int ks = dyn.k[st.s];
        T* sB = sA + kc * ks;
        __syncthreads();  // the previous term's factors are no longer read
        stage_batched<8>(varena + blks[st.blk_cs].soff, kc * ks, tid, NT, [&](int t, T v) { sA[t] = v; });
        stage_batched<8>(varena + blks[st.blk_sd].soff, ks * kd, tid, NT, [&](int t, T v) { sB[t] = v; });
        __syncthreads();
        schur_term_mfma<T, NT / 64>(acc, sA, sB, kc, ks, kd);
      }
      __syncthreads();  // acc tiles were written by their waves
      for (int t = tid; t < kc * kd; t += NT) {
        const int i = t / kd, j = t - i * kd;
        out[size_t(oc + i) * nD + od + j] = T(acc[t]);
      }
      __syncthreads();  // the next task restages
      continue;
    }
    if (!WIDE) {
      // the block and its factors exceed the LDS, but there are few output
      // tiles: one output per thread, FP64 dot products from memory
      for (int t = tid; t < kc * kd; t += NT) {
        const int i = t / kd, j = t % kd;
        double v = tk.src == -2 ? (i == j ? 1.0 : 0.0) : (src ? double(src[t]) : 0.0);
        for (int e = tk.sep_begin; e < tk.sep_end; ++e) {
          const DSepTerm st = terms[e];
          const int ks = dyn.k[st.s];
          const T* Acs = varena + blks[st.blk_cs].soff;
          const T* Asd = varena + blks[st.blk_sd].soff;
          double acc = 0.0;
          for (int u = 0; u < ks; ++u) acc += double(Acs[size_t(i) * ks + u]) * double(Asd[size_t(u) * kd + j]);
          v -= acc;
        }
        out[size_t(oc + i) * nD + od + j] = T(v);
      }
      continue;
    }
    // wide blocks (3D fronts): 16 x 64 output tiles on the matrix cores
    // (FP64), one wave per tile, the factors' entries read from memory, every
    // separator term accumulated before the tile is written
    if constexpr (WIDE) {
      const int w = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
      const int nti = (kc + 15) >> 4, ncg = (kd + 63) >> 6;
      for (int unit = w; unit < nti * ncg; unit += NT / 64) {
        const int ti = unit / ncg, cg = unit - ti * ncg, i0 = 16 * ti, j0 = 64 * cg;
        const int nct = ((kd - j0 < 64 ? kd - j0 : 64) + 15) >> 4;
        gg_v4 acc[4] = {};
        for (int e = tk.sep_begin; e < tk.sep_end; ++e) {
          const DSepTerm st = terms[e];
          const int ks = dyn.k[st.s];
          const T* Acs = varena + blks[st.blk_cs].soff;
          const T* Asd = varena + blks[st.blk_sd].soff;
          wave_tile_mfma(
              [&](int i, int u) {
                const double v = double(Acs[size_t(i < kc ? i : kc - 1) * ks + (u < ks ? u : ks - 1)]);
                return i < kc && u < ks ? v : 0.0;
              },
              [&](int u, int col) {
                const int j = j0 + col;
                return double(Asd[size_t(u < ks ? u : ks - 1) * kd + (j < kd ? j : kd - 1)]);
              },
              i0, 0, ks, nct, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + lk + 4 * r;
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            const int j = j0 + 16 * cc + li;
            if (i < kc && j < kd && cc < nct) {
              const double v0 = tk.src == -2 ? (i == j ? 1.0 : 0.0) : (src ? double(src[size_t(i) * kd + j]) : 0.0);
              out[size_t(oc + i) * nD + od + j] = T(v0 - acc[cc][r]);
            }
          }
        }
      }
    }
  }
}

}  // namespace spalu
