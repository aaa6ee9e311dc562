// Solve kernels: x = V~ W~ b (eqs. (4.12)-(4.13)) applied to nrhs columns
// at once, and the FP64 residual of iterative refinement.  The working
// vector W is DOF-major (W[v*nrhs + j]) so a segment's gather of its DOFs
// reads nrhs contiguous values per DOF.
#pragma once

#include <type_traits>
#include "device_common.hpp"
#include "kernels_factor.hpp"
#include "layout.hpp"

namespace spalu {

// Layout changes between the caller's column-major FP64 vectors (ld) and
// the DOF-major working layout W[v * nrhs + j] in the storage type, through
// an LDS tile of RHS_TV vertices x RHS_TJ columns (grid: vertex tiles x
// column tiles), so both sides are read and written with consecutive
// addresses.
constexpr int RHS_TV = 64;
constexpr int RHS_TJ = 32;

template <typename T>
__global__ __launch_bounds__(WG) void k_rhs_in(const double* B, int64_t ldb, int64_t n, int nrhs, T* W) {
  __shared__ double tile[RHS_TJ][RHS_TV + 1];
  const int64_t v0 = int64_t(blockIdx.x) * RHS_TV;
  const int j0 = blockIdx.y * RHS_TJ;
  const int nv = n - v0 < RHS_TV ? int(n - v0) : RHS_TV;
  const int nj = nrhs - j0 < RHS_TJ ? nrhs - j0 : RHS_TJ;
  for (int t = threadIdx.x; t < RHS_TV * RHS_TJ; t += WG) {
    const int j = t / RHS_TV, vl = t % RHS_TV;
    if (j < nj && vl < nv) tile[j][vl] = B[v0 + vl + (j0 + j) * ldb];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nv * nj; t += WG) {
    const int vl = t / nj, j = t - vl * nj;
    W[(v0 + vl) * nrhs + j0 + j] = T(tile[j][vl]);
  }
}

template <typename T>
__global__ __launch_bounds__(WG) void k_rhs_out(const T* W, int64_t n, int nrhs, double* X, int64_t ldx,
                                                int accumulate) {
  __shared__ double tile[RHS_TJ][RHS_TV + 1];
  const int64_t v0 = int64_t(blockIdx.x) * RHS_TV;
  const int j0 = blockIdx.y * RHS_TJ;
  const int nv = n - v0 < RHS_TV ? int(n - v0) : RHS_TV;
  const int nj = nrhs - j0 < RHS_TJ ? nrhs - j0 : RHS_TJ;
  for (int t = threadIdx.x; t < nv * nj; t += WG) {
    const int vl = t / nj, j = t - vl * nj;
    tile[j][vl] = double(W[(v0 + vl) * nrhs + j0 + j]);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < RHS_TV * RHS_TJ; t += WG) {
    const int j = t / RHS_TV, vl = t % RHS_TV;
    if (j < nj && vl < nv) {
      double* x = X + v0 + vl + (j0 + j) * ldx;
      *x = accumulate ? *x + tile[j][vl] : tile[j][vl];
    }
  }
}

// Leaf interiors: Z_I = A_II^{-1} W_I (forward) or
// W_I = A_II^{-1} (B_I - A_IB W_B) (backward), with the stored inverse
// (transposed: entry (i, q) at q * ni + i) staged in LDS (one coalesced
// load) and the right-hand sides beside it.
template <typename T, bool BACKWARD>
__global__ __launch_bounds__(WG) void k_leaf_solve(const DLeaf* leaves, int nleaf, GridGeom g,
                                                   const int64_t* rowptr, const int32_t* colind,
                                                   const double* vals, const int32_t* iarena,
                                                   const T* varena, const T* B0, T* W, T* Z, int nrhs) {
  extern __shared__ double lds[];
  const int lf = blockIdx.x;
  if (lf >= nleaf) return;
  const DLeaf L = leaves[lf];
  const int ni = L.ni, tid = threadIdx.x;
  if (ni == 0) return;
  const int w0 = L.hi[0] - L.lo[0] + 1, w1 = L.hi[1] - L.lo[1] + 1;
  const T* Ai = varena + L.lu_off;
  const bool stage = ni * ni + ni <= LDS_DOUBLES;
  double* sA = lds;
  double* X = stage ? lds + ni * ni : lds;
  const int room = stage ? LDS_DOUBLES - ni * ni : LDS_DOUBLES;
  const int jc = room / ni < nrhs ? room / ni : nrhs;
  if (stage) {
    for (int t = tid; t < ni * ni; t += WG) sA[t] = double(Ai[t]);
  }
  for (int j0 = 0; j0 < nrhs; j0 += jc) {
    const int nc = nrhs - j0 < jc ? nrhs - j0 : jc;
    for (int t = tid; t < ni * nc; t += WG) {
      const int i = t / nc, j = t % nc;
      const int ix = i % w0, iy = (i / w0) % w1, iz = i / (w0 * w1);
      const int u = (L.lo[0] + ix) + g.nx * ((L.lo[1] + iy) + g.ny * (L.lo[2] + iz));
      double v;
      if (!BACKWARD) {
        v = double(B0[size_t(u) * nrhs + j0 + j]);
      } else {
        v = double(B0[size_t(u) * nrhs + j0 + j]);
        for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
          const int w = colind[e];
          int cw[3];
          vcoords(g, w, cw);
          const bool inside = cw[0] >= L.lo[0] && cw[0] <= L.hi[0] && cw[1] >= L.lo[1] &&
                              cw[1] <= L.hi[1] && cw[2] >= L.lo[2] && cw[2] <= L.hi[2];
          if (!inside) v -= vals[e] * double(W[size_t(w) * nrhs + j0 + j]);
        }
      }
      X[t] = v;
    }
    __syncthreads();
    for (int t = tid; t < ni * nc; t += WG) {
      const int i = t / nc, j = t % nc;
      double acc = 0.0;
      if (stage) {
        for (int q = 0; q < ni; ++q) acc += sA[q * ni + i] * X[q * nc + j];
      } else {
        for (int q = 0; q < ni; ++q) acc += double(Ai[size_t(q) * ni + i]) * X[q * nc + j];
      }
      const int ix = i % w0, iy = (i / w0) % w1, iz = i / (w0 * w1);
      const int u = (L.lo[0] + ix) + g.nx * ((L.lo[1] + iy) + g.ny * (L.lo[2] + iz));
      if (BACKWARD)
        W[size_t(u) * nrhs + j0 + j] = T(acc);
      else
        Z[size_t(u) * nrhs + j0 + j] = T(acc);
    }
    __syncthreads();
  }
}

// The same for leaves of at most 64 interior vertices, one wave each: lane q
// gathers the right-hand sides of vertex q (a chunk of 16, zero beyond the
// last one) into LDS, then lane i forms row i of A_II^{-1} times the chunk,
// reading the transposed inverse (consecutive lanes, consecutive addresses)
// in batches of loads issued together.
constexpr int LEAF_SOLVE_CHUNK = 16;

// x[j] = src[j] for j < nc (0 beyond): a full chunk loads unconditionally,
// so that all its loads are in flight together.
template <typename T>
__device__ inline void load_chunk(const T* src, int nc, double x[LEAF_SOLVE_CHUNK]) {
  if (nc == LEAF_SOLVE_CHUNK) {
#pragma unroll
    for (int j = 0; j < LEAF_SOLVE_CHUNK; ++j) x[j] = double(src[j]);
  } else {
#pragma unroll
    for (int j = 0; j < LEAF_SOLVE_CHUNK; ++j) x[j] = j < nc ? double(src[j]) : 0.0;
  }
}

__host__ __device__ inline int leaf_solve_wave_lds_bytes(int ni) { return 8 * LEAF_SOLVE_CHUNK * ni; }

// One 16 x 16 output tile (rows i0.., all 16 columns of a chunk) of the
// product A X on the matrix cores, one wave: A (rows x K) with entry (i, k)
// at A[k * lda + i] (the transposed storage of the leaf matrices), X (K x 16)
// row-major in LDS, zero outside [0, rows) x [0, K).  FP64 16x16x4 MFMA for
// both storage types (the solve accumulates in FP64, as the refinement's
// last digits need).  Lane l supplies A[i0 + l%16][k0 + l/16] and
// X[k0 + l/16][l%16] (clamped addresses, zero outside) and receives column
// l % 16 of rows leaf_tile_row(i0, r).
template <typename T>
__device__ inline void leaf_tile_mfma(const T* A, int lda, int rows, int K, const double* X, int i0, double out[4]) {
  constexpr int KS = 16;  // k-steps whose operand loads are issued together (K <= 64: one batch)
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int i = i0 + li;
  const bool irow = i < rows;
  const int ic = irow ? i : rows - 1;
  typedef double v4 __attribute__((ext_vector_type(4)));
  v4 d = {0.0, 0.0, 0.0, 0.0};
  for (int kb = 0; kb < K; kb += 4 * KS) {
    T av[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = kb + 4 * s + lk;
      av[s] = A[size_t(k < K ? k : K - 1) * lda + ic];
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      if (kb + 4 * s >= K) break;
      const int k = kb + 4 * s + lk;
      const bool kin = k < K;
      const double b = X[(kin ? k : K - 1) * LEAF_SOLVE_CHUNK + li];
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(irow && kin ? double(av[s]) : 0.0, kin ? b : 0.0, d, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) out[r] = d[r];
}

// Row of result r of this lane in a tile of leaf_tile_mfma.
__device__ inline int leaf_tile_row(int i0, int r) { return i0 + ((threadIdx.x & 63) >> 4) + 4 * r; }

// Vertex of interior row i of a leaf box.
__device__ inline int leaf_vertex(const DLeaf& L, GridGeom g, int w0, int w1, int i) {
  const int ix = i % w0, iy = (i / w0) % w1, iz = i / (w0 * w1);
  return (L.lo[0] + ix) + g.nx * ((L.lo[1] + iy) + g.ny * (L.lo[2] + iz));
}

template <typename T, bool BACKWARD>
__global__ __launch_bounds__(64) void k_leaf_solve_wave(const DLeaf* leaves, int nleaf, GridGeom g,
                                                        const int64_t* rowptr, const int32_t* colind,
                                                        const double* vals, const T* varena, const T* B0,
                                                        T* W, T* Z, int nrhs) {
  extern __shared__ double lds[];
  constexpr int CH = LEAF_SOLVE_CHUNK;
  const int lf = blockIdx.x;
  if (lf >= nleaf) return;
  const DLeaf L = leaves[lf];
  const int ni = L.ni, lane = threadIdx.x;
  if (ni == 0) return;
  const int w0 = L.hi[0] - L.lo[0] + 1, w1 = L.hi[1] - L.lo[1] + 1, w2 = L.hi[2] - L.lo[2] + 1;
  double* X = lds;
  const bool act = lane < ni;
  const int ix = lane % w0, iy = (lane / w0) % w1, iz = lane / (w0 * w1);
  const int u = act ? (L.lo[0] + ix) + g.nx * ((L.lo[1] + iy) + g.ny * (L.lo[2] + iz)) : 0;
  // stencil entries of row u (at most 8, |d| <= 1 in up to three axes):
  // columns and values loaded together; outside couplings kept
  constexpr int ME = 8;
  int wo[ME];
  double ao[ME];
  if (BACKWARD) {
    const int64_t e0 = act ? rowptr[u] : 0, e1 = act ? rowptr[u + 1] : 0;
    int cols[ME];
    double vv[ME];
#pragma unroll
    for (int m = 0; m < ME; ++m) {
      const int64_t e = e0 + m < e1 ? e0 + m : (e1 > e0 ? e1 - 1 : 0);
      cols[m] = act && e1 > e0 ? colind[e] : 0;
      vv[m] = act && e1 > e0 ? vals[e] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < ME; ++m) {
      const bool out = e0 + m < e1 && box_nbr(g, w0, w1, w2, ix, iy, iz, lane, u, cols[m]) < 0;
      wo[m] = out ? cols[m] : u;
      ao[m] = out ? vv[m] : 0.0;
    }
  }
  const T* Ai = varena + L.lu_off + (act ? lane : 0);  // column lane of the transposed inverse
  T* dst = BACKWARD ? W : Z;
  for (int j0 = 0; j0 < nrhs; j0 += CH) {
    const int nc = nrhs - j0 < CH ? nrhs - j0 : CH;
    if (act) {
      double v[CH];
      load_chunk(B0 + size_t(u) * nrhs + j0, nc, v);
      if (BACKWARD) {
        for (int m = 0; m < ME; ++m) {
          if (ao[m] == 0.0) continue;
          double wv[CH];
          load_chunk(W + size_t(wo[m]) * nrhs + j0, nc, wv);
#pragma unroll
          for (int j = 0; j < CH; ++j) v[j] = fma(-ao[m], wv[j], v[j]);
        }
        for (int64_t e = rowptr[u] + ME; e < rowptr[u + 1]; ++e) {  // rows longer than ME
          const int w = colind[e];
          if (box_nbr(g, w0, w1, w2, ix, iy, iz, lane, u, w) >= 0) continue;
          double wv[CH];
          load_chunk(W + size_t(w) * nrhs + j0, nc, wv);
#pragma unroll
          for (int j = 0; j < CH; ++j) v[j] = fma(-vals[e], wv[j], v[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) X[lane * CH + j] = v[j];
    }
    wave_sync();
    if (!BACKWARD) {
      // Z = A_II^{-1} X on the matrix cores, 16 rows at a time
      const int jj = lane & 15;
      for (int i0 = 0; i0 < ni; i0 += 16) {
        double o[4];
        leaf_tile_mfma<T>(varena + L.lu_off, ni, ni, ni, X, i0, o);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = leaf_tile_row(i0, r);
          if (row < ni && jj < nc) dst[size_t(leaf_vertex(L, g, w0, w1, row)) * nrhs + j0 + jj] = T(o[r]);
        }
      }
    } else if (act) {
      double acc[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) acc[j] = 0.0;
      // row lane of A_II^{-1} in batches of 16 loads issued together
      for (int q0 = 0; q0 < ni; q0 += 16) {
        T av[16];
#pragma unroll
        for (int b = 0; b < 16; ++b) av[b] = Ai[size_t(q0 + b < ni ? q0 + b : ni - 1) * ni];
#pragma unroll
        for (int b = 0; b < 16; ++b)
          if (q0 + b < ni) {
            const double a = double(av[b]);
            const double* xq = X + (q0 + b) * CH;
#pragma unroll
            for (int j = 0; j < CH; ++j) acc[j] = fma(a, xq[j], acc[j]);
          }
      }
      T* out = dst + size_t(u) * nrhs + j0;
#pragma unroll
      for (int j = 0; j < CH; ++j)
        if (j < nc) out[j] = T(acc[j]);
    }
    wave_sync();
  }
}

// W_u = B_u - sum over leaf-interior neighbours i of a_ui Z_i, for every
// separator vertex u (the list sepv); leaf interiors of W are written only by
// the backward leaf solve.
template <typename T>
__global__ void k_sep_from_leaves(int64_t nsep, const int32_t* sepv, const int8_t* seplev,
                                  const int64_t* rowptr, const int32_t* colind, const double* vals,
                                  const T* B0, const T* Z, T* W, int nrhs) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nsep * nrhs) return;
  const int u = sepv[t / nrhs];
  const int j = int(t % nrhs);
  double acc = 0.0;
  for (int64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
    const int w = colind[e];
    if (seplev[w] == 0) acc += vals[e] * double(Z[size_t(w) * nrhs + j]);
  }
  const size_t idx = size_t(u) * nrhs + j;
  W[idx] = T(double(B0[idx]) - acc);
}

// Per segment of level l: forward (U_T, then P and L^{-1}) or backward
// (U^{-1}, then L_T) on its DOFs in [remainder; skeleton] order, with the
// packed inverses of the two-stage LU (and T) staged in LDS, in the storage
// type, when they fit SEG_SOLVE_LDS_BYTES beside two right-hand-side columns.
constexpr int SEG_SOLVE_LDS_BYTES = 65536;

// In the symmetric form (sym) the forward row operator takes the stored
// diagonal in place of the unit one (the balanced R = Delta^{-1} L^{-1} of
// the segment factorization; the interchanges are the identity).
template <typename T, bool BACKWARD>
__global__ __launch_bounds__(WG) void k_seg_solve(const DSeg* segs, int nseg, const int32_t* iarena,
                                                  const T* varena, DLevelDyn dyn, T* W, int nrhs, int sym) {
  extern __shared__ double lds[];
  const int c = blockIdx.x;
  if (c >= nseg) return;
  const int tid = threadIdx.x;
  const DSeg S = segs[c];
  const int n = dyn.n[c];
  if (n == 0) return;
  const int k = dyn.k[c], nr = dyn.nr[c];
  const bool sp = dyn.passes[c] > 0 && nr > 0 && k > 0;
  const int32_t* dofs = iarena + S.ioff;
  const int32_t* piv = dofs + 2 * S.cap;
  const T* Inv = varena + S.lu_off;
  const T* Tm = varena + S.t_off;
  const int nt = sp ? k * nr : 0;
  const int sbytes = ((n * n + nt) * int(sizeof(T)) + 15) & ~15;  // staged inverse and T
  const bool stage = sbytes + 2 * n * 8 <= SEG_SOLVE_LDS_BYTES;
  if (!stage && 2 * n * 8 > SEG_SOLVE_LDS_BYTES) {
    // too large for the staging buffer: poison the result so the residual
    // check reports the failure instead of returning a wrong solution
    for (int t = tid; t < n * nrhs; t += WG) W[size_t(dofs[t / nrhs]) * nrhs + t % nrhs] = T(NAN);
    return;
  }
  T* sI = reinterpret_cast<T*>(lds);  // packed inverse (staged)
  T* sT = sI + n * n;                 // T (staged)
  double* X = stage ? reinterpret_cast<double*>(reinterpret_cast<char*>(lds) + sbytes) : lds;
  const int room = (SEG_SOLVE_LDS_BYTES - (stage ? sbytes : 0)) / 8;
  const int jc = room / (2 * n) < nrhs ? room / (2 * n) : nrhs;
  if (stage) {
    stage_batched<8>(Inv, n * n, tid, WG, [&](int t, T v) { sI[t] = v; });
    if (nt > 0) stage_batched<8>(Tm, nt, tid, WG, [&](int t, T v) { sT[t] = v; });
  }
  for (int j0 = 0; j0 < nrhs; j0 += jc) {
    const int nc = nrhs - j0 < jc ? nrhs - j0 : jc;
    double* Yb = X + size_t(n) * nc;
    for (int t = tid; t < n * nc; t += WG) {
      const int i = t / nc, j = t % nc;
      X[t] = double(W[size_t(dofs[i]) * nrhs + j0 + j]);
    }
    __syncthreads();
    if (!BACKWARD) {
      if (sp) {
        for (int t = tid; t < nr * nc; t += WG) {
          const int q = t / nc, j = t % nc;
          double s = 0.0;
          if (stage)
            for (int i = 0; i < k; ++i) s += sT[i * nr + q] * X[size_t(nr + i) * nc + j];
          else
            for (int i = 0; i < k; ++i) s += double(Tm[size_t(i) * nr + q]) * X[size_t(nr + i) * nc + j];
          X[t] -= s;
        }
        __syncthreads();
      }
      // P: row i of P X is row piv[i] of X
      for (int t = tid; t < n * nc; t += WG) Yb[t] = X[size_t(piv[t / nc]) * nc + t % nc];
      __syncthreads();
      for (int t = tid; t < n * nc; t += WG) X[t] = Yb[t];
      __syncthreads();
      for (int t = tid; t < n * nc; t += WG) {
        const int i = t / nc, j = t % nc;
        double v = X[t];
        if (stage) {
          const T* row = sI + i * n;
          if (sym) v *= double(row[i]);
          for (int u = 0; u < i; ++u) v += row[u] * X[size_t(u) * nc + j];
        } else {
          const T* row = Inv + size_t(i) * n;
          if (sym) v *= double(row[i]);
          for (int u = 0; u < i; ++u) v += double(row[u]) * X[size_t(u) * nc + j];
        }
        W[size_t(dofs[i]) * nrhs + j0 + j] = T(v);
      }
    } else {
      for (int t = tid; t < n * nc; t += WG) {
        const int i = t / nc, j = t % nc;
        double v = 0.0;
        if (stage) {
          const T* row = sI + i * n;
          for (int u = i; u < n; ++u) v += row[u] * X[size_t(u) * nc + j];
        } else {
          const T* row = Inv + size_t(i) * n;
          for (int u = i; u < n; ++u) v += double(row[u]) * X[size_t(u) * nc + j];
        }
        Yb[t] = v;
      }
      __syncthreads();
      if (sp) {
        for (int t = tid; t < k * nc; t += WG) {
          const int i = t / nc, j = t % nc;
          double s = 0.0;
          if (stage)
            for (int q = 0; q < nr; ++q) s += sT[i * nr + q] * Yb[size_t(q) * nc + j];
          else
            for (int q = 0; q < nr; ++q) s += double(Tm[size_t(i) * nr + q]) * Yb[size_t(q) * nc + j];
          Yb[size_t(nr + i) * nc + j] -= s;
        }
        __syncthreads();
      }
      for (int t = tid; t < n * nc; t += WG) {
        const int i = t / nc, j = t % nc;
        W[size_t(dofs[i]) * nrhs + j0 + j] = T(Yb[t]);
      }
    }
    __syncthreads();
  }
}

// Backward leaf solve from the forward result: x_I = y_I - X x_B with
// X = A_II^{-1} A_IB (stored transposed by the one-wave leaf factor) and x_B
// the boundary values; one wave per leaf of at most 64 interior vertices.
// The boundary values of a chunk of right-hand sides are staged in LDS and
// X x_B is formed on the matrix cores, 16 rows at a time.
__host__ __device__ inline int leaf_bwd_x_lds_bytes(int nb) { return 8 * LEAF_SOLVE_CHUNK * (nb > 0 ? nb : 1); }

template <typename T>
__global__ __launch_bounds__(64) void k_leaf_solve_bwd_x(const DLeaf* leaves, int nleaf, GridGeom g,
                                                         const int32_t* iarena, const T* varena, T* W,
                                                         const T* Z, int nrhs) {
  extern __shared__ double lds[];
  constexpr int CH = LEAF_SOLVE_CHUNK;
  const int lf = blockIdx.x;
  if (lf >= nleaf) return;
  const DLeaf L = leaves[lf];
  const int ni = L.ni, nb = L.nb, lane = threadIdx.x;
  if (ni == 0) return;
  const int w0 = L.hi[0] - L.lo[0] + 1, w1 = L.hi[1] - L.lo[1] + 1;
  const int32_t* bverts = iarena + L.ioff;
  double* XB = lds;  // nb x CH boundary values
  for (int j0 = 0; j0 < nrhs; j0 += CH) {
    const int nc = nrhs - j0 < CH ? nrhs - j0 : CH;
    for (int b = lane; b < nb; b += 64) {
      double xb[CH];
      load_chunk(W + size_t(bverts[b]) * nrhs + j0, nc, xb);
#pragma unroll
      for (int j = 0; j < CH; ++j) XB[b * CH + j] = xb[j];
    }
    wave_sync();
    // x_I = y_I - X x_B on the matrix cores, 16 rows at a time
    const int jj = lane & 15;
    for (int i0 = 0; i0 < ni; i0 += 16) {
      double o[4];
      leaf_tile_mfma<T>(varena + L.x_off, ni, ni, nb, XB, i0, o);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = leaf_tile_row(i0, r);
        if (row < ni && jj < nc) {
          const size_t at = size_t(leaf_vertex(L, g, w0, w1, row)) * nrhs + j0 + jj;
          W[at] = T(double(Z[at]) - o[r]);
        }
      }
    }
    wave_sync();
  }
}

// acc[c] += A[i0 + rows, 0:K] W[idx[0:K], j0 + 16c + cols] on the matrix
// cores (FP64 16x16x4 for both storage types): wave w of the block owns
// output rows 16w..16w+15 of the pass of ib <= GG_ROWS rows, and acc[c]
// holds, in lane l, column 16c + l%16 of rows 16w + l/16 + 4r (r < 4), as
// gg_row/gg_col give.  A is row-major with leading dimension lda.  Tiles of
// GG_TILE columns of A and GG_TILE gathered rows of W go through LDS, zero
// padded to full tiles; the next tile's loads are issued before the current
// tile's products, so their latency hides behind the matrix cores.
constexpr int GG_TILE = 32;
constexpr int GG_ROWS = 64;                // 4 waves x 16 rows
constexpr int GG_COLS = 64;                // 4 column tiles of 16
constexpr int GG_LDA = GG_TILE + 2;        // A tile row stride: a half-wave's reads hit distinct banks
constexpr int GG_LDX = GG_COLS + 16;       // W tile row stride: rows k and k+1 on opposite bank halves
constexpr int GG_LDS_DOUBLES = GG_ROWS * GG_LDA + GG_TILE * GG_LDX;

__device__ inline int gg_row(int r) { return ((threadIdx.x >> 6) << 4) + ((threadIdx.x & 63) >> 4) + 4 * r; }
__device__ inline int gg_col(int c) { return 16 * c + (threadIdx.x & 15); }

template <typename T>
__device__ inline void gathered_gemm_acc(const T* A, int lda, int i0, int ib, int K, const int32_t* idx,
                                         const T* W, int nrhs, int j0, int nc, double* sA, double* sX,
                                         gg_v4 acc[4]) {
  if (K <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  // staging: A rows ar + 8m at column ac, W rows xr + 4m at column xc (m < 8)
  const int ac = tid & 31, ar = tid >> 5, xc = tid & 63, xr = tid >> 6;
  T ra[8], rx[8];
  auto fetch = [&](int u0) {
    const int kt = K - u0 < GG_TILE ? K - u0 : GG_TILE;
    const int u = u0 + (ac < kt ? ac : kt - 1);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int i = ar + 8 * m;
      ra[m] = A[size_t(i0 + (i < ib ? i : ib - 1)) * lda + u];
    }
    const int j = j0 + (xc < nc ? xc : nc - 1);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int r = xr + 4 * m;
      rx[m] = W[size_t(idx[u0 + (r < kt ? r : kt - 1)]) * nrhs + j];
    }
  };
  fetch(0);
  for (int u0 = 0; u0 < K; u0 += GG_TILE) {
    const int kt = K - u0 < GG_TILE ? K - u0 : GG_TILE;
    __syncthreads();  // the previous tile is consumed
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int i = ar + 8 * m, r = xr + 4 * m;
      sA[i * GG_LDA + ac] = i < ib && ac < kt ? double(ra[m]) : 0.0;
      sX[r * GG_LDX + xc] = r < kt && xc < nc ? double(rx[m]) : 0.0;
    }
    __syncthreads();
    if (u0 + GG_TILE < K) fetch(u0 + GG_TILE);
    if (16 * w < ib) {
      const double* pa = sA + (16 * w + li) * GG_LDA + lk;
      const double* px = sX + lk * GG_LDX + li;
      for (int k0 = 0; k0 < kt; k0 += 4) {
        const double a = pa[k0];
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (16 * c < nc) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, px[k0 * GG_LDX + 16 * c], acc[c], 0, 0, 0);
      }
    }
  }
}

// Forward separator elimination (Z_l): owner = non-separator segment a,
// W[skel_a] -= sum over level-l separators s next to a of A'_{a,s} W[skel_s].
// Block (a, y) takes skeleton rows 64y .. 64y+63 of segment a.
template <typename T>
__global__ __launch_bounds__(WG) void k_sep_fwd(const DSeg* segs, int nseg, const DNbr* nbrs,
                                                const DBlk* blks, const int32_t* iarena, const T* varena,
                                                DLevelDyn dyn, T* W, int nrhs) {
  __shared__ double sA[GG_ROWS * GG_LDA];
  __shared__ double sX[GG_TILE * GG_LDX];
  const int a = blockIdx.x;
  if (a >= nseg) return;
  const DSeg S = segs[a];
  if (S.flags & SEG_IS_SEP) return;
  const int ka = dyn.k[a], nra = dyn.nr[a];
  const int i0 = int(blockIdx.y) * GG_ROWS;
  if (i0 >= ka) return;
  bool any = false;
  for (int e = S.nbr_begin; e < S.nbr_end; ++e) any |= nbrs[e].d_is_sep != 0;
  if (!any) return;
  const int32_t* da = iarena + S.ioff + nra;
  const int ib = ka - i0 < GG_ROWS ? ka - i0 : GG_ROWS;
  for (int j0 = 0; j0 < nrhs; j0 += GG_COLS) {
    const int nc = nrhs - j0 < GG_COLS ? nrhs - j0 : GG_COLS;
    gg_v4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = gg_v4{0.0, 0.0, 0.0, 0.0};
    for (int e = S.nbr_begin; e < S.nbr_end; ++e) {
      const DNbr nb = nbrs[e];
      if (!nb.d_is_sep) continue;
      const int ks = dyn.k[nb.d], nrs = dyn.nr[nb.d];
      gathered_gemm_acc(varena + blks[nb.blk_cd].soff, ks, i0, ib, ks, iarena + segs[nb.d].ioff + nrs, W,
                        nrhs, j0, nc, sA, sX, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = gg_row(r);
      if (i >= ib) continue;
      const size_t base = size_t(da[i0 + i]) * nrhs + j0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int j = gg_col(c);
        if (j < nc) W[base + j] = T(double(W[base + j]) - acc[c][r]);
      }
    }
  }
}

// Backward separator elimination (Z_u): owner = separator s,
// W[skel_s] -= sum over its neighbours b of A'_{s,b} W[skel_b].
// Block (s, y) takes skeleton rows 64y .. 64y+63 of separator s.
template <typename T>
__global__ __launch_bounds__(WG) void k_sep_bwd(const DSeg* segs, int nseg, const DNbr* nbrs,
                                                const DBlk* blks, const int32_t* iarena, const T* varena,
                                                DLevelDyn dyn, T* W, int nrhs) {
  __shared__ double sA[GG_ROWS * GG_LDA];
  __shared__ double sX[GG_TILE * GG_LDX];
  const int s = blockIdx.x;
  if (s >= nseg) return;
  const DSeg S = segs[s];
  if (!(S.flags & SEG_IS_SEP)) return;
  const int ks = dyn.k[s], nrs = dyn.nr[s];
  const int i0 = int(blockIdx.y) * GG_ROWS;
  if (i0 >= ks) return;
  const int32_t* ds = iarena + S.ioff + nrs;
  const int ib = ks - i0 < GG_ROWS ? ks - i0 : GG_ROWS;
  for (int j0 = 0; j0 < nrhs; j0 += GG_COLS) {
    const int nc = nrhs - j0 < GG_COLS ? nrhs - j0 : GG_COLS;
    gg_v4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = gg_v4{0.0, 0.0, 0.0, 0.0};
    for (int e = S.nbr_begin; e < S.nbr_end; ++e) {
      const DNbr nb = nbrs[e];
      const int kb = dyn.k[nb.d], nrb = dyn.nr[nb.d];
      gathered_gemm_acc(varena + blks[nb.blk_cd].soff, kb, i0, ib, kb, iarena + segs[nb.d].ioff + nrb, W,
                        nrhs, j0, nc, sA, sX, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = gg_row(r);
      if (i >= ib) continue;
      const size_t base = size_t(ds[i0 + i]) * nrhs + j0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int j = gg_col(c);
        if (j < nc) W[base + j] = T(double(W[base + j]) - acc[c][r]);
      }
    }
  }
}

constexpr int SW_LD = GG_LDX;  // FP64 LDS row of 64 right-hand sides

// NW waves per segment of at most 16 * NW * TPW DOFs: forward (U_T, then P
// and L^{-1}) or backward (U^{-1}, then L_T) on its DOFs in [remainder;
// skeleton] order.  The segment's rows of 64 right-hand sides are staged in
// LDS in FP64; every product runs on the matrix cores in 16 x 64 output
// tiles (tile t on wave t % NW), its operator entries (T, the packed
// inverses) read from global memory.  One wave (NW = 1) serves the fine
// levels' many small segments, four waves the coarse levels' larger ones.
// In the symmetric form (sym) the forward operator's diagonal is the stored
// one, as in k_seg_solve.
__host__ __device__ inline int seg_solve_mfma_lds_bytes(int rows) { return 8 * rows * SW_LD; }
constexpr int SEG_MFMA_BLOCK_N = 128;  // largest segment of the four-wave shape (4 waves x 2 tiles)

template <typename T, bool BACKWARD, int NW, int TPW>
__global__ __launch_bounds__(64 * NW) void k_seg_solve_mfma(const DSeg* segs, int nseg, const int32_t* iarena,
                                                            const T* varena, DLevelDyn dyn, T* W, int nrhs,
                                                            int sym) {
  extern __shared__ double lds[];
  constexpr int NMAX = 16 * NW * TPW;
  const int c = blockIdx.x;
  if (c >= nseg) return;
  const int n = dyn.n[c];
  if (n == 0 || n > NMAX) return;  // (never on a level launched with this shape)
  const DSeg S = segs[c];
  const int k = dyn.k[c], nr = dyn.nr[c];
  const bool sp = dyn.passes[c] > 0 && nr > 0 && k > 0;
  const int32_t* dofs = iarena + S.ioff;
  const int32_t* piv = dofs + 2 * S.cap;
  const T* Inv = varena + S.lu_off;
  const T* Tm = varena + S.t_off;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  auto sync = [] {
    if constexpr (NW == 1)
      wave_sync();
    else
      __syncthreads();
  };
  // a row's DOF and permutation source: from lanes of the wave when the
  // segment fits one wave's lanes, else from memory
  const int mdof = lane < n ? dofs[lane] : 0;
  const int mpiv = lane < n ? piv[lane] : 0;
  auto dof_of = [&](int i) { return NMAX <= 64 ? __shfl(mdof, i) : dofs[i]; };
  auto piv_of = [&](int i) { return NMAX <= 64 ? __shfl(mpiv, i) : piv[i]; };
  double* X = lds;
  auto xrow = [&](int u, int col) { return X[(u < n ? u : n - 1) * SW_LD + col]; };
  const int ntile = (n + 15) >> 4;
  for (int j0 = 0; j0 < nrhs; j0 += 64) {
    const int nc = nrhs - j0 < 64 ? nrhs - j0 : 64;
    const int nct = (nc + 15) >> 4;
    const int col = lane < nc ? lane : nc - 1;
    // rows i = w + NW * b of the segment, 16 loads in flight per lane
    for (int i0 = w; i0 < n; i0 += 16 * NW) {
      T v[16];
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const int i = i0 + NW * b < n ? i0 + NW * b : n - 1;
        v[b] = W[size_t(dof_of(i)) * nrhs + j0 + col];
      }
#pragma unroll
      for (int b = 0; b < 16; ++b)
        if (i0 + NW * b < n) X[(i0 + NW * b) * SW_LD + lane] = lane < nc ? double(v[b]) : 0.0;
    }
    sync();
    if (!BACKWARD) {
      if (sp) {
        // remainder rows: x_q -= sum_i T_iq x_{nr+i} (reads skeleton rows only)
        for (int t = w; 16 * t < nr; t += NW) {
          gg_v4 acc[4] = {};
          wave_tile_mfma(
              [&](int q, int i) {
                const double tv = double(Tm[size_t(i < k ? i : k - 1) * nr + (q < nr ? q : nr - 1)]);
                return q < nr && i < k ? tv : 0.0;
              },
              [&](int i, int cc) { return xrow(nr + i, cc); }, 16 * t, 0, k, nct, acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int q = 16 * t + lk + 4 * r;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc)
              if (q < nr && cc < nct) X[q * SW_LD + 16 * cc + li] -= acc[cc][r];
          }
        }
        sync();
      }
      // P, then the unit lower L^{-1}: y_i = x_piv[i] + sum_{u<i} (L^{-1})_iu x_piv[u]
      for (int t = w; t < ntile; t += NW) {
        const int i0 = 16 * t;
        gg_v4 acc[4] = {};
        wave_tile_mfma(
            [&](int i, int u) {
              const double l = double(Inv[size_t(i < n ? i : n - 1) * n + (u < n ? u : n - 1)]);
              return i < n && u < i ? l : (i < n && u == i ? (sym ? l : 1.0) : 0.0);
            },
            [&](int u, int cc) { return X[piv_of(u < n ? u : n - 1) * SW_LD + cc]; }, i0, 0,
            i0 + 16 < n ? i0 + 16 : n, nct, acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + lk + 4 * r;
          const size_t base = size_t(dof_of(i < n ? i : n - 1)) * nrhs + j0;
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            const int j = 16 * cc + li;
            if (i < n && j < nc) W[base + j] = T(acc[cc][r]);
          }
        }
      }
    } else {
      // y = U^{-1} x: tile t reads rows u >= 16 t only
      if constexpr (NW == 1) {
        // one wave, top tile first: each result replaces rows no later tile reads
        for (int t = 0; t < ntile; ++t) {
          const int i0 = 16 * t;
          gg_v4 acc[4] = {};
          wave_tile_mfma(
              [&](int i, int u) {
                const double v = double(Inv[size_t(i < n ? i : n - 1) * n + (u < n ? u : n - 1)]);
                return i < n && u >= i && u < n ? v : 0.0;
              },
              xrow, i0, i0, n, nct, acc);
          wave_sync();
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = i0 + lk + 4 * r;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc)
              if (i < n && cc < nct) X[i * SW_LD + 16 * cc + li] = acc[cc][r];
          }
          wave_sync();
        }
      } else {
        // several waves: every tile of the block first, then the results
        gg_v4 acc[TPW][4] = {};
#pragma unroll
        for (int p = 0; p < TPW; ++p) {
          const int i0 = 16 * (w + NW * p);
          if (i0 < n)
            wave_tile_mfma(
                [&](int i, int u) {
                  const double v = double(Inv[size_t(i < n ? i : n - 1) * n + (u < n ? u : n - 1)]);
                  return i < n && u >= i && u < n ? v : 0.0;
                },
                xrow, i0, i0, n, nct, acc[p]);
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < TPW; ++p)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * (w + NW * p) + lk + 4 * r;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc)
              if (i < n && cc < nct) X[i * SW_LD + 16 * cc + li] = acc[p][cc][r];
          }
        __syncthreads();
      }
      if (sp) {
        // skeleton rows: y_{nr+i} -= sum_q T_iq y_q (reads remainder rows only)
        for (int t = w; 16 * t < k; t += NW) {
          const int i0 = 16 * t;
          gg_v4 acc[4] = {};
          wave_tile_mfma(
              [&](int i, int q) {
                const double tv = double(Tm[size_t(i < k ? i : k - 1) * nr + (q < nr ? q : nr - 1)]);
                return i < k && q < nr ? tv : 0.0;
              },
              xrow, i0, 0, nr, nct, acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = i0 + lk + 4 * r;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc)
              if (i < k && cc < nct) X[(nr + i) * SW_LD + 16 * cc + li] -= acc[cc][r];
          }
        }
        sync();
      }
      for (int i = w; i < n; i += NW) {
        const size_t d = size_t(dof_of(i));
        if (lane < nc) W[d * nrhs + j0 + lane] = T(X[i * SW_LD + lane]);
      }
    }
    sync();
  }
}

// One wave per owner segment with at most 64 neighbours, for levels whose
// skeletons hold at most 64 DOFs; block (a, y) forms skeleton rows
// 16 RT y .. 16 RT (y+1) - 1 of owner a: forward (owner = non-separator a,
// neighbours = the level's separators s): W[skel_a] -= A'_{a,s} W[skel_s];
// backward (owner = separator s, all its neighbours b):
// W[skel_s] -= A'_{s,b} W[skel_b].  A table of the stacked neighbour rows
// (K <= rows_cap: DOF, offset of the column in the neighbour's scaled block,
// that block's row length) is built in LDS first; then each k-step of the
// matrix-core product loads its operator entries and right-hand-side rows
// straight from global memory, SEP_KS k-steps at a time.
constexpr int SEP_KS = 4;  // k-steps whose loads are issued together

__host__ __device__ inline int sep_mfma_lds_bytes(int rows_cap) { return 16 * (rows_cap > 0 ? rows_cap : 1); }

template <typename T, bool FWD, int RT>
__global__ __launch_bounds__(64) void k_sep_mfma(const DSeg* segs, int nseg, const DNbr* nbrs, const DBlk* blks,
                                                 const int32_t* iarena, const T* varena, DLevelDyn dyn, T* W,
                                                 int nrhs, int rows_cap) {
  extern __shared__ double lds[];
  __shared__ int m_off[64], m_kb[64];
  __shared__ int64_t m_dofo[64], m_soff[64];
  int64_t* t_ao = reinterpret_cast<int64_t*>(lds);
  int* t_dof = reinterpret_cast<int*>(t_ao + rows_cap);
  int* t_ld = t_dof + rows_cap;
  const int a = blockIdx.x;
  if (a >= nseg) return;
  const DSeg S = segs[a];
  if (FWD == ((S.flags & SEG_IS_SEP) != 0)) return;  // not an owner on this pass
  const int ka = dyn.k[a], nra = dyn.nr[a];
  const int r0 = int(blockIdx.y) * 16 * RT;
  const int ne = S.nbr_end - S.nbr_begin;
  if (r0 >= ka || ne > 64) return;  // (more neighbours never on a level launched with this kernel)
  const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
  int kb = 0;
  int64_t dofo = 0, soff = 0;
  if (lane < ne) {
    const DNbr nb = nbrs[S.nbr_begin + lane];
    if (!FWD || nb.d_is_sep) {
      kb = dyn.k[nb.d];
      dofo = segs[nb.d].ioff + dyn.nr[nb.d];
      soff = blks[nb.blk_cd].soff;
    }
  }
  // inclusive prefix of the neighbours' row counts
  int off = kb;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(off, o);
    if (lane >= o) off += v;
  }
  const int K = __shfl(off, 63);
  if (K == 0 || K > rows_cap) return;  // (K > rows_cap never: the level's bound)
  m_off[lane] = off - kb;
  m_kb[lane] = kb;
  m_dofo[lane] = dofo;
  m_soff[lane] = soff;
  wave_sync();
  // stacked row t belongs to the last neighbour with rows starting at or
  // before t; four rows per lane per pass, their loads issued together
  for (int t0 = 0; t0 < K; t0 += 256) {
    int e4[4], d4[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int t = t0 + lane + 64 * h < K ? t0 + lane + 64 * h : K - 1;
      int e = 0;
      for (int f = 0; f < ne; ++f)
        if (m_kb[f] > 0 && m_off[f] <= t) e = f;
      e4[h] = e;
      d4[h] = iarena[m_dofo[e] + (t - m_off[e])];
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int t = t0 + lane + 64 * h;
      if (t < K) {
        t_dof[t] = d4[h];
        t_ao[t] = m_soff[e4[h]] + (t - m_off[e4[h]]);
        t_ld[t] = m_kb[e4[h]];
      }
    }
  }
  wave_sync();
  const int32_t* da = iarena + S.ioff + nra;
  for (int j0 = 0; j0 < nrhs; j0 += 64) {
    const int nc = nrhs - j0 < 64 ? nrhs - j0 : 64;
    const int nct = (nc + 15) >> 4;
    gg_v4 acc[RT][4] = {};
    // full chunks read columns j0 + 16c + l%16 at constant offsets; a last,
    // partial chunk clamps them to its nc columns
    auto tiles = [&](auto full) {
      for (int u0 = 0; u0 < K; u0 += 4 * SEP_KS) {
        int dof[SEP_KS], ld[SEP_KS];
        int64_t ao[SEP_KS];
#pragma unroll
        for (int s = 0; s < SEP_KS; ++s) {
          const int t = u0 + 4 * s + lk < K ? u0 + 4 * s + lk : K - 1;
          dof[s] = t_dof[t];
          ao[s] = t_ao[t];
          ld[s] = t_ld[t];
        }
        T bv[SEP_KS][4], av[RT][SEP_KS];
#pragma unroll
        for (int s = 0; s < SEP_KS; ++s) {
          const T* wr = W + size_t(dof[s]) * nrhs + j0;
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            const int j = 16 * cc + li;
            bv[s][cc] = decltype(full)::value ? wr[j] : wr[j < nc ? j : nc - 1];
          }
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int s = 0; s < SEP_KS; ++s) {
            const int i = r0 + 16 * rt + li;
            av[rt][s] = varena[ao[s] + int64_t(i < ka ? i : ka - 1) * ld[s]];
          }
#pragma unroll
        for (int s = 0; s < SEP_KS; ++s) {
          if (u0 + 4 * s >= K) break;
          const bool in = u0 + 4 * s + lk < K;
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            if (r0 + 16 * rt >= ka) break;
            const double av_ = in && r0 + 16 * rt + li < ka ? double(av[rt][s]) : 0.0;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc)
              if (cc < nct)
                acc[rt][cc] = __builtin_amdgcn_mfma_f64_16x16x4f64(av_, double(bv[s][cc]), acc[rt][cc], 0, 0, 0);
          }
        }
      }
    };
    if (nc == 64)
      tiles(std::true_type{});
    else
      tiles(std::false_type{});
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + 16 * rt + lk + 4 * r;
        if (i >= ka) continue;
        const size_t base = size_t(da[i]) * nrhs + j0;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int j = 16 * cc + li;
          if (j < nc) W[base + j] = T(double(W[base + j]) - acc[rt][cc][r]);
        }
      }
  }
}

// Sum over the 64 lanes of a wave by DPP lane moves (no LDS traffic):
// pairs, quads, half rows and rows, then row 0 into row 1 and rows 0-1 into
// rows 2-3, so that lane 63 ends with the total, which is broadcast.
union DppF64 {
  double d;
  int i[2];
};
template <int CTRL, int ROWS>
__device__ inline double dpp_move_f64(double x) {
  DppF64 u, o;
  u.d = x;
  o.i[0] = __builtin_amdgcn_update_dpp(0, u.i[0], CTRL, ROWS, 0xF, false);
  o.i[1] = __builtin_amdgcn_update_dpp(0, u.i[1], CTRL, ROWS, 0xF, false);
  return o.d;
}
__device__ inline double wave_sum_dpp(double v) {
  v += dpp_move_f64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move_f64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move_f64<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_move_f64<0x140, 0xF>(v);  // row_mirror
  v += dpp_move_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  DppF64 u, o;
  u.d = v;
  o.i[0] = __builtin_amdgcn_readlane(u.i[0], 63);
  o.i[1] = __builtin_amdgcn_readlane(u.i[1], 63);
  return o.d;
}

// r = b - A x in FP64 and per-wave partial sums of ||r_j||^2 and ||b_j||^2
// (part[j * nparts + wave], nparts = 4 per block) for a deterministic
// reduction: one thread per row, its stencil entries (at most 8 held in
// registers) read once, then every right-hand side in turn, the next
// column's loads issued before this column's sums; entries past a row's
// length are not loaded.  r goes to R (FP64, column-major, ld n), or, with
// TO_RHS, straight into the solve's right-hand side (row-major, storage
// type T) through an LDS transpose of 128-byte row pieces.
template <typename T, bool TO_RHS>
__global__ __launch_bounds__(WG) void k_residual(int64_t n, int nrhs, const int64_t* rowptr,
                                                 const int32_t* colind, const double* vals,
                                                 const double* B, int64_t ldb, const double* X,
                                                 int64_t ldx, double* R, T* Rw, double* part_r, double* part_b,
                                                 int nparts) {
  constexpr int ME = 8;
  constexpr int JT = 128 / int(sizeof(T));  // columns per transposed piece
  const int64_t v = int64_t(blockIdx.x) * WG + threadIdx.x;
  const int lane = threadIdx.x & 63, pidx = blockIdx.x * NWAVE + (threadIdx.x >> 6);
  const bool live = v < n;
  const int64_t vr = live ? v : n - 1;
  const int64_t e0 = rowptr[vr], e1 = rowptr[vr + 1];
  const int cnt = e1 - e0 < ME ? int(e1 - e0) : ME;
  int cols[ME];
  double vv[ME];
#pragma unroll
  for (int m = 0; m < ME; ++m) {
    const bool in = m < cnt;
    cols[m] = in ? colind[e0 + m] : int(vr);
    vv[m] = in ? vals[e0 + m] : 0.0;
  }
  double xn[ME], bn;
  auto fetch = [&](int j) {
    const double* x = X + j * ldx;
    bn = B[vr + j * ldb];
#pragma unroll
    for (int m = 0; m < ME; ++m)
      if (m < cnt) xn[m] = x[cols[m]];
  };
  fetch(0);
  for (int j = 0; j < nrhs; ++j) {
    double xc[ME];
#pragma unroll
    for (int m = 0; m < ME; ++m) xc[m] = xn[m];
    const double b = bn;
    if (j + 1 < nrhs) fetch(j + 1);
    double ax = 0.0;
#pragma unroll
    for (int m = 0; m < ME; ++m)
      if (m < cnt) ax += vv[m] * xc[m];
    if (e1 - e0 > ME) {  // rows longer than ME
      const double* x = X + j * ldx;
      for (int64_t e = e0 + ME; e < e1; ++e) ax += vals[e] * x[colind[e]];
    }
    const double r = b - ax;
    if constexpr (TO_RHS) {
      __shared__ T tile[WG][JT + 1];
      const int jj = j % JT;
      tile[threadIdx.x][jj] = T(r);
      if (jj == JT - 1 || j == nrhs - 1) {
        __syncthreads();
        const int jc = jj + 1, jb = j - jj;
        const int64_t v0 = int64_t(blockIdx.x) * WG;
        for (int t = threadIdx.x; t < WG * jc; t += WG) {
          const int vl = t / jc, cc = t - vl * jc;
          if (v0 + vl < n) Rw[(v0 + vl) * nrhs + jb + cc] = tile[vl][cc];
        }
        __syncthreads();
      }
    } else {
      if (live) R[v + j * n] = r;
    }
    const double sr = wave_sum_dpp(live ? r * r : 0.0);
    const double sb = wave_sum_dpp(live ? b * b : 0.0);
    if (lane == 0) {
      part_r[size_t(j) * nparts + pidx] = sr;
      part_b[size_t(j) * nparts + pidx] = sb;
    }
  }
}

// out[j] = sum of the nblk partial sums part[j * nblk + b] (one block per j).
__global__ __launch_bounds__(WG) void k_reduce_cols(const double* part, int nblk, double* out) {
  __shared__ double red[NWAVE];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += WG) s += part[size_t(j) * nblk + b];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[j] = s;
}

// ---------------------------------------------------------------------------
// Flexible GMRES on the correction equation A d = r (GMRES-based iterative
// refinement): the factor is the right preconditioner, applied in the storage
// precision; the Krylov basis, the Hessenberg matrix and the residual are
// FP64.  Every right-hand-side column has its own Krylov space and all
// columns advance together.  Basis blocks V, Z hold vector i of column j at
// [(i * nrhs + j) * n].  Per-column state (ks, kstate_doubles(m) each):
// H ((m+1) x m, column-major), the rotations cs[m], sn[m], g[m+1], y[m], and
// the reciprocal norm of the newest basis vector.
// ---------------------------------------------------------------------------
__host__ __device__ inline int kstate_doubles(int m) { return (m + 1) * m + 2 * m + (m + 1) + m + 1; }

// Wc = A Zc (column-major, ld n): one thread per row; the row's stencil
// entries (at most 8) are read once into registers, then every right-hand
// side in turn, its loads independent of each other.
__global__ __launch_bounds__(WG) void k_spmv(int64_t n, int nrhs, const int64_t* rowptr, const int32_t* colind,
                                             const double* vals, const double* Zc, double* Wc) {
  constexpr int ME = 8;
  const int64_t v = int64_t(blockIdx.x) * WG + threadIdx.x;
  if (v >= n) return;
  const int64_t e0 = rowptr[v], e1 = rowptr[v + 1];
  int cols[ME];
  double vv[ME];
#pragma unroll
  for (int m = 0; m < ME; ++m) {
    const bool in = e0 + m < e1;
    cols[m] = in ? colind[e0 + m] : int(v);
    vv[m] = in ? vals[e0 + m] : 0.0;
  }
  for (int j = 0; j < nrhs; ++j) {
    const double* z = Zc + size_t(j) * n;
    double ax = 0.0;
#pragma unroll
    for (int m = 0; m < ME; ++m) ax += vv[m] * z[cols[m]];
    for (int64_t e = e0 + ME; e < e1; ++e) ax += vals[e] * z[colind[e]];  // rows longer than ME
    Wc[v + size_t(j) * n] = ax;
  }
}

// Rows per thread of the Gram-Schmidt kernels; their per-wave partial sums
// go to part[(i * nrhs + j) * nparts + wave] with nparts = 4 per block of
// KRY_ROWS * 256 rows.
constexpr int KRY_ROWS = 4;

// One wave-level partial of each of <w_j, V_i[:, j]> (i < cnt) and
// ||w_j||^2 (i = cnt) over this thread's rows, w read once.
__device__ inline void kry_dots(const double (&w)[KRY_ROWS], const double* V, int64_t n, int nrhs, int j,
                                int cnt, int64_t base, double* part, int nparts) {
  const int lane = threadIdx.x & 63, pidx = blockIdx.x * NWAVE + (threadIdx.x >> 6);
  for (int i = 0; i <= cnt; ++i) {
    double a = 0.0;
    if (i < cnt) {
      const double* Vi = V + (size_t(i) * nrhs + j) * n;
      double y[KRY_ROWS];
#pragma unroll
      for (int r = 0; r < KRY_ROWS; ++r) {
        const int64_t v = base + r * WG;
        y[r] = Vi[v < n ? v : n - 1];
      }
#pragma unroll
      for (int r = 0; r < KRY_ROWS; ++r) a += w[r] * y[r];
    } else {
#pragma unroll
      for (int r = 0; r < KRY_ROWS; ++r) a += w[r] * w[r];
    }
    a = wave_sum(a);
    if (lane == 0) part[(size_t(i) * nrhs + j) * nparts + pidx] = a;
  }
}

// Partial sums of <w_j, V_i[:, j]> for i < cnt and of ||w_j||^2; reduced by
// k_reduce_cols over the (cnt + 1) * nrhs rows of part.
__global__ __launch_bounds__(WG) void k_kdots(int64_t n, int nrhs, const double* V, int cnt, const double* Wc,
                                              double* part, int nparts) {
  const int j = blockIdx.y;
  const int64_t base = int64_t(blockIdx.x) * WG * KRY_ROWS + threadIdx.x;
  double w[KRY_ROWS];
#pragma unroll
  for (int r = 0; r < KRY_ROWS; ++r) {
    const int64_t v = base + r * WG;
    w[r] = v < n ? Wc[v + j * n] : 0.0;
  }
  kry_dots(w, V, n, nrhs, j, cnt, base, part, nparts);
}

// First Gram-Schmidt pass fused with the dots of the second:
// w_j -= sum_{i < cnt} h[i * nrhs + j] V_i[:, j] (written back), then the
// partial sums of k_kdots for the new w_j.
__global__ __launch_bounds__(WG) void k_korth_dots(int64_t n, int nrhs, const double* V, int cnt,
                                                   const double* h, double* Wc, double* part, int nparts) {
  const int j = blockIdx.y;
  const int64_t base = int64_t(blockIdx.x) * WG * KRY_ROWS + threadIdx.x;
  double w[KRY_ROWS];
#pragma unroll
  for (int r = 0; r < KRY_ROWS; ++r) {
    const int64_t v = base + r * WG;
    w[r] = v < n ? Wc[v + j * n] : 0.0;
  }
  for (int i = 0; i < cnt; ++i) {
    const double* Vi = V + (size_t(i) * nrhs + j) * n;
    const double hi = h[i * nrhs + j];
#pragma unroll
    for (int r = 0; r < KRY_ROWS; ++r) {
      const int64_t v = base + r * WG;
      const double y = Vi[v < n ? v : n - 1];  // rows past n keep w = 0
      w[r] -= v < n ? hi * y : 0.0;
    }
  }
#pragma unroll
  for (int r = 0; r < KRY_ROWS; ++r) {
    const int64_t v = base + r * WG;
    if (v < n) Wc[v + j * n] = w[r];
  }
  kry_dots(w, V, n, nrhs, j, cnt, base, part, nparts);
}

// Second Gram-Schmidt pass fused with the normalisation:
// Vout[:, j] = (w_j - sum_{i < cnt} h[i * nrhs + j] V_i[:, j]) times the
// column's reciprocal norm (w_j itself is left as it is).
__global__ __launch_bounds__(WG) void k_korth_scale(int64_t n, int nrhs, int m, const double* V, int cnt,
                                                    const double* h, const double* ks, const double* Wc,
                                                    double* Vout) {
  const int j = blockIdx.y;
  const int64_t base = int64_t(blockIdx.x) * WG * KRY_ROWS + threadIdx.x;
  double w[KRY_ROWS];
#pragma unroll
  for (int r = 0; r < KRY_ROWS; ++r) {
    const int64_t v = base + r * WG;
    w[r] = v < n ? Wc[v + j * n] : 0.0;
  }
  for (int i = 0; i < cnt; ++i) {
    const double* Vi = V + (size_t(i) * nrhs + j) * n;
    const double hi = h[i * nrhs + j];
#pragma unroll
    for (int r = 0; r < KRY_ROWS; ++r) {
      const int64_t v = base + r * WG;
      const double y = Vi[v < n ? v : n - 1];  // rows past n keep w = 0
      w[r] -= v < n ? hi * y : 0.0;
    }
  }
  const double inv = ks[size_t(j) * kstate_doubles(m) + kstate_doubles(m) - 1];
#pragma unroll
  for (int r = 0; r < KRY_ROWS; ++r) {
    const int64_t v = base + r * WG;
    if (v < n) Vout[size_t(j) * n + v] = w[r] * inv;
  }
}

// Starts a cycle: g = (beta, 0, ...), beta = sqrt(nr[j]); the reciprocal
// norm scales the residual into the first basis vector.
__global__ void k_kstart(int nrhs, int m, const double* nr, double* ks) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  double* K = ks + size_t(j) * kstate_doubles(m);
  double* g = K + (m + 1) * m + 2 * m;
  const double beta = sqrt(fmax(nr[j], 0.0));
  for (int i = 0; i <= m; ++i) g[i] = 0.0;
  g[0] = beta;
  K[kstate_doubles(m) - 1] = beta > 0.0 ? 1.0 / beta : 0.0;
}

// Vi[:, j] = Wc[:, j] times the column's reciprocal norm.
__global__ __launch_bounds__(WG) void k_kscale(int64_t n, int m, const double* ks, const double* Wc, double* Vi) {
  const int j = blockIdx.y;
  const int64_t v = int64_t(blockIdx.x) * WG + threadIdx.x;
  if (v >= n) return;
  Vi[size_t(j) * n + v] = Wc[v + j * n] * ks[size_t(j) * kstate_doubles(m) + kstate_doubles(m) - 1];
}

// Arnoldi column c: H[0..c][c] = h1 + h2 (two classical Gram-Schmidt
// passes), H[c+1][c] = sqrt(||w||^2 - |h2|^2); the previous Givens rotations
// are applied, a new one annihilates H[c+1][c] and updates g; est[j] =
// |g[c+1]|, the residual norm of the correction equation.
__global__ void k_karnoldi(int nrhs, int m, int c, const double* h1, const double* h2, double* ks, double* est) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  double* K = ks + size_t(j) * kstate_doubles(m);
  double* H = K + size_t(c) * (m + 1);
  double* cs = K + (m + 1) * m;
  double* sn = cs + m;
  double* g = sn + m;
  double s2 = 0.0;
  for (int r = 0; r <= c; ++r) {
    const double b = h2[r * nrhs + j];
    H[r] = h1[r * nrhs + j] + b;
    s2 += b * b;
  }
  const double hn = sqrt(fmax(h2[(c + 1) * nrhs + j] - s2, 0.0));
  H[c + 1] = hn;
  K[kstate_doubles(m) - 1] = hn > 0.0 ? 1.0 / hn : 0.0;
  for (int r = 0; r < c; ++r) {
    const double t = cs[r] * H[r] + sn[r] * H[r + 1];
    H[r + 1] = -sn[r] * H[r] + cs[r] * H[r + 1];
    H[r] = t;
  }
  const double a = H[c], b = H[c + 1];
  const double den = sqrt(a * a + b * b);
  const double cc = den > 0.0 ? a / den : 1.0, ss = den > 0.0 ? b / den : 0.0;
  cs[c] = cc;
  sn[c] = ss;
  H[c] = den;
  H[c + 1] = 0.0;
  g[c + 1] = -ss * g[c];
  g[c] = cc * g[c];
  est[j] = fabs(g[c + 1]);
}

// y = R^{-1} g over the first k columns (R: the rotated Hessenberg matrix).
__global__ void k_ksolve(int nrhs, int m, int k, double* ks) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  double* K = ks + size_t(j) * kstate_doubles(m);
  const double* g = K + (m + 1) * m + 2 * m;
  double* y = K + (m + 1) * m + 2 * m + (m + 1);
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int t = i + 1; t < k; ++t) s -= K[size_t(t) * (m + 1) + i] * y[t];
    const double d = K[size_t(i) * (m + 1) + i];
    y[i] = d != 0.0 ? s / d : 0.0;
  }
}

// X[:, j] += sum_{i < k} y_i Z_i[:, j].
__global__ __launch_bounds__(WG) void k_kupdate(int64_t n, int nrhs, int m, int k, const double* ks,
                                                const double* Zb, double* X, int64_t ldx) {
  const int j = blockIdx.y;
  const int64_t v = int64_t(blockIdx.x) * WG + threadIdx.x;
  if (v >= n) return;
  const double* y = ks + size_t(j) * kstate_doubles(m) + (m + 1) * m + 2 * m + (m + 1);
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc += y[i] * Zb[(size_t(i) * nrhs + j) * n + v];
  X[v + j * ldx] += acc;
}

}  // namespace spalu
