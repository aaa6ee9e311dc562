// Factorization kernels (Algorithm 2).  One workgroup per leaf, segment or
// block of a level; all segments of a level go in one launch.  T is the
// storage type of blocks and factors (double for the plain form, float for
// the mixed form); pivoted LUs of diagonal blocks and the ID's triangular
// solve always run in FP64.
#pragma once

#include "device_common.hpp"
#include "layout.hpp"

namespace spalu {

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

// ---------------------------------------------------------------------------
// Leaf elimination (eq. (4.8)): LU of A_II and S = A_BI A_II^{-1} A_IB.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(WG) void k_leaf_factor(const DLeaf* leaves, int nleaf, GridGeom g,
                                                    const int64_t* rowptr, const int32_t* colind,
                                                    const double* vals, int32_t* iarena, T* varena,
                                                    double* gscratch, int64_t gscr_stride, int* status) {
  extern __shared__ double lds[];
  __shared__ int s_piv;
  const int lf = blockIdx.x;
  if (lf >= nleaf) return;
  const DLeaf L = leaves[lf];
  const int ni = L.ni, nb = L.nb, tid = threadIdx.x;
  const int w0 = L.hi[0] - L.lo[0] + 1, w1 = L.hi[1] - L.lo[1] + 1;
  const int32_t* bverts = iarena + L.ioff;
  int32_t* piv = iarena + L.ioff + nb;
  const bool fits = leaf_lds_need(ni, nb) <= LEAF_LDS_DOUBLES;
  double* A = fits ? lds : gscratch + size_t(lf) * gscr_stride;
  double* X = A + ni * ni;
  for (int t = tid; t < ni * ni + ni * nb; t += WG) A[t] = 0.0;
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
          if (bverts[b] == w) {
            X[i * nb + b] = vals[e];
            break;
          }
      }
    }
  }
  __syncthreads();
  if (block_lu_window(A, ni, ni, 0, piv, &s_piv)) atomicOr(status, 1);
  __syncthreads();
  // X = A_II^{-1} A_IB
  block_lower_solve<double>(A, ni, piv, ni, X, nb, nb);
  block_upper_solve<double>(A, ni, ni, X, nb, nb);
  // S = A_BI X (boundary rows, sparse)
  T* S = varena + L.s_off;
  for (int t = tid; t < nb * nb; t += WG) {
    const int b = t / nb, c = t % nb;
    const int u = bverts[b];
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
  // A_II^{-1} (stored in place of the LU; the solve applies it as a product)
  __syncthreads();
  double* Ai = A + ni * ni;
  for (int t = tid; t < ni * ni; t += WG) Ai[t] = (t / ni == t % ni) ? 1.0 : 0.0;
  __syncthreads();
  block_lower_solve<double>(A, ni, piv, ni, Ai, ni, ni);
  block_upper_solve<double>(A, ni, ni, Ai, ni, ni);
  T* LUo = varena + L.lu_off;
  for (int t = tid; t < ni * ni; t += WG) LUo[t] = T(Ai[t]);
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
  }
}

// Level-L blocks: A restricted to (c, d) minus the leaf Schur contributions.
template <typename T>
__global__ __launch_bounds__(WG) void k_assemble_leafL(const DBlk* blks, int nblk, const DSeg* segs,
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
  for (int t = threadIdx.x; t < nc * nd; t += WG) {
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
};

// CPQR of Y (m x n, column-major, ld) with fresh column norms each step and
// the tie rule of the oracle; returns k and writes |R_11| to *r11.  perm[]
// (original column index per position) is permuted alongside.
__device__ int block_cpqr(double* Y, int ld, int m, int n, int* perm, double eps, double* nrm,
                          double* s_scal, int* s_int, double* r11_out) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int kk = m < n ? m : n;
  int k = kk;
  double r11 = 0.0;
  for (int j = 0; j < kk; ++j) {
    for (int col = j + wv; col < n; col += NWAVE) {
      double s = 0.0;
      for (int i = j + lane; i < m; i += 64) {
        const double y = Y[size_t(col) * ld + i];
        s += y * y;
      }
      s = wave_sum(s);
      if (lane == 0) nrm[col] = sqrt(s);
    }
    __syncthreads();
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
      }
    }
    __syncthreads();
    const double mx = s_scal[0];
    const int q = s_int[0];
    if (j == 0) r11 = mx;
    if (mx == 0.0 || mx <= eps * r11) {
      k = j;
      break;
    }
    if (q != j) {
      for (int i = tid; i < m; i += WG) {
        const double t = Y[size_t(j) * ld + i];
        Y[size_t(j) * ld + i] = Y[size_t(q) * ld + i];
        Y[size_t(q) * ld + i] = t;
      }
      if (tid == 0) {
        const int t = perm[j];
        perm[j] = perm[q];
        perm[q] = t;
      }
    }
    __syncthreads();
    const double alpha = nrm[q];
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
    for (int col = j + 1 + wv; col < n; col += NWAVE) {
      double w = 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) w += Y[size_t(j) * ld + i] * Y[size_t(col) * ld + i];
      w = wave_sum(w) + v0 * Y[size_t(col) * ld + j];
      const double f = 2.0 * w / vv;
      if (lane == 0) Y[size_t(col) * ld + j] -= f * v0;
      for (int i = j + 1 + lane; i < m; i += 64) Y[size_t(col) * ld + i] -= f * Y[size_t(j) * ld + i];
    }
    __syncthreads();
    if (tid == 0) Y[size_t(j) * ld + j] = -sg * alpha;
    __syncthreads();
  }
  *r11_out = r11;
  return k;
}

// LDS-resident ID: sizes for which all coupling rows, the work matrix and
// a sampling tile fit the 48 KB staging buffer.
constexpr int ID_LDS_DOUBLES = 6144;
constexpr int ID_TILE = 32;            // G tile is ID_TILE x ID_TILE
constexpr int ID_MAXR = 1024;          // rows
constexpr int ID_MAXNB = 64;           // neighbour segments

__device__ inline bool id_fits_lds(int n, int R, int nnb) {
  // n <= 64: a 32-row sampling tile times n columns is at most 8 outputs
  // per thread (the per-thread accumulators)
  return nnb <= ID_MAXNB && R <= ID_MAXR && n <= 64 &&
         2 * R * n + ID_TILE * ID_TILE + 9 * n <= ID_LDS_DOUBLES;
}

// Rows of the stacked coupling matrix: 2 * sum of neighbour sizes.
__device__ inline int id_rows(const DSeg& S, const DNbr* nbrs, const DLevelDyn& dyn) {
  int R = 0;
  for (int e = S.nbr_begin; e < S.nbr_end; ++e) R += 2 * dyn.n[nbrs[e].d];
  return R;
}

template <typename T>
__global__ __launch_bounds__(WG) void k_seg_id(const DSeg* segs, int nseg, const DNbr* nbrs,
                                               const DBlk* blks, GridGeom g, int32_t* iarena,
                                               T* varena, double* scratch, DLevelDyn dyn,
                                               IdParams prm) {
  extern __shared__ double lds[];
  __shared__ double s_nrm[512];
  __shared__ double s_scal[4];
  __shared__ int s_int[4];
  __shared__ int s_w[NWAVE];
  __shared__ int s_cnt[2];
  const int c = blockIdx.x;
  if (c >= nseg) return;
  const int tid = threadIdx.x;
  const DSeg S = segs[c];
  const int n = dyn.n[c];
  const bool do_id = (S.flags & SEG_REGULAR) && (S.flags & SEG_HAS_NBR) && prm.eps > 0.0 && n > 0;
  if (do_id && id_fits_lds(n, id_rows(S, nbrs, dyn), S.nbr_end - S.nbr_begin)) return;
  int32_t* dofs = iarena + S.ioff;
  int32_t* perm = dofs + S.cap;
  int32_t* tag = perm + 2 * S.cap;  // after piv
  for (int i = tid; i < n; i += WG) perm[i] = i;
  if (!do_id) {
    if (tid == 0) {
      dyn.k[c] = n;
      dyn.nr[c] = 0;
      dyn.h[c] = 0;
      dyn.passes[c] = 0;
    }
    return;
  }
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
  // 1. stack [A_{n,c}; A_{c,n}^T] row by row, split near / far
  for (int e = S.nbr_begin; e < S.nbr_end; ++e) {
    const DNbr nb = nbrs[e];
    const int nd = dyn.n[nb.d];
    const int32_t* dd = iarena + segs[nb.d].ioff;
    for (int half = 0; half < 2; ++half) {
      const T* blk = varena + blks[half == 0 ? nb.blk_dc : nb.blk_cd].off;
      for (int base = 0; base < nd; base += WG) {
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
        const int pn = block_scan_flag(valid && near, s_w, &tn);
        const int pf = block_scan_flag(valid && !near, s_w, &tf);
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
    for (int t = tid; t < nN * n; t += WG) {
      const int j = t / nN, i = t % nN;
      Yg[size_t(j) * rc + i] = BN[size_t(j) * rc + i];
    }
    if (!sampled) {
      for (int t = tid; t < nF * n; t += WG) {
        const int f = t / n, j = t % n;
        Yg[size_t(j) * rc + nN + f] = BF[size_t(f) * n + j];
      }
    } else {
      const double sc = 1.0 / sqrt(double(h));
      for (int t = tid; t < h * n; t += WG) {
        const int i = t % h, j = t / h;
        Yg[size_t(j) * rc + nN + i] = 0.0;
      }
      for (int t = tid; t < prm.probes * n; t += WG) P[t] = 0.0;
      const int hp = h + prm.probes;  // sample rows, then probe rows
      for (int i0 = 0; i0 < hp; i0 += 32) {
        const int ih = hp - i0 < 32 ? hp - i0 : 32;
        for (int f0 = 0; f0 < nF; f0 += 64) {
          const int fw = nF - f0 < 64 ? nF - f0 : 64;
          __syncthreads();
          for (int t = tid; t < ih * fw; t += WG) {
            const int ii = t / fw, f = t % fw;
            const int row = i0 + ii;
            const int stream = row < h ? 0 : 1;
            const int r = row < h ? row : row - h;
            lds[ii * 64 + f] = gauss_entry(prm.seed, prm.level, stream, r, tag[2 * (f0 + f)], c,
                                           tag[2 * (f0 + f) + 1]);
          }
          __syncthreads();
          for (int t = tid; t < ih * n; t += WG) {
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
      for (int t = tid; t < h * n; t += WG) {
        const int i = t % h, j = t / h;
        Yg[size_t(j) * rc + nN + i] *= sc;
      }
    }
    for (int i = tid; i < n; i += WG) perm[i] = i;
    __syncthreads();
    // 3. CPQR (staged in LDS when it fits)
    const bool inlds = size_t(m) * n <= LDS_DOUBLES;
    double* Y = inlds ? lds : Yg;
    const int ld = inlds ? m : int(rc);
    if (inlds) {
      for (int t = tid; t < m * n; t += WG) {
        const int j = t / m, i = t % m;
        lds[t] = Yg[size_t(j) * rc + i];
      }
    }
    double* nrm = n <= 512 ? s_nrm : P + 8 * n;
    __syncthreads();
    k = block_cpqr(Y, ld, m, n, perm, prm.eps, nrm, s_scal, s_int, &r11);
    __syncthreads();
    // 4. T = R11^{-1} R12 (back substitution in FP64, in place in Y)
    const int nr = n - k;
    for (int q = tid; q < nr; q += WG) {
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
        for (int q = tid; q < nr; q += WG) {
          double e = P[pr * n + perm[k + q]];
          for (int t = 0; t < k; ++t) e -= P[pr * n + perm[t]] * Y[size_t(k + q) * ld + t];
          s += e * e;
        }
        s = block_sum(s, s_scal);
        worst = fmax(worst, sqrt(s));
      }
      accept = worst <= prm.tau * prm.eps * r11;
    }
    if (accept) {
      for (int t = tid; t < k * nr; t += WG) {
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
  }
}


// The same ID with every operand in LDS (small segments: the fine levels,
// where nearly all segments live).  One parallel gather of the stacked rows
// [A_{n,s}; A_{s,n}^T], one block scan to place near rows in Y and far rows
// in B_F, then sampling, CPQR, T and the probe check without leaving LDS.
template <typename T>
__global__ __launch_bounds__(WG) void k_seg_id_lds(const DSeg* segs, int nseg, const DNbr* nbrs,
                                                   const DBlk* blks, GridGeom g, int32_t* iarena,
                                                   T* varena, DLevelDyn dyn, IdParams prm) {
  extern __shared__ double lds[];
  __shared__ int s_noff[ID_MAXNB + 1];
  __shared__ int s_tag[2 * ID_MAXR];
  __shared__ int s_dst[ID_MAXR];
  __shared__ int s_perm[512];
  __shared__ double s_scal[4];
  __shared__ int s_int[4];
  __shared__ int s_w[NWAVE];
  const int c = blockIdx.x;
  if (c >= nseg) return;
  const int tid = threadIdx.x;
  const DSeg S = segs[c];
  const int n = dyn.n[c];
  const bool do_id = (S.flags & SEG_REGULAR) && (S.flags & SEG_HAS_NBR) && prm.eps > 0.0 && n > 0;
  const int nnb = S.nbr_end - S.nbr_begin;
  if (!do_id) return;  // handled (identity) by the global kernel
  const int R = id_rows(S, nbrs, dyn);
  if (!id_fits_lds(n, R, nnb)) return;
  int32_t* dofs = iarena + S.ioff;
  int32_t* perm = dofs + S.cap;
  if (tid == 0) {
    int o = 0;
    for (int e = 0; e < nnb; ++e) {
      s_noff[e] = o;
      o += 2 * dyn.n[nbrs[S.nbr_begin + e].d];
    }
    s_noff[nnb] = o;
  }
  __syncthreads();
  if (R == 0) {
    for (int i = tid; i < n; i += WG) perm[i] = i;
    if (tid == 0) {
      dyn.k[c] = n;
      dyn.nr[c] = 0;
      dyn.h[c] = 0;
      dyn.passes[c] = 0;
    }
    return;
  }
  double* Y = lds;                          // column-major, ld R
  double* BF = lds + size_t(R) * n;         // far rows, row-major (ld n)
  double* Gt = BF + size_t(R) * n;          // sampling tile
  double* P = Gt + ID_TILE * ID_TILE;       // probe rows (8 x n)
  double* nrm = P + 8 * n;                  // column norms (n)
  // 1. classify rows (near / far) and place them
  int nN = 0, nF = 0;
  for (int base = 0; base < R; base += WG) {
    const int r = base + tid;
    const bool valid = r < R;
    bool near = false;
    int v = 0, half = 0;
    if (valid) {
      int e = 0;
      while (s_noff[e + 1] <= r) ++e;
      const DNbr nb = nbrs[S.nbr_begin + e];
      const int nd = dyn.n[nb.d];
      const int q = r - s_noff[e];
      half = q / nd;
      v = iarena[segs[nb.d].ioff + (q % nd)];
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
    const int pn = block_scan_flag(valid && near, s_w, &tn);
    const int pf = block_scan_flag(valid && !near, s_w, &tf);
    if (valid) {
      if (near) {
        s_dst[r] = nN + pn;
      } else {
        s_dst[r] = -(nF + pf) - 1;
        s_tag[2 * (nF + pf)] = v;
        s_tag[2 * (nF + pf) + 1] = half;
      }
    }
    nN += tn;
    nF += tf;
  }
  __syncthreads();
  // 2. gather values: near rows into Y, far rows into BF
  for (int t = tid; t < R * n; t += WG) {
    const int r = t / n, j = t % n;
    int e = 0;
    while (s_noff[e + 1] <= r) ++e;
    const DNbr nb = nbrs[S.nbr_begin + e];
    const int nd = dyn.n[nb.d];
    const int q = r - s_noff[e];
    const int half = q / nd, i = q % nd;
    const double val = half == 0 ? double(varena[blks[nb.blk_dc].off + size_t(i) * n + j])
                                 : double(varena[blks[nb.blk_cd].off + size_t(j) * nd + i]);
    const int dst = s_dst[r];
    if (dst >= 0)
      Y[size_t(j) * R + dst] = val;
    else
      BF[size_t(-dst - 1) * n + j] = val;
  }
  __syncthreads();
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
    if (passes > 1) {
      // the previous CPQR overwrote the near rows: gather them again
      for (int t = tid; t < R * n; t += WG) {
        const int r = t / n, j = t % n;
        const int dst = s_dst[r];
        if (dst < 0) continue;
        int e = 0;
        while (s_noff[e + 1] <= r) ++e;
        const DNbr nb = nbrs[S.nbr_begin + e];
        const int nd = dyn.n[nb.d];
        const int q = r - s_noff[e];
        const int half = q / nd, i = q % nd;
        Y[size_t(j) * R + dst] = half == 0 ? double(varena[blks[nb.blk_dc].off + size_t(i) * n + j])
                                           : double(varena[blks[nb.blk_cd].off + size_t(j) * nd + i]);
      }
    }
    if (!sampled) {
      for (int t = tid; t < nF * n; t += WG) {
        const int f = t / n, j = t % n;
        Y[size_t(j) * R + nN + f] = BF[size_t(f) * n + j];
      }
    } else {
      const double sc = 1.0 / sqrt(double(h));
      const int hp = h + prm.probes;
      for (int i0 = 0; i0 < hp; i0 += ID_TILE) {
        const int ih = hp - i0 < ID_TILE ? hp - i0 : ID_TILE;
        // each thread owns (row, column) outputs of this row tile
        double acc[8];
        for (int a = 0; a < 8; ++a) acc[a] = 0.0;
        for (int f0 = 0; f0 < nF; f0 += ID_TILE) {
          const int fw = nF - f0 < ID_TILE ? nF - f0 : ID_TILE;
          __syncthreads();
          for (int t = tid; t < ih * fw; t += WG) {
            const int ii = t / fw, f = t % fw;
            const int row = i0 + ii;
            const int stream = row < h ? 0 : 1;
            const int rr = row < h ? row : row - h;
            Gt[ii * ID_TILE + f] = gauss_entry(prm.seed, prm.level, stream, rr, s_tag[2 * (f0 + f)], c,
                                               s_tag[2 * (f0 + f) + 1]);
          }
          __syncthreads();
          int a = 0;
          for (int t = tid; t < ih * n; t += WG, ++a) {
            const int ii = t / n, j = t % n;
            double sacc = 0.0;
            for (int f = 0; f < fw; ++f) sacc += Gt[ii * ID_TILE + f] * BF[size_t(f0 + f) * n + j];
            if (a < 8) acc[a] += sacc;
          }
        }
        int a = 0;
        for (int t = tid; t < ih * n; t += WG, ++a) {
          const int ii = t / n, j = t % n;
          const int row = i0 + ii;
          if (row < h)
            Y[size_t(j) * R + nN + row] = acc[a] * sc;
          else
            P[(row - h) * n + j] = acc[a];
        }
      }
    }
    for (int i = tid; i < n; i += WG) s_perm[i] = i;
    __syncthreads();
    // 3. CPQR in LDS
    k = block_cpqr(Y, R, m, n, s_perm, prm.eps, nrm, s_scal, s_int, &r11);
    __syncthreads();
    // 4. T = R11^{-1} R12 in place
    const int nr = n - k;
    for (int q = tid; q < nr; q += WG) {
      double* col = Y + size_t(k + q) * R;
      for (int i = k - 1; i >= 0; --i) {
        double sv = col[i];
        for (int t = i + 1; t < k; ++t) sv -= Y[size_t(t) * R + i] * col[t];
        col[i] = sv / Y[size_t(i) * R + i];
      }
    }
    __syncthreads();
    bool accept = true;
    if (sampled) {
      double worst = 0.0;
      for (int pr = 0; pr < prm.probes; ++pr) {
        double sv = 0.0;
        for (int q = tid; q < nr; q += WG) {
          double e = P[pr * n + s_perm[k + q]];
          for (int t = 0; t < k; ++t) e -= P[pr * n + s_perm[t]] * Y[size_t(k + q) * R + t];
          sv += e * e;
        }
        sv = block_sum(sv, s_scal);
        worst = fmax(worst, sqrt(sv));
      }
      accept = worst <= prm.tau * prm.eps * r11;
    }
    if (accept) {
      for (int t = tid; t < k * nr; t += WG) {
        const int i = t / nr, q = t % nr;
        Tm[t] = T(Y[size_t(k + q) * R + i]);
      }
      for (int i = tid; i < n; i += WG) perm[i] = s_perm[i];
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
  }
}

// ---------------------------------------------------------------------------
// Transform U_t A L_t of the diagonal block and two-stage LU (eqs. (2.7),
// (4.10)); the DOF list is reordered to [remainder; skeleton].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(WG) void k_seg_lu(const DSeg* segs, int nseg, const DBlk* blks,
                                               int32_t* iarena, T* varena, double* scratch,
                                               DLevelDyn dyn, int* status) {
  extern __shared__ double lds[];
  __shared__ int s_piv;
  const int c = blockIdx.x;
  if (c >= nseg) return;
  const int tid = threadIdx.x;
  const DSeg S = segs[c];
  const int n = dyn.n[c];
  if (n == 0) return;
  const int k = dyn.k[c], nr = dyn.nr[c];
  const bool sp = dyn.passes[c] > 0;
  int32_t* dofs = iarena + S.ioff;
  int32_t* perm = dofs + S.cap;
  int32_t* piv = perm + S.cap;
  int32_t* tmp = piv + S.cap;  // tag region, >= cap ints
  const T* M = varena + blks[S.diag_blk].off;
  const bool inlds = 2 * size_t(n) * n <= LDS_DOUBLES;
  double* W = inlds ? lds : scratch + S.scr_off;
  double* X = W + size_t(n) * n;  // inverse workspace
  // gather in [r; s] order: o[p] = perm[k + p] (p < nr), perm[p - nr]
  for (int t = tid; t < n * n; t += WG) {
    const int p = t / n, q = t % n;
    const int op = sp ? (p < nr ? perm[k + p] : perm[p - nr]) : p;
    const int oq = sp ? (q < nr ? perm[k + q] : perm[q - nr]) : q;
    W[t] = double(M[size_t(op) * n + oq]);
  }
  __syncthreads();
  if (sp && nr > 0 && k > 0) {
    const T* Tm = varena + S.t_off;  // k x nr
    // columns: W[:, q] -= W[:, nr:] T[:, q]
    for (int t = tid; t < n * nr; t += WG) {
      const int p = t / nr, q = t % nr;
      double s = 0.0;
      for (int i = 0; i < k; ++i) s += W[size_t(p) * n + nr + i] * double(Tm[size_t(i) * nr + q]);
      W[size_t(p) * n + q] -= s;
    }
    __syncthreads();
    // rows: W[p, :] -= T[:, p]^T W[nr:, :]
    for (int t = tid; t < nr * n; t += WG) {
      const int p = t / n, q = t % n;
      double s = 0.0;
      for (int i = 0; i < k; ++i) s += double(Tm[size_t(i) * nr + p]) * W[size_t(nr + i) * n + q];
      W[size_t(p) * n + q] -= s;
    }
    __syncthreads();
  }
  if (block_lu_window(W, n, n, sp ? nr : 0, piv, &s_piv)) atomicOr(status, 1);
  __syncthreads();
  // packed inverses: strictly lower part of L^{-1} (unit diagonal implied)
  // and upper part of U^{-1}, so every later application is a product
  T* LU = varena + S.lu_off;
  block_packed_inverse(W, n, X, LU);
  if (sp) {
    for (int p = tid; p < n; p += WG) tmp[p] = dofs[p < nr ? perm[k + p] : perm[p - nr]];
    __syncthreads();
    for (int p = tid; p < n; p += WG) dofs[p] = tmp[p];
  }
}

// Coupling scaling: A'_{cd} = L_ss,c^{-1} P_s,c A_cd[s_c, s_d] U_ss,d^{-1},
// with the skeleton blocks of the packed inverses of c and d (the inverse of
// a block triangular matrix has the inverse of its trailing diagonal block as
// its trailing diagonal block).
template <typename T>
__global__ __launch_bounds__(WG) void k_blk_scale(const DBlk* blks, const int32_t* blk_list, int nlist,
                                                  const DSeg* segs, const int32_t* iarena, T* varena,
                                                  DLevelDyn dyn) {
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
  const bool spc = dyn.passes[c] > 0, spd = dyn.passes[d] > 0;
  const int32_t* permc = iarena + segs[c].ioff + segs[c].cap;
  const int32_t* permd = iarena + segs[d].ioff + segs[d].cap;
  const int32_t* pivc = permc + segs[c].cap;
  const T* A = varena + B.off;
  T* out = varena + B.soff;
  const T* Lc = varena + segs[c].lu_off;  // packed inverse of c
  const T* Ud = varena + segs[d].lu_off;  // packed inverse of d
  // row map of the skeleton-part pivots of c: row i of P_s X is row rm[i]
  __shared__ int s_rm[1024];
  int* rm = kc <= 1024 ? s_rm : reinterpret_cast<int*>(lds);
  if (tid == 0) {
    for (int i = 0; i < kc; ++i) rm[i] = i;
    for (int j = 0; j < kc; ++j) {
      const int p = pivc[nrc + j] - nrc;
      const int t = rm[j];
      rm[j] = rm[p];
      rm[p] = t;
    }
  }
  __syncthreads();
  const bool inlds = 2 * size_t(kc) * kd <= LDS_DOUBLES && kc <= 1024;
  if (inlds) {
    double* X = lds;
    double* Yb = lds + size_t(kc) * kd;
    for (int t = tid; t < kc * kd; t += WG) {
      const int i = t / kd, j = t % kd;
      const int r = rm[i];
      const int si = spc ? permc[r] : r, sj = spd ? permd[j] : j;
      X[t] = double(A[size_t(si) * nd + sj]);
    }
    __syncthreads();
    for (int t = tid; t < kc * kd; t += WG) {
      const int i = t / kd, j = t % kd;
      double v = X[t];
      const T* lrow = Lc + size_t(nrc + i) * nc + nrc;
      for (int u = 0; u < i; ++u) v += double(lrow[u]) * X[size_t(u) * kd + j];
      Yb[t] = v;
    }
    __syncthreads();
    for (int t = tid; t < kc * kd; t += WG) {
      const int i = t / kd, j = t % kd;
      double v = 0.0;
      for (int u = 0; u <= j; ++u) v += Yb[size_t(i) * kd + u] * double(Ud[size_t(nrd + u) * nd + nrd + j]);
      out[t] = T(v);
    }
  } else {
    // large block: in place in the output region; columns for L^{-1}
    // (rows descending), then rows for U^{-1} (columns descending)
    for (int t = tid; t < kc * kd; t += WG) {
      const int i = t / kd, j = t % kd;
      const int r = rm[i];
      const int si = spc ? permc[r] : r, sj = spd ? permd[j] : j;
      out[t] = A[size_t(si) * nd + sj];
    }
    __syncthreads();
    for (int j = tid; j < kd; j += WG)
      for (int i = kc - 1; i > 0; --i) {
        double v = double(out[size_t(i) * kd + j]);
        const T* lrow = Lc + size_t(nrc + i) * nc + nrc;
        for (int u = 0; u < i; ++u) v += double(lrow[u]) * double(out[size_t(u) * kd + j]);
        out[size_t(i) * kd + j] = T(v);
      }
    __syncthreads();
    for (int i = tid; i < kc; i += WG)
      for (int j = kd - 1; j >= 0; --j) {
        double v = 0.0;
        for (int u = 0; u <= j; ++u)
          v += double(out[size_t(i) * kd + u]) * double(Ud[size_t(nrd + u) * nd + nrd + j]);
        out[size_t(i) * kd + j] = T(v);
      }
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
  }
}

// Separator elimination fused with the merge: every level-(l-1) block is
// assembled from identity / scaled level-l blocks minus A'_{c,s} A'_{s,d}
// for the level-l separators s next to both c and d (Z_l, Z_u, E_(l)).
template <typename T>
__global__ __launch_bounds__(WG) void k_merge_elim(const DBlk* ublks, int nublk, const int32_t* task_ptr,
                                                   const DTask* tasks, const DSepTerm* terms,
                                                   const DBlk* blks, T* varena, DLevelDyn dyn,
                                                   DLevelDyn udyn) {
  const int b = blockIdx.x;
  if (b >= nublk) return;
  const int tid = threadIdx.x;
  const DBlk U = ublks[b];
  const int nC = udyn.n[U.c], nD = udyn.n[U.d];
  T* out = varena + U.off;
  for (int t = tid; t < nC * nD; t += WG) out[t] = T(0);
  __syncthreads();
  for (int q = task_ptr[b]; q < task_ptr[b + 1]; ++q) {
    const DTask tk = tasks[q];
    const int kc = dyn.k[tk.c], kd = dyn.k[tk.d];
    const int oc = dyn.off[tk.c], od = dyn.off[tk.d];
    const T* src = tk.src >= 0 ? varena + blks[tk.src].soff : nullptr;
    for (int t = tid; t < kc * kd; t += WG) {
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
  }
}

}  // namespace spalu
