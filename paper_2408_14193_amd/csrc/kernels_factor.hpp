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
