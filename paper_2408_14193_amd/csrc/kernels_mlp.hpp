// Segment-rank predictor: per-segment features, BF16 inference of the
// 12-64-64-1 network (FP32 accumulation), and FP32 training kernels
// (forward, backward, Adam).  The predicted rank fraction y sets the first
// sample count of a segment's ID to ceil(margin * n * y) + p; the ID's probe
// check still decides and falls back to doubling.
#pragma once

#include "device_common.hpp"
#include "kernels_factor.hpp"
#include "layout.hpp"

namespace spalu {

constexpr int MLP_NF = 12;
constexpr int MLP_H = 64;
constexpr int MLP_OFF_MU = 0;
constexpr int MLP_OFF_SD = 12;
constexpr int MLP_OFF_W1 = 24;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_NF;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_H;
constexpr int MLP_NPARAM = MLP_OFF_B3 + 1;

// Round to the nearest bfloat16 (ties to even), returned as float.
__device__ inline float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

// Per-vertex parts of the features, once per factorization (a vertex shows
// up again at every coarser level its skeleton survives to): vf[3v] =
// (S - a_vv) m / S with S the sum of |a_vw| over its m off-diagonal entries
// (-inf when S = 0), vf[3v+1] = log(|a_vv| h^2 / 2dim) (0 without a
// diagonal), vf[3v+2] = sum |a_vw - a_wv| / sum (|a_vw| + |a_wv|) (0 when
// that is 0/0).
__global__ __launch_bounds__(WG) void k_vertex_features(int64_t nv, const int64_t* rowptr, const int32_t* colind,
                                                        const double* vals, GridGeom g, int dim, double* vf) {
  const int64_t v = int64_t(blockIdx.x) * WG + threadIdx.x;
  if (v >= nv) return;
  const double h = 1.0 / double((g.nx > g.ny ? (g.nx > g.nz ? g.nx : g.nz) : (g.ny > g.nz ? g.ny : g.nz)) + 1);
  double Ssum = 0.0, diag = 0.0, num = 0.0, den = 0.0;
  int m = 0;
  for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
    const int j = colind[e];
    const double a = vals[e];
    if (j == v) {
      diag = a;
    } else {
      Ssum += fabs(a);
      ++m;
      const double at = csr_at(rowptr, colind, vals, j, int(v));
      num += fabs(a - at);
      den += fabs(a) + fabs(at);
    }
  }
  vf[3 * v] = Ssum > 0.0 ? (Ssum - diag) * m / Ssum : -INFINITY;
  vf[3 * v + 1] = diag != 0.0 ? log(fabs(diag) * h * h / (2.0 * dim)) : 0.0;
  vf[3 * v + 2] = den > 0.0 ? num / den : 0.0;
}

// Features of every segment of a level; one wave per segment: log2(n+1),
// log2(span), wavelengths across the segment, log2(coupled DOFs + 1),
// near-row fraction, l/L, log10(1/eps)/16, on-separator flag, boundary
// contact, mean and std of log(a_vv h^2 / 2dim), mean stencil asymmetry.
// The per-vertex parts come from k_vertex_features; the neighbours' DOFs are
// spread over the lanes as one list (neighbour sizes prefix-summed).
__global__ __launch_bounds__(64) void k_features(const DSeg* segs, int nseg, const DNbr* nbrs, GridGeom g,
                                                 int dim, int L, int level, double eps, const int32_t* iarena,
                                                 DLevelDyn dyn, const double* vf, float* feats) {
  const int c = blockIdx.x;
  if (c >= nseg) return;
  const int lane = threadIdx.x;
  const DSeg S = segs[c];
  const int n = dyn.n[c];
  const int32_t* dofs = iarena + S.ioff;
  double kh2 = 0.0, gs = 0.0, gs2 = 0.0, as = 0.0;
  for (int i = lane; i < n; i += 64) {
    const int v = dofs[i];
    const double kv = vf[3 * size_t(v)], gv = vf[3 * size_t(v) + 1], av = vf[3 * size_t(v) + 2];
    kh2 = fmax(kh2, kv);
    gs += gv;
    gs2 += gv * gv;
    as += av;
  }
  kh2 = wave_max(kh2);
  gs = wave_sum(gs);
  gs2 = wave_sum(gs2);
  as = wave_sum(as);
  // neighbour b0 + lane of a batch of 64: its size and DOF list offset,
  // and where its DOFs start in the batch's list
  __shared__ int64_t s_ioff[64];
  __shared__ int s_excl[64];
  const int nnb = S.nbr_end - S.nbr_begin;
  double nV = 0.0, nearc = 0.0;
  for (int b0 = 0; b0 < nnb; b0 += 64) {
    const int e = b0 + lane, nb = nnb - b0 < 64 ? nnb - b0 : 64;
    int nd = 0;
    int64_t io = 0;
    if (e < nnb) {
      const int d = nbrs[S.nbr_begin + e].d;
      nd = dyn.n[d];
      io = segs[d].ioff;
    }
    int incl = nd;  // inclusive prefix sum of the sizes over the lanes
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    const int tot = __shfl(incl, 63, 64);
    s_ioff[lane] = io;
    s_excl[lane] = incl - nd;
    wave_sync();
    nV += double(tot);
    double cnt = 0.0;
    for (int t = lane; t < tot; t += 64) {
      int owner = 0;  // the last neighbour whose list starts at or before t
      for (int q = 1; q < nb; ++q)
        if (s_excl[q] <= t) owner = q;
      int cv[3];
      vcoords(g, iarena[s_ioff[owner] + (t - s_excl[owner])], cv);
      int dist = 0;
      for (int a = 0; a < 3; ++a) {
        int da = S.lo[a] - cv[a];
        if (cv[a] - S.hi[a] > da) da = cv[a] - S.hi[a];
        if (da > dist) dist = da;
      }
      cnt += dist <= S.thr ? 1.0 : 0.0;
    }
    nearc += 2.0 * wave_sum(cnt);
    wave_sync();
  }
  if (lane == 0) {
    int span = 0;
    bool touches = false;
    const int gd[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
      const int sa = S.hi[a] - S.lo[a] + 1;
      if (sa > span) span = sa;
      if (a < dim && (S.lo[a] == 0 || S.hi[a] == gd[a] - 1)) touches = true;
    }
    const double mean = n > 0 ? gs / n : 0.0;
    const double var = n > 0 ? fmax(gs2 / n - mean * mean, 0.0) : 0.0;
    float* f = feats + size_t(c) * MLP_NF;
    f[0] = float(log2(double(n + 1)));
    f[1] = float(log2(double(span)));
    f[2] = float(span * sqrt(kh2) / (2.0 * 3.141592653589793));
    f[3] = float(log2(nV + 1.0));
    f[4] = float(nV > 0.0 ? nearc / (2.0 * nV) : 0.0);
    f[5] = float(double(level) / L);
    f[6] = float(log10(1.0 / eps) / 16.0);
    f[7] = (S.flags & SEG_IS_SEP) ? 1.f : 0.f;
    f[8] = touches ? 1.f : 0.f;
    f[9] = float(mean);
    f[10] = float(sqrt(var));
    f[11] = float(n > 0 ? as / n : 0.0);
  }
}

// BF16 inference: weights and activations rounded to bfloat16, products
// accumulated in FP32; writes the start sample count of every regular
// segment (0 for the others, -1 for a segment predicted incompressible, which
// the ID launches then keep whole).  A group of MLP_G lanes per segment (16
// segments per block): lane l of a group forms hidden units 4l .. 4l+3 of
// each layer from the transposed weights in LDS (conflict-free rows), the
// group shares its activations through LDS, and its first lane sums the
// output layer; every sum keeps the order of the plain loop.
constexpr int MLP_G = 16;
constexpr int MLP_UPL = MLP_H / MLP_G;  // hidden units per lane

__global__ __launch_bounds__(256) void k_mlp_rank(const float* feats, int nseg, const float* params,
                                                  const DSeg* segs, DLevelDyn dyn, float margin, int pad,
                                                  float skip, int32_t* h_out) {
  constexpr int NGRP = 256 / MLP_G;
  __shared__ float sW[MLP_NPARAM];      // mu, sd, W1^T, b1, W2^T, b2, W3, b3 (BF16-rounded weights)
  __shared__ float sA[NGRP][2][MLP_H];  // per group: layer-1 and layer-2 activations
  for (int t = threadIdx.x; t < MLP_NPARAM; t += blockDim.x) {
    int d = t;  // destination: W1 and W2 transposed
    if (t >= MLP_OFF_W1 && t < MLP_OFF_B1) {
      const int o = (t - MLP_OFF_W1) / MLP_NF, k = (t - MLP_OFF_W1) % MLP_NF;
      d = MLP_OFF_W1 + k * MLP_H + o;
    } else if (t >= MLP_OFF_W2 && t < MLP_OFF_B2) {
      const int o = (t - MLP_OFF_W2) / MLP_H, k = (t - MLP_OFF_W2) % MLP_H;
      d = MLP_OFF_W2 + k * MLP_H + o;
    }
    sW[d] = t < MLP_OFF_W1 ? params[t] : bf16_round(params[t]);
  }
  __syncthreads();
  const int grp = threadIdx.x / MLP_G, l = threadIdx.x % MLP_G;
  const int c = blockIdx.x * NGRP + grp;
  if (c >= nseg) return;  // whole groups leave together
  float x[MLP_NF];
#pragma unroll
  for (int k = 0; k < MLP_NF; ++k)
    x[k] = bf16_round((feats[size_t(c) * MLP_NF + k] - sW[MLP_OFF_MU + k]) / sW[MLP_OFF_SD + k]);
  float* a1 = sA[grp][0];
  float* a2 = sA[grp][1];
  float acc[MLP_UPL];
#pragma unroll
  for (int u = 0; u < MLP_UPL; ++u) acc[u] = sW[MLP_OFF_B1 + l * MLP_UPL + u];
#pragma unroll
  for (int k = 0; k < MLP_NF; ++k)
#pragma unroll
    for (int u = 0; u < MLP_UPL; ++u) acc[u] += sW[MLP_OFF_W1 + k * MLP_H + l * MLP_UPL + u] * x[k];
#pragma unroll
  for (int u = 0; u < MLP_UPL; ++u) a1[l * MLP_UPL + u] = bf16_round(acc[u] > 0.f ? acc[u] : 0.f);
  wave_sync();
#pragma unroll
  for (int u = 0; u < MLP_UPL; ++u) acc[u] = sW[MLP_OFF_B2 + l * MLP_UPL + u];
  for (int k = 0; k < MLP_H; ++k) {
    const float hk = a1[k];
#pragma unroll
    for (int u = 0; u < MLP_UPL; ++u) acc[u] += sW[MLP_OFF_W2 + k * MLP_H + l * MLP_UPL + u] * hk;
  }
#pragma unroll
  for (int u = 0; u < MLP_UPL; ++u) a2[l * MLP_UPL + u] = bf16_round(acc[u] > 0.f ? acc[u] : 0.f);
  wave_sync();
  if (l != 0) return;
  float z = sW[MLP_OFF_B3];
  for (int o = 0; o < MLP_H; ++o) z += sW[MLP_OFF_W3 + o] * a2[o];
  const float y = 1.f / (1.f + expf(-z));
  const int n = dyn.n[c];
  const bool reg = (segs[c].flags & SEG_REGULAR) && (segs[c].flags & SEG_HAS_NBR);
  // predicted incompressible (rank n y within skip of n): kept whole, -1
  const bool keep = skip > 0.f && float(n) * y >= float(n) - skip;
  h_out[c] = !reg ? 0 : keep ? -1 : int(ceilf(margin * float(n) * y)) + pad;
}

// ---------------------------------------------------------------------------
// Training (FP32).  C[i][j] = beta C[i][j] + sum_k A[i*ai + k*ak] B[k*bk + j*bj],
// one thread per output, fixed summation order (deterministic).
// ---------------------------------------------------------------------------
__global__ void k_gemm_f32(int M, int N, int K, const float* A, int ai, int ak, const float* B, int bk, int bj,
                           float* C, int ldc, float beta) {
  const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M || j >= N) return;
  float acc = 0.f;
  for (int k = 0; k < K; ++k) acc += A[size_t(i) * ai + size_t(k) * ak] * B[size_t(k) * bk + size_t(j) * bj];
  C[size_t(i) * ldc + j] = beta != 0.f ? beta * C[size_t(i) * ldc + j] + acc : acc;
}

__global__ void k_mlp_normalize(const float* X, int B, const float* params, float* Xn) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * MLP_NF) return;
  const int k = t % MLP_NF;
  Xn[t] = (X[t] - params[MLP_OFF_MU + k]) / params[MLP_OFF_SD + k];
}

// H = relu(Z + b) in place (rows of width MLP_H).
__global__ void k_bias_relu(float* Z, int B, const float* b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * MLP_H) return;
  const float v = Z[t] + b[t % MLP_H];
  Z[t] = v > 0.f ? v : 0.f;
}

// y = sigmoid(H2 w3 + b3); dz = 2/B (y - t) y (1 - y); per-row squared error.
__global__ void k_mlp_out(const float* H2, int B, const float* params, const float* t, float* y, float* dz,
                          float* sq) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= B) return;
  float z = params[MLP_OFF_B3];
  for (int k = 0; k < MLP_H; ++k) z += H2[size_t(r) * MLP_H + k] * params[MLP_OFF_W3 + k];
  const float yy = 1.f / (1.f + expf(-z));
  y[r] = yy;
  if (t) {
    const float e = yy - t[r];
    dz[r] = 2.f / float(B) * e * yy * (1.f - yy);
    sq[r] = e * e;
  }
}

// dH2 = dz w3^T masked by H2 > 0.
__global__ void k_mlp_dh2(const float* dz, const float* H2, int B, const float* params, float* dH2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * MLP_H) return;
  const int r = t / MLP_H, k = t % MLP_H;
  dH2[t] = H2[t] > 0.f ? dz[r] * params[MLP_OFF_W3 + k] : 0.f;
}

__global__ void k_mask_pos(float* D, const float* H, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && !(H[t] > 0.f)) D[t] = 0.f;
}

// out[j] = sum_r D[r*ld + j] (column sums, fixed order).
__global__ void k_colsum(const float* D, int B, int ncol, int ld, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncol) return;
  float s = 0.f;
  for (int r = 0; r < B; ++r) s += D[size_t(r) * ld + j];
  out[j] = s;
}

__global__ void k_mean(const float* v, int B, float* out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  float s = 0.f;
  for (int r = 0; r < B; ++r) s += v[r];
  *out = s / float(B);
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int n0, int n1, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int i = n0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n1) return;
  const float mm = b1 * m[i] + (1.f - b1) * g[i];
  const float vv = b2 * v[i] + (1.f - b2) * g[i] * g[i];
  m[i] = mm;
  v[i] = vv;
  p[i] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

}  // namespace spalu
