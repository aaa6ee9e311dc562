// Device helpers shared by the kernels: wave64 reductions, the counter-based
// Gaussian generator and small block-cooperative dense routines.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace spalu {

constexpr int WG = 256;      // threads per workgroup (4 wave64)
constexpr int NWAVE = WG / 64;
constexpr int LDS_DOUBLES = 4096;  // dynamic LDS staging buffer (32 KB)
constexpr int LEAF_LDS_DOUBLES = 6144;  // leaf factorization staging (48 KB)
constexpr int LEAF_MAX_NI = 512;        // interior vertices of a leaf box (7^3 = 343 in 3D)

// Staging doubles of a leaf: A_II (inverted in place), A_IB,
// A_II^{-1} A_IB, one column and the boundary vertex list.
__host__ __device__ inline int leaf_lds_need(int ni, int nb) { return ni * ni + 2 * ni * nb + ni + (nb + 1) / 2; }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// (value, index) max; ties go to the smaller index.
__device__ inline void wave_argmax(double& v, int& i) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int oi = __shfl_xor(i, o, 64);
    const bool take = (ov > v) | ((ov == v) & (oi < i));
    v = take ? ov : v;
    i = take ? oi : i;
  }
}

// (key, index) min; ties go to the smaller index.
__device__ inline void wave_argmin_int(int& key, int& i) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    int ok = __shfl_xor(key, o, 64);
    int oi = __shfl_xor(i, o, 64);
    if (ok < key || (ok == key && oi < i)) {
      key = ok;
      i = oi;
    }
  }
}

// Block-wide sum of one double per thread (all threads call).
__device__ inline double block_sum(double v, double* red /* NWAVE */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < NWAVE; ++k) s += red[k];
  return s;
}

// Exclusive prefix count of a predicate over the workgroup; returns the
// thread's offset and writes the total to *total (all threads call).
__device__ inline int block_scan_flag(bool f, int* wtot /* NWAVE */, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t m = __ballot(f);
  const uint64_t below = lane == 0 ? 0ull : (m & ((~0ull) >> (64 - lane)));
  const int inwave = __popcll(below);
  __syncthreads();
  if (lane == 0) wtot[w] = __popcll(m);
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NWAVE; ++k) {
    if (k < w) off += wtot[k];
    tot += wtot[k];
  }
  *total = tot;
  return off + inwave;
}

// Philox4x32-10 (Salmon et al., SC'11).
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = uint64_t(0xD2511F53u) * c[0];
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c[2];
    const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
    const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Orders the LDS accesses of one wave (no workgroup barrier).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Both normals of one Philox draw: rows 2*pair (cos branch) and 2*pair+1
// (sin branch) of the same stream, as gauss_entry defines them.
__device__ inline void gauss_pair(uint32_t seed, int level, int stream, int pair, int vert, int seg, int half,
                                  double* even, double* odd) {
  uint32_t c[4] = {uint32_t(pair), uint32_t(vert), uint32_t(seg), uint32_t(half)};
  philox4x32_10(c, seed, uint32_t(2 * level + stream));
  const uint64_t a = ((uint64_t(c[1]) << 32) | c[0]) >> 11;
  const uint64_t b = ((uint64_t(c[3]) << 32) | c[2]) >> 11;
  const double u1 = double(a) * 0x1p-53 + 0x1p-54;
  const double u2 = double(b) * 0x1p-53 + 0x1p-54;
  const double r = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * 3.141592653589793 * u2;
  *even = r * cos(ang);
  *odd = r * sin(ang);
}

// Normal number of row `row` for the DOF (vert, half) of segment `seg`:
// key (seed, 2*level+stream), counter (row>>1, vert, seg, half), two 53-bit
// uniforms, Box-Muller (cos branch for even rows, sin for odd).
__device__ inline double gauss_entry(uint32_t seed, int level, int stream, int row, int vert, int seg,
                                     int half) {
  uint32_t c[4] = {uint32_t(row) >> 1, uint32_t(vert), uint32_t(seg), uint32_t(half)};
  philox4x32_10(c, seed, uint32_t(2 * level + stream));
  const uint64_t a = ((uint64_t(c[1]) << 32) | c[0]) >> 11;
  const uint64_t b = ((uint64_t(c[3]) << 32) | c[2]) >> 11;
  const double u1 = double(a) * 0x1p-53 + 0x1p-54;
  const double u2 = double(b) * 0x1p-53 + 0x1p-54;
  const double r = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * 3.141592653589793 * u2;
  return (row & 1) ? r * sin(ang) : r * cos(ang);
}

// LU with partial pivoting, row-major A (n x n, leading dimension ld), in
// place.  Steps j < split search rows [j, split), later steps rows [j, n)
// (remainder first, then skeleton).  piv[j] = row swapped with row j.
// Ties in |a| go to the smaller row.  Returns 1 if a pivot was zero.
__device__ inline int block_lu_window(double* A, int n, int ld, int split, int* piv, int* s_piv) {
  int singular = 0;
  const int tid = threadIdx.x;
  for (int j = 0; j < n; ++j) {
    const int hi = j < split ? split : n;
    if (tid < 64) {
      double bv = -1.0;
      int bi = 1 << 30;
      for (int i = j + tid; i < hi; i += 64) {
        const double a = fabs(A[size_t(i) * ld + j]);
        if (a > bv) {
          bv = a;
          bi = i;
        }
      }
      wave_argmax(bv, bi);
      if (tid == 0) *s_piv = bi < n ? bi : j;
    }
    __syncthreads();
    const int p = *s_piv;
    if (p != j)
      for (int c = tid; c < n; c += WG) {
        const double t = A[size_t(j) * ld + c];
        A[size_t(j) * ld + c] = A[size_t(p) * ld + c];
        A[size_t(p) * ld + c] = t;
      }
    if (tid == 0) piv[j] = p;
    __syncthreads();
    const double d = A[size_t(j) * ld + j];
    if (d == 0.0) {
      singular = 1;
      continue;  // uniform: every thread read the same d
    }
    for (int i = j + 1 + tid; i < n; i += WG) A[size_t(i) * ld + j] /= d;
    __syncthreads();
    const int m = n - j - 1;
    for (int t = tid; t < m * m; t += WG) {
      const int i = j + 1 + t / m, c = j + 1 + t % m;
      A[size_t(i) * ld + c] -= A[size_t(i) * ld + j] * A[size_t(j) * ld + c];
    }
    __syncthreads();
  }
  return singular;
}

// X (n x ncol, row-major, ld) <- L^{-1} P X with the unit-lower L and the
// swaps piv of a packed LU (row-major, ldl).  Threads own columns of X for
// the swaps, then (row, column) pairs per elimination step.
template <typename TL>
__device__ inline void block_lower_solve(const TL* LU, int ldl, const int* piv, int n, double* X, int ldx,
                                         int ncol) {
  const int tid = threadIdx.x;
  for (int c = tid; c < ncol; c += WG)
    for (int j = 0; j < n; ++j) {
      const int p = piv[j];
      if (p != j) {
        const double t = X[size_t(j) * ldx + c];
        X[size_t(j) * ldx + c] = X[size_t(p) * ldx + c];
        X[size_t(p) * ldx + c] = t;
      }
    }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int m = n - j - 1;
    for (int t = tid; t < m * ncol; t += WG) {
      const int i = j + 1 + t / ncol, c = t % ncol;
      X[size_t(i) * ldx + c] -= double(LU[size_t(i) * ldl + j]) * X[size_t(j) * ldx + c];
    }
    __syncthreads();
  }
}

// X (n x ncol) <- U^{-1} X with the upper triangle of a packed LU.
template <typename TL>
__device__ inline void block_upper_solve(const TL* LU, int ldl, int n, double* X, int ldx, int ncol) {
  const int tid = threadIdx.x;
  for (int j = n - 1; j >= 0; --j) {
    for (int c = tid; c < ncol; c += WG) X[size_t(j) * ldx + c] /= double(LU[size_t(j) * ldl + j]);
    __syncthreads();
    for (int t = tid; t < j * ncol; t += WG) {
      const int i = t / ncol, c = t % ncol;
      X[size_t(i) * ldx + c] -= double(LU[size_t(i) * ldl + j]) * X[size_t(j) * ldx + c];
    }
    __syncthreads();
  }
}

// Packed inverses of a unit-lower / upper LU (row-major n x n in W):
// out[i][j] = (L^{-1})[i][j] for i > j, (U^{-1})[i][j] for i <= j.  X is an
// n x n double workspace.
template <typename TO>
__device__ inline void block_packed_inverse(const double* W, int n, double* X, TO* out) {
  const int tid = threadIdx.x;
  // L^{-1}: forward elimination on the identity (columns c <= j are live)
  for (int t = tid; t < n * n; t += WG) X[t] = (t / n == t % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int m = n - j - 1;
    for (int t = tid; t < m * (j + 1); t += WG) {
      const int i = j + 1 + t / (j + 1), cidx = t % (j + 1);
      X[size_t(i) * n + cidx] -= W[size_t(i) * n + j] * X[size_t(j) * n + cidx];
    }
    __syncthreads();
  }
  for (int t = tid; t < n * n; t += WG)
    if (t / n > t % n) out[t] = TO(X[t]);
  __syncthreads();
  // U^{-1}: back substitution on the identity
  for (int t = tid; t < n * n; t += WG) X[t] = (t / n == t % n) ? 1.0 : 0.0;
  __syncthreads();
  block_upper_solve<double>(W, n, n, X, n, n);
  for (int t = tid; t < n * n; t += WG)
    if (t / n <= t % n) out[t] = TO(X[t]);
  __syncthreads();
}

}  // namespace spalu
