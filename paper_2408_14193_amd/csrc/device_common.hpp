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

// Block-wide sum of one double per thread (all threads of NW waves call).
template <int NW = NWAVE>
__device__ inline double block_sum(double v, double* red /* NW */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < NW; ++k) s += red[k];
  return s;
}

// Exclusive prefix count of a predicate over the workgroup of NW waves;
// returns the thread's offset and writes the total to *total (all threads
// call).
template <int NW = NWAVE>
__device__ inline int block_scan_flag(bool f, int* wtot /* NW */, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t m = __ballot(f);
  const uint64_t below = lane == 0 ? 0ull : (m & ((~0ull) >> (64 - lane)));
  const int inwave = __popcll(below);
  __syncthreads();
  if (lane == 0) wtot[w] = __popcll(m);
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    if (k < w) off += wtot[k];
    tot += wtot[k];
  }
  *total = tot;
  return off + inwave;
}

// A zero pivot in a diagonal block of the given level (L + 1 for a leaf):
// bit 0 of status[0] is set and status[1] keeps the largest such level, the
// first one in elimination order.
__device__ inline void flag_singular(int* status, int level) {
  atomicOr(status, 1);
  atomicMax(status + 1, level);
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

// The same pair with the Box-Muller step in single precision (the uniforms
// rounded to float): for factors stored in FP32, whose far rows carry FP32
// rounding already.
__device__ inline void gauss_pair_f32(uint32_t seed, int level, int stream, int pair, int vert, int seg, int half,
                                      float* even, float* odd) {
  uint32_t c[4] = {uint32_t(pair), uint32_t(vert), uint32_t(seg), uint32_t(half)};
  philox4x32_10(c, seed, uint32_t(2 * level + stream));
  const uint64_t a = ((uint64_t(c[1]) << 32) | c[0]) >> 11;
  const uint64_t b = ((uint64_t(c[3]) << 32) | c[2]) >> 11;
  const float u1 = float(double(a) * 0x1p-53 + 0x1p-54);
  const float u2 = float(double(b) * 0x1p-53 + 0x1p-54);
  const float r = sqrtf(-2.0f * logf(u1));
  float sn, cs;
  sincospif(2.0f * u2, &sn, &cs);
  *even = r * cs;
  *odd = r * sn;
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

}  // namespace spalu
