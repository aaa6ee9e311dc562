// One-wave product tiles on the matrix cores (FP64 16x16x4 MFMA), shared by
// the factorization's and the solve's kernels.
#pragma once

namespace spalu {

typedef double gg_v4 __attribute__((ext_vector_type(4)));

// One wave's product tile on the matrix cores:
// acc[c] += sum over u in [u0, u1) of a(i, u) b(u, 16c + l%16) for the
// 16-row tile at i0, FP64 16x16x4 MFMA.  Lane l of a k-step supplies
// a(i0 + l%16, u) and b(u, .) for u = k0 + l/16 (a() loads with clamped
// addresses and returns 0 outside the operator, b() reads clamped rows);
// the operator entries of SW_KS k-steps are loaded together before their
// products.  Lane l receives column 16c + l%16 of rows i0 + l/16 + 4r.
constexpr int SW_KS = 8;

template <typename AF, typename BF>
__device__ inline void wave_tile_mfma(AF a, BF b, int i0, int u0, int u1, int nct, gg_v4 acc[4]) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int i = i0 + li;
  for (int ub = u0; ub < u1; ub += 4 * SW_KS) {
    double av[SW_KS];
#pragma unroll
    for (int s = 0; s < SW_KS; ++s) av[s] = ub + 4 * s < u1 ? a(i, ub + 4 * s + lk) : 0.0;
#pragma unroll
    for (int s = 0; s < SW_KS; ++s) {
      if (ub + 4 * s >= u1) break;
      const int u = ub + 4 * s + lk;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < nct) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], b(u, 16 * c + li), acc[c], 0, 0, 0);
    }
  }
}

}  // namespace spalu
