// Device helpers shared by the kernels that evaluate k(x_i, x_j) from X:
// squared Euclidean distance by the norm expansion (RBF) or L1 distance
// (Laplacian), then exp(-gamma d) = exp2(-gamma log2(e) d) (Section 1).
#pragma once

#include <hip/hip_runtime.h>

namespace kqr {

constexpr float kLog2e = 1.4426950408889634f;

// Distance of row x_i (norm q_i) to x_j (norm q_j), fixed padded dimension.
template <int PMAX, bool LAP>
__device__ __forceinline__ float pair_dist(const float* xi, float qi, const float* xj, float qj) {
  if (LAP) {
    float d = 0.f;
#pragma unroll
    for (int k = 0; k < PMAX; ++k) d += fabsf(xi[k] - xj[k]);
    return d;
  } else {
    float g = 0.f;
#pragma unroll
    for (int k = 0; k < PMAX; ++k) g = fmaf(xi[k], xj[k], g);
    return fmaxf(qi + qj - 2.f * g, 0.f);
  }
}

// Same with a run-time dimension (rows read from global memory).
__device__ __forceinline__ float pair_dist_dyn(const float* __restrict__ xi, float qi, const float* __restrict__ xj,
                                               float qj, int p, bool lap) {
  if (lap) {
    float d = 0.f;
    for (int k = 0; k < p; ++k) d += fabsf(xi[k] - xj[k]);
    return d;
  }
  float g = 0.f;
  for (int k = 0; k < p; ++k) g = fmaf(xi[k], xj[k], g);
  return fmaxf(qi + qj - 2.f * g, 0.f);
}

}  // namespace kqr
