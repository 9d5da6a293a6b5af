// Device helpers shared by the kernels that evaluate k(x_i, x_j) from X:
// squared Euclidean distance by the norm expansion (RBF) or L1 distance
// (Laplacian), then exp(-gamma d) = exp2(-gamma log2(e) d) (Section 1).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace kqr {

constexpr float kLog2e = 1.4426950408889634f;

// 2^x on the transcendental unit (one v_exp_f32, about 1 ulp).  Results below
// the smallest normal FP32, 2^-126, may come out as zero: a kernel entry that
// small is far below the rounding of any sum it enters.  In the normal range
// this is the instruction exp2f is built on, without exp2f's rescaling of
// subnormal results (five more lane operations per entry).  Every kernel that
// forms k(x_i, x_j) from X uses it, so stored and recomputed entries agree
// bit for bit.
__device__ __forceinline__ float kexp2(float x) { return __builtin_amdgcn_exp2f(x); }

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

// Symmetric K stored once as the upper triangle of kPkT x kPkT tiles, tile
// (I, J), I <= J, at tile index I nt - I (I - 1) / 2 + (J - I) (nt tiles per
// side), each tile row-major.
constexpr int kPkT = 128;

__host__ __device__ __forceinline__ int64_t pk_tile_index(int64_t I, int64_t J, int64_t nt) {
  return I * nt - I * (I - 1) / 2 + (J - I);
}

// Element offset of K[i][j] in that layout.
__host__ __device__ __forceinline__ size_t pk_offset(int64_t i, int64_t j, int64_t nt) {
  const int64_t I = i / kPkT, J = j / kPkT;
  return J >= I ? size_t(pk_tile_index(I, J, nt)) * kPkT * kPkT + size_t(i % kPkT) * kPkT + size_t(j % kPkT)
                : size_t(pk_tile_index(J, I, nt)) * kPkT * kPkT + size_t(j % kPkT) * kPkT + size_t(i % kPkT);
}

// Strips of `strip` tiles over tile-rows I = 0..nt-1 of the upper triangle,
// row I holding nt - I tiles: T(M) = sum_{m=1..M} ceil(m / strip) strips over
// the last M rows.
__host__ __device__ __forceinline__ int64_t pk_strips_tail(int64_t M, int64_t strip) {
  const int64_t q = M / strip, r = M % strip;
  return strip * q * (q + 1) / 2 + r * (q + 1);
}

// Workgroup b of the 1-D strip grid -> (tile-row I, strip k within the row):
// rows before I hold pk_strips_tail(nt) - pk_strips_tail(nt - I) strips.
__device__ __forceinline__ void pk_strip_coords(int64_t b, int64_t nt, int64_t strip, int64_t& I, int64_t& k) {
  const int64_t total = pk_strips_tail(nt, strip);
  int64_t lo = 0, hi = nt - 1;  // largest I whose first strip index is <= b
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (total - pk_strips_tail(nt - mid, strip) <= b) lo = mid;
    else hi = mid - 1;
  }
  I = lo;
  k = b - (total - pk_strips_tail(nt - lo, strip));
}

}  // namespace kqr
