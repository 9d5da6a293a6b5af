// Deterministic block reductions shared by the solver's kernels.
#pragma once

#include "kqr_internal.h"

namespace kqr {

// out[q] = sum over b < nblocks of partials[b nq + q], in a fixed order (one
// 256-thread block).
__device__ __forceinline__ void finish_sums(const double* __restrict__ partials, int nblocks, int nq,
                                            double* __restrict__ out) {
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = 0; q < nq; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partials[b * nq + q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) sh[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[q] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
  }
}

// Vectors up to this length are reduced by a single workgroup (no second
// pass); longer ones by up to kRedBlocks workgroups whose partials a
// finishing launch adds.  Workgroups never wait for one another: on a GPU
// whose L2 is split over several dies, making one workgroup's writes visible
// to another inside a kernel costs an L2 write-back per workgroup.
constexpr int64_t kOneBlockN = 8192;

// Block partials; with a single workgroup they are the result and go to out
// directly, otherwise reduce_finalize adds them afterwards.
template <int NQ>
__device__ __forceinline__ void block_sums(double (&v)[NQ], double* __restrict__ partials, double* __restrict__ out) {
  __shared__ double sh[NQ][kRedThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = v[q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) sh[q][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kRedThreads / 64; ++w) s += sh[threadIdx.x][w];
    if (gridDim.x == 1) out[threadIdx.x] = s;
    else partials[blockIdx.x * NQ + threadIdx.x] = s;
  }
}

}  // namespace kqr
