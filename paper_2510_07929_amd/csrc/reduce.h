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

// Vectors up to this length are reduced by a single workgroup of
// kOneBlockThreads threads (no second pass); longer ones by up to kRedBlocks
// workgroups of kRedThreads whose partials a finishing launch adds.
// Workgroups never wait for one another: on a GPU whose L2 is split over
// several dies, making one workgroup's writes visible to another inside a
// kernel costs an L2 write-back per workgroup.
constexpr int64_t kOneBlockN = 16384;
constexpr int kOneBlockThreads = 1024;

// Block partials (any block size up to 1024); with a single workgroup they
// are the result and go to out directly, otherwise reduce_finalize adds them
// afterwards.  block_sums_at takes the block's index and the grid's size
// explicitly (several grids sharing one launch).
template <int NQ>
__device__ __forceinline__ void block_sums_at(double (&v)[NQ], double* __restrict__ partials,
                                              double* __restrict__ out, int blk, int nblk) {
  __shared__ double sh[NQ][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = int(blockDim.x) >> 6;
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
    for (int w = 0; w < nw; ++w) s += sh[threadIdx.x][w];
    if (nblk == 1) out[threadIdx.x] = s;
    else partials[blk * NQ + threadIdx.x] = s;
  }
}

template <int NQ>
__device__ __forceinline__ void block_sums(double (&v)[NQ], double* __restrict__ partials, double* __restrict__ out) {
  block_sums_at<NQ>(v, partials, out, int(blockIdx.x), int(gridDim.x));
}

// Sum of v over the (single) workgroup in block_sums' order, returned to
// every thread.
__device__ __forceinline__ double block_sum_all(double v) {
  __shared__ double sh[16];
  __shared__ double tot;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = int(blockDim.x) >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[w];
    tot = s;
  }
  __syncthreads();
  const double r = tot;
  __syncthreads();  // sh and tot are free for the next call
  return r;
}

// Launch shape of an O(n) reduction: one workgroup of kOneBlockThreads up
// to kOneBlockN elements, else one kRedThreads-thread workgroup per
// kRedThreads elements up to kRedBlocks (grid-stride beyond).
struct RedShape {
  unsigned blocks, threads;
};
inline RedShape red_shape(int64_t n) {
  if (n <= kOneBlockN) return RedShape{1u, unsigned(kOneBlockThreads)};
  const int64_t b = (n + kRedThreads - 1) / kRedThreads;
  return RedShape{unsigned(b < kRedBlocks ? b : kRedBlocks), unsigned(kRedThreads)};
}

}  // namespace kqr
