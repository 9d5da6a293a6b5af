// The linear kernel k(x, x') = x^T x' (Table 2) in factored form: K = X X^T
// has rank at most p, so K v = X (X^T v) costs O(n p) and is never stored.
// Products and sums are FP64 on the FP32 entries of X (the exact operator).
#include "kqr_internal.h"

namespace kqr {

constexpr int kLinBlocks = 256;

// part[b * p + k] = sum over the rows of block b's grid stride of X[i][k] v[i]
template <int PMAX>
__global__ __launch_bounds__(256) void lin_xtv_kernel(const float* __restrict__ X, int64_t n, int p,
                                                      const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double sh[PMAX][4];
  double acc[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) acc[k] = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double vi = v[i];
    float x[PMAX];
#pragma unroll
    for (int k = 0; k < PMAX; ++k) x[k] = X[i * p + min(k, p - 1)];  // every load issued, then used
#pragma unroll
    for (int k = 0; k < PMAX; ++k)
      if (k < p) acc[k] = fma(double(x[k]), vi, acc[k]);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    double s = acc[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) sh[k][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < p) {
    const int k = threadIdx.x;
    part[int64_t(blockIdx.x) * p + k] = ((sh[k][0] + sh[k][1]) + sh[k][2]) + sh[k][3];
  }
}

// u[i ldu] = shift + scale * sum_k Xr[i][k] t[k]
__global__ void lin_xt_kernel(const float* __restrict__ Xr, int64_t m, int p, const double* __restrict__ t,
                              double scale, double shift, double* __restrict__ u, int64_t ldu) {
  __shared__ double ts[64];
  if (threadIdx.x < p) ts[threadIdx.x] = t[threadIdx.x];
  __syncthreads();
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
  for (int k = 0; k < p; ++k) s = fma(double(Xr[i * p + k]), ts[k], s);
  u[i * ldu] = shift + scale * s;
}

size_t lin_scratch_doubles(int p) { return size_t(kLinBlocks) * p + 64; }

static void lin_xtv(const float* X, int64_t n, int p, const double* v, double* scratch, hipStream_t st) {
  double* part = scratch;
  double* t = scratch + size_t(kLinBlocks) * p;
  const dim3 grid(kLinBlocks);
  if (p <= 4) lin_xtv_kernel<4><<<grid, 256, 0, st>>>(X, n, p, v, part);
  else if (p <= 16) lin_xtv_kernel<16><<<grid, 256, 0, st>>>(X, n, p, v, part);
  else if (p <= 64) lin_xtv_kernel<64><<<grid, 256, 0, st>>>(X, n, p, v, part);
  else fail(KQR_EINVAL, "feature dimension p=%d exceeds 64", p);
  KQR_LAUNCH_CHECK();
  reduce_finalize(part, kLinBlocks, p, t, st);  // t = X^T v, blocks added in a fixed order
}

void lin_apply(const float* X, int64_t n, int p, const double* v, double* u, int64_t ldu, double* scratch,
               hipStream_t st) {
  if (n <= 0) return;
  lin_xtv(X, n, p, v, scratch, st);
  const double* t = scratch + size_t(kLinBlocks) * p;
  lin_xt_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, st>>>(X, n, p, t, 1.0, 0.0, u, ldu);
  KQR_LAUNCH_CHECK();
}

void lin_predict(const float* Xtr, int64_t n, int p, const double* alpha, const float* Xnew, int64_t m, double scale,
                 double shift, double* f, double* scratch, hipStream_t st) {
  if (m <= 0) return;
  lin_xtv(Xtr, n, p, alpha, scratch, st);
  const double* t = scratch + size_t(kLinBlocks) * p;
  lin_xt_kernel<<<dim3((unsigned)((m + 255) / 256)), 256, 0, st>>>(Xnew, m, p, t, scale, shift, f, 1);
  KQR_LAUNCH_CHECK();
}

// F[i][k] = X[i][k] for k < p, 0 for p <= k < ldf (the exact factor of X X^T)
__global__ void lin_factor_kernel(const float* __restrict__ X, int64_t n, int p, float* __restrict__ F, int64_t ldf) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= n * ldf) return;
  const int64_t i = t / ldf;
  const int k = int(t % ldf);
  F[t] = k < p ? X[i * p + k] : 0.f;
}

void lin_factor(const float* X, int64_t n, int p, float* F, int64_t ldf, hipStream_t st) {
  if (n <= 0) return;
  const int64_t tot = n * ldf;
  lin_factor_kernel<<<dim3((unsigned)((tot + 255) / 256)), 256, 0, st>>>(X, n, p, F, ldf);
  KQR_LAUNCH_CHECK();
}

}  // namespace kqr
