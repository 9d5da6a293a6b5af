// Randomly pivoted Cholesky, F = RPCholesky(K, r), K_hat = F F^T (Section 3,
// preconditioner (3.2)).  Step i:
//   s    = first j with sum_{l<=j} d_l > u_i * sum(d)     (pivot ~ residual diagonal)
//   g    = K[:, s] - F[:, :i] F[s, :i]^T
//   F[:, i] = g / sqrt(g_s),  d <- max(d - F[:, i]^2, 0),  d_s <- 0
// The pivot is found on the device (block sums, then a wave-parallel scan of
// the selected block), so a step needs no host round trip; the host reads the
// pivot and the residual trace once per step for the early stop.
#include "vec.h"

#include <cmath>
#include <cstring>

namespace kqr {

namespace {
constexpr int kSelBlocks = 256;
}

__global__ __launch_bounds__(256) void rpc_blocksum_kernel(const double* __restrict__ d, int64_t n,
                                                           int64_t chunk, double* __restrict__ bsum) {
  __shared__ double sh[4];
  const int64_t i0 = int64_t(blockIdx.x) * chunk;
  const int64_t i1 = min(n, i0 + chunk);
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) s += d[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// One wave: locate the block whose running total passes u*total, then scan it
// 64 entries at a time with a wave prefix sum.  out: piv[step], info[0] = total.
__global__ __launch_bounds__(64) void rpc_select_kernel(const double* __restrict__ d, int64_t n, int64_t chunk,
                                                        const double* __restrict__ bsum, int nblk, double u,
                                                        int step, int64_t* __restrict__ piv,
                                                        double* __restrict__ info) {
  const int lane = threadIdx.x;
  __shared__ double pref[kSelBlocks + 1];
  if (lane == 0) {
    double acc = 0.0;
    pref[0] = 0.0;
    for (int b = 0; b < nblk; ++b) {
      acc += bsum[b];
      pref[b + 1] = acc;
    }
  }
  __syncthreads();
  const double total = pref[nblk];
  const double target = u * total;
  int bsel = -1;
  for (int b = 0; b < nblk; ++b)
    if (pref[b + 1] > target && bsum[b] > 0.0) { bsel = b; break; }
  int64_t found = -1;
  if (bsel >= 0) {
    double run = pref[bsel];
    // scan from the selected block onwards (a later block only if rounding of
    // the block sums and of the running sum disagree near the target)
    const int64_t i0 = int64_t(bsel) * chunk;
    const int64_t i1 = n;
    for (int64_t base = i0; base < i1 && found < 0; base += 64) {
      const int64_t i = base + lane;
      const double di = i < i1 ? d[i] : 0.0;
      double incl = di;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
      }
      const bool hit = (i < i1) && (run + incl > target) && di > 0.0;
      const unsigned long long m = __ballot(hit);
      if (m) {
        found = base + __ffsll((long long)m) - 1;
      } else {
        run += __shfl(incl, 63);
      }
    }
  }
  if (found < 0) {  // rounding put u*total at the very end: take the last positive entry
    for (int64_t base = ((n - 1) / 64) * 64; base >= 0 && found < 0; base -= 64) {
      const int64_t i = base + lane;
      const bool pos = i < n && d[i] > 0.0;
      const unsigned long long m = __ballot(pos);
      if (m) found = base + 63 - __clzll((long long)m);
    }
  }
  if (lane == 0) {
    piv[step] = found;
    info[0] = total;
  }
}

// g_j = krow_j - sum_{k<i} F[j][k] F[s][k]  (one wave per row j)
__global__ __launch_bounds__(256) void rpc_gcol_kernel(const float* __restrict__ F, int64_t n, int64_t ldf, int i,
                                                       const int64_t* __restrict__ piv, int step,
                                                       const double* __restrict__ krow,
                                                       double* __restrict__ g) {
  extern __shared__ float fs[];
  const int64_t s = piv[step];
  for (int k = threadIdx.x; k < i; k += 256) fs[k] = F[s * ldf + k];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nw = int64_t(gridDim.x) * 4;
  for (int64_t j = int64_t(blockIdx.x) * 4 + wave; j < n; j += nw) {
    const float* row = F + j * ldf;
    double acc = 0.0;
    for (int k = lane; k < i; k += 64) acc = fma(double(row[k]), double(fs[k]), acc);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) g[j] = krow[j] - acc;
  }
}

// F[:, i] = g / sqrt(g_s); d = max(d - f^2, 0); d_s = 0
__global__ __launch_bounds__(256) void rpc_update_kernel(float* __restrict__ F, int64_t n, int64_t ldf, int i,
                                                         const int64_t* __restrict__ piv, int step,
                                                         const double* __restrict__ g, double* __restrict__ d) {
  const int64_t s = piv[step];
  const double gs = g[s];
  const double inv = gs > 0.0 ? 1.0 / sqrt(gs) : 0.0;
  for (int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; j < n; j += int64_t(gridDim.x) * blockDim.x) {
    const double f = g[j] * inv;
    F[j * ldf + i] = float(f);
    d[j] = (j == s) ? 0.0 : fmax(d[j] - f * f, 0.0);
  }
}

__global__ void rpc_diag_kernel(const KMat km, int64_t n, double* __restrict__ d) {
  const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (j >= n) return;
  if (!km.K) { d[j] = 1.0; return; }  // k(x, x) = exp(0) for both kernels
  if (km.dtype == KQR_BF16)
    d[j] = __uint_as_float(uint32_t(static_cast<const uint16_t*>(km.K)[j * km.ld + j]) << 16);
  else
    d[j] = static_cast<const float*>(km.K)[j * km.ld + j];
}

std::vector<int64_t> rpcholesky(const KMat& km, const float* X, const float* sqn, int64_t n, int p, KernelSpec ks,
                                int64_t rank, const double* uniforms, float* F, int64_t ldf, hipStream_t st) {
  std::vector<int64_t> pivots;
  if (rank <= 0 || n <= 0) return pivots;
  rank = std::min<int64_t>(rank, n);
  if (rank > 1024) fail(KQR_EINVAL, "RPCholesky rank %lld exceeds 1024", (long long)rank);
  DevBuf d(size_t(n) * sizeof(double)), g(size_t(n) * sizeof(double)), krow(size_t(n) * sizeof(double));
  DevBuf bsum(kSelBlocks * sizeof(double)), piv(size_t(rank) * sizeof(int64_t)), info(2 * sizeof(double));
  HostPinned h(sizeof(int64_t) + sizeof(double));
  rpc_diag_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, st>>>(km, n, d.as<double>());
  KQR_LAUNCH_CHECK();
  const int64_t chunk = (n + kSelBlocks - 1) / kSelBlocks;
  double tr0 = -1.0;
  const unsigned upd_grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  for (int64_t i = 0; i < rank; ++i) {
    rpc_blocksum_kernel<<<kSelBlocks, 256, 0, st>>>(d.as<double>(), n, chunk, bsum.as<double>());
    KQR_LAUNCH_CHECK();
    rpc_select_kernel<<<1, 64, 0, st>>>(d.as<double>(), n, chunk, bsum.as<double>(), kSelBlocks, uniforms[i],
                                        int(i), piv.as<int64_t>(), info.as<double>());
    KQR_LAUNCH_CHECK();
    KQR_CHECK_HIP(hipMemcpyAsync(h.ptr, piv.as<int64_t>() + i, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    KQR_CHECK_HIP(hipMemcpyAsync(h.as<char>() + sizeof(int64_t), info.ptr, sizeof(double), hipMemcpyDeviceToHost, st));
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    const int64_t s = *h.as<int64_t>();
    double total;
    memcpy(&total, h.as<char>() + sizeof(int64_t), sizeof(double));
    if (tr0 < 0.0) tr0 = total;
    if (!(total > 1e-14 * tr0) || s < 0) break;
    pivots.push_back(s);
    kernel_row(km, X, sqn, n, p, ks, s, krow.as<double>(), st);
    rpc_gcol_kernel<<<kRedBlocks, 256, size_t(std::max<int64_t>(i, 1)) * sizeof(float), st>>>(
        F, n, ldf, int(i), piv.as<int64_t>(), int(i), krow.as<double>(), g.as<double>());
    KQR_LAUNCH_CHECK();
    rpc_update_kernel<<<upd_grid, 256, 0, st>>>(F, n, ldf, int(i), piv.as<int64_t>(), int(i), g.as<double>(),
                                                d.as<double>());
    KQR_LAUNCH_CHECK();
  }
  KQR_CHECK_HIP(hipStreamSynchronize(st));
  return pivots;
}

}  // namespace kqr
