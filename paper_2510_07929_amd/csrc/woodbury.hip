// Preconditioner (3.2) applied through Lemma 1 (Sherman-Morrison-Woodbury):
//   P = F F^T + c 1 1^T + L,  U = [F 1],  C = diag(I_r, 1/c) + U^T L^{-1} U,
//   P^{-1} w = L^{-1} w - L^{-1} U C^{-1} U^T L^{-1} w.
// The (r+1) x (r+1) core is formed (split-n SYRK with FP64 products of the
// FP32 factor), Cholesky-factored and solved in FP64 on the device.
#include "vec.h"

#include <algorithm>
#include <cmath>

namespace kqr {

namespace {
constexpr int kT = 64;        // core tile edge
constexpr int kSubRows = 32;  // rows staged per LDS step of the SYRK
constexpr int kGtBlocks = 256;
}  // namespace

// U(i, a) = F(i, a) for a < r, 1 for a == r, 0 beyond; 0 for i >= n.
__device__ __forceinline__ double u_at(const float* __restrict__ F, int64_t ldf, int64_t n, int r,
                                       int64_t i, int a) {
  if (i >= n) return 0.0;
  if (a < r) return double(F[i * ldf + a]);
  return a == r ? 1.0 : 0.0;
}

__device__ __forceinline__ void tile_coords(int t, int& ta, int& tb) {
  int a = int((sqrtf(8.f * t + 1.f) - 1.f) * 0.5f);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  ta = a;
  tb = t - a * (a + 1) / 2;
}

// part[s][tile][64x64] = sum over rows of chunk s of (U_ia / L_i) U_ib.
__global__ __launch_bounds__(256) void syrk_kernel(const float* __restrict__ F, int64_t n, int r,
                                                   int64_t ldf, const double* __restrict__ L,
                                                   int ntile, int64_t chunk, double* __restrict__ part) {
  __shared__ double A[kSubRows][kT + 1];
  __shared__ double B[kSubRows][kT + 1];
  int ta, tb;
  tile_coords(blockIdx.x, ta, tb);
  const int s = blockIdx.y;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  const int64_t i0 = int64_t(s) * chunk;
  const int64_t i1 = min(n, i0 + chunk);
  for (int64_t ib = i0; ib < i1; ib += kSubRows) {
    for (int e = threadIdx.x; e < kSubRows * kT; e += 256) {
      const int ii = e / kT, k = e % kT;
      const int64_t i = ib + ii;
      const bool ok = i < i1;
      const double w = ok ? 1.0 / L[i] : 0.0;
      A[ii][k] = ok ? u_at(F, ldf, n, r, i, ta * kT + k) * w : 0.0;
      B[ii][k] = ok ? u_at(F, ldf, n, r, i, tb * kT + k) : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int ii = 0; ii < kSubRows; ++ii) {
      double av[4], bv[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) av[p] = A[ii][ty * 4 + p];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q] = B[ii][tx * 4 + q];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fma(av[p], bv[q], acc[p][q]);
    }
    __syncthreads();
  }
  double* out = part + (int64_t(s) * ntile + blockIdx.x) * (kT * kT);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) out[(ty * 4 + p) * kT + tx * 4 + q] = acc[p][q];
}

// C[a][b] (a >= b, inside R1) = identity/core diagonal + sum_s part[s][tile]
__global__ __launch_bounds__(256) void syrk_reduce_kernel(const double* __restrict__ part, int nsplit,
                                                          int ntile, int r, int R1, double c,
                                                          double* __restrict__ C, int64_t ldc) {
  int ta, tb;
  tile_coords(blockIdx.x, ta, tb);
  for (int e = threadIdx.x; e < kT * kT; e += 256) {
    const int a = ta * kT + e / kT, b = tb * kT + e % kT;
    if (a >= R1 || b >= R1 || b > a) continue;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t(k) * ntile + blockIdx.x) * (kT * kT) + e];
    if (a == b) s += (a < r) ? 1.0 : 1.0 / c;
    C[int64_t(a) * ldc + b] = s;
  }
}

// ---------------------------------------------------------------- blocked Cholesky (lower)
// Diagonal block: one wave factors C[kb:kb+nb, kb:kb+nb] in LDS.
__global__ __launch_bounds__(64) void chol_diag_kernel(double* __restrict__ C, int64_t ldc, int kb, int nb,
                                                       int* __restrict__ flag) {
  __shared__ double A[kT][kT + 1];
  const int l = threadIdx.x;
  for (int i = 0; i < nb; ++i)
    if (l < nb) A[i][l] = C[int64_t(kb + i) * ldc + kb + l];
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (l == 0) {
      double piv = A[j][j];
      if (!(piv > 0.0) || !isfinite(piv)) {
        flag[0] = 1;
        piv = 1e-300;
      }
      A[j][j] = sqrt(piv);
    }
    __syncthreads();
    if (l > j && l < nb) A[l][j] /= A[j][j];
    __syncthreads();
    if (l > j && l < nb)
      for (int k = j + 1; k <= l; ++k) A[l][k] = fma(-A[l][j], A[k][j], A[l][k]);
    __syncthreads();
  }
  for (int i = 0; i < nb; ++i)
    if (l <= i) C[int64_t(kb + i) * ldc + kb + l] = A[i][l];
}

// Panel: rows i >= kb+nb solve x L_kk^T = C[i, kb:kb+nb] (one thread per row).
__global__ __launch_bounds__(64) void chol_panel_kernel(double* __restrict__ C, int64_t ldc, int kb, int nb,
                                                        int R1) {
  __shared__ double Lk[kT][kT + 1];
  for (int e = threadIdx.x; e < kT * kT; e += 64) {
    const int i = e / kT, k = e % kT;
    Lk[i][k] = (i < nb && k <= i) ? C[int64_t(kb + i) * ldc + kb + k] : 0.0;
  }
  __syncthreads();
  const int64_t i = int64_t(kb) + nb + int64_t(blockIdx.x) * 64 + threadIdx.x;
  if (i >= R1) return;
  double x[kT];
  double* row = C + i * ldc + kb;
#pragma unroll
  for (int k = 0; k < kT; ++k) x[k] = k < nb ? row[k] : 0.0;
#pragma unroll
  for (int j = 0; j < kT; ++j) {
    if (j < nb) {
      x[j] /= Lk[j][j];
#pragma unroll
      for (int k = j + 1; k < kT; ++k) x[k] = fma(-x[j], Lk[k][j], x[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < kT; ++k)
    if (k < nb) row[k] = x[k];
}

// Trailing update of the lower part: C[i][j] -= sum_k P[i][k] P[j][k], j <= i.
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ C, int64_t ldc, int kb, int nb,
                                                          int R1) {
  __shared__ double Pi[kT][kT + 1];
  __shared__ double Pj[kT][kT + 1];
  int ta, tb;
  tile_coords(blockIdx.x, ta, tb);
  const int base = kb + nb;
  const int i0 = base + ta * kT, j0 = base + tb * kT;
  for (int e = threadIdx.x; e < kT * kT; e += 256) {
    const int a = e / kT, k = e % kT;
    Pi[a][k] = (i0 + a < R1 && k < nb) ? C[int64_t(i0 + a) * ldc + kb + k] : 0.0;
    Pj[a][k] = (j0 + a < R1 && k < nb) ? C[int64_t(j0 + a) * ldc + kb + k] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  for (int k = 0; k < nb; ++k) {
    double av[4], bv[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) av[p] = Pi[ty * 4 + p][k];
#pragma unroll
    for (int q = 0; q < 4; ++q) bv[q] = Pj[tx * 4 + q][k];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] = fma(av[p], bv[q], acc[p][q]);
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + ty * 4 + p, j = j0 + tx * 4 + q;
      if (i < R1 && j <= i) C[int64_t(i) * ldc + j] -= acc[p][q];
    }
}

// ---------------------------------------------------------------- apply
// g = w / L ; partial t[a] = sum_{rows of this block} U_ia g_i.  Rows of the
// block's chunk are staged in LDS 1024 at a time.
constexpr int kGtStage = 1024;
__global__ __launch_bounds__(256) void wood_gt_kernel(const float* __restrict__ F, int64_t n, int r,
                                                      int64_t ldf, int R1, const double* __restrict__ L,
                                                      const double* __restrict__ w, double* __restrict__ g,
                                                      int64_t chunk, double* __restrict__ part) {
  __shared__ double gs[kGtStage];
  const int64_t i0 = int64_t(blockIdx.x) * chunk;
  const int64_t i1 = min(n, i0 + chunk);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // columns a = tid + 256 q (R1 <= 1024)
  for (int64_t sb = i0; sb < i1; sb += kGtStage) {
    const int cnt = int(min<int64_t>(kGtStage, i1 - sb));
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += 256) {
      const double gi = w[sb + k] / L[sb + k];
      g[sb + k] = gi;
      gs[k] = gi;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = threadIdx.x + 256 * q;
      if (a < r) {
        for (int k = 0; k < cnt; ++k) acc[q] = fma(double(F[(sb + k) * ldf + a]), gs[k], acc[q]);
      } else if (a == r) {
        for (int k = 0; k < cnt; ++k) acc[q] += gs[k];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = threadIdx.x + 256 * q;
    if (a < R1) part[int64_t(blockIdx.x) * R1 + a] = acc[q];
  }
}

// t = sum of partials ; s = C^{-1} t = Lc^{-T} Lc^{-1} t (one workgroup, FP64).
__global__ __launch_bounds__(256) void wood_solve_kernel(const double* __restrict__ part, int nblk, int R1,
                                                         const double* __restrict__ C, int64_t ldc,
                                                         double* __restrict__ s_out) {
  __shared__ double y[1024];
  __shared__ double D[kT][kT + 1];
  const int tid = threadIdx.x;
  for (int a = tid; a < R1; a += 256) {
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += part[int64_t(b) * R1 + a];
    y[a] = acc;
  }
  __syncthreads();
  // forward: Lc y = t
  for (int kb = 0; kb < R1; kb += kT) {
    const int nb = min(kT, R1 - kb);
    for (int e = tid; e < kT * kT; e += 256) {
      const int i = e / kT, k = e % kT;
      D[i][k] = (i < nb && k <= i) ? C[int64_t(kb + i) * ldc + kb + k] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      double yl = tid < nb ? y[kb + tid] : 0.0;
      for (int j = 0; j < nb; ++j) {
        if (tid == j) yl /= D[j][j];
        const double yj = __shfl(yl, j);
        if (tid > j && tid < nb) yl = fma(-D[tid][j], yj, yl);
      }
      if (tid < nb) y[kb + tid] = yl;
    }
    __syncthreads();
    for (int i = kb + nb + tid; i < R1; i += 256) {
      const double* row = C + int64_t(i) * ldc + kb;
      double acc = y[i];
      for (int k = 0; k < nb; ++k) acc = fma(-row[k], y[kb + k], acc);
      y[i] = acc;
    }
    __syncthreads();
  }
  // backward: Lc^T x = y
  const int nblocks = (R1 + kT - 1) / kT;
  for (int bi = nblocks - 1; bi >= 0; --bi) {
    const int kb = bi * kT;
    const int nb = min(kT, R1 - kb);
    for (int e = tid; e < kT * kT; e += 256) {
      const int i = e / kT, k = e % kT;
      D[i][k] = (i < nb && k <= i) ? C[int64_t(kb + i) * ldc + kb + k] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      double xl = tid < nb ? y[kb + tid] : 0.0;
      for (int j = nb - 1; j >= 0; --j) {
        if (tid == j) xl /= D[j][j];
        const double xj = __shfl(xl, j);
        if (tid < j) xl = fma(-D[j][tid], xj, xl);
      }
      if (tid < nb) y[kb + tid] = xl;
    }
    __syncthreads();
    for (int i = tid; i < kb; i += 256) {
      double acc = y[i];
      for (int k = 0; k < nb; ++k) acc = fma(-C[int64_t(kb + k) * ldc + i], y[kb + k], acc);
      y[i] = acc;
    }
    __syncthreads();
  }
  for (int a = tid; a < R1; a += 256) s_out[a] = y[a];
}

// out_i = g_i - (sum_a F_ia s_a + s_r) / L_i ; optional partial dot_with . out
__global__ __launch_bounds__(256) void wood_out_kernel(const float* __restrict__ F, int64_t n, int r,
                                                       int64_t ldf, const double* __restrict__ L,
                                                       const double* __restrict__ g,
                                                       const double* __restrict__ s,
                                                       double* __restrict__ out,
                                                       const double* __restrict__ dot_with,
                                                       double* __restrict__ partials) {
  extern __shared__ double ss[];
  __shared__ double wsum[4];
  for (int a = threadIdx.x; a <= r; a += 256) ss[a] = s[a];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nw = int64_t(gridDim.x) * 4;
  double dacc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 4 + wave; i < n; i += nw) {
    const float* row = F + i * ldf;
    double acc = 0.0;
    for (int a = lane; a < r; a += 64) acc = fma(double(row[a]), ss[a], acc);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    const double o = g[i] - (acc + ss[r]) / L[i];
    if (lane == 0) {
      out[i] = o;
      if (dot_with) dacc = fma(o, dot_with[i], dacc);
    }
  }
  if (partials) {
    if (lane == 0) wsum[wave] = dacc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
  }
}

// ---------------------------------------------------------------- class
Woodbury::Woodbury(const float* F, int64_t n, int64_t r, int64_t ldf)
    : F_(F), n_(n), r_(r), ldf_(ldf), R1_(r + 1), hflag_(sizeof(int)) {
  if (R1_ > 1024) fail(KQR_EINVAL, "preconditioner rank %lld exceeds 1023", (long long)r);
  ldc_ = R1_;
  C_.alloc(size_t(R1_) * ldc_ * sizeof(double));
  const int nt = int((R1_ + kT - 1) / kT);
  const int ntile = nt * (nt + 1) / 2;
  nsplit_ = std::max(1, std::min(32, 1024 / ntile));
  const size_t syrk_part = size_t(nsplit_) * ntile * kT * kT;
  const size_t gt_part = size_t(kGtBlocks) * R1_;
  part_.alloc(std::max(syrk_part, gt_part) * sizeof(double));
  g_.alloc(size_t(std::max<int64_t>(n, 1)) * sizeof(double));
  s_.alloc(size_t(R1_) * sizeof(double));
  flag_.alloc(sizeof(int));
}

bool Woodbury::build(const double* L, double c, hipStream_t st) {
  L_ = L;
  c_ = c;
  const int R1 = int(R1_);
  const int nt = (R1 + kT - 1) / kT;
  const int ntile = nt * (nt + 1) / 2;
  int64_t chunk = (n_ + nsplit_ - 1) / nsplit_;
  chunk = (chunk + kSubRows - 1) / kSubRows * kSubRows;
  syrk_kernel<<<dim3(ntile, nsplit_), 256, 0, st>>>(F_, n_, int(r_), ldf_, L, ntile, chunk, part_.as<double>());
  KQR_LAUNCH_CHECK();
  syrk_reduce_kernel<<<ntile, 256, 0, st>>>(part_.as<double>(), nsplit_, ntile, int(r_), R1, c, C_.as<double>(),
                                            ldc_);
  KQR_LAUNCH_CHECK();
  KQR_CHECK_HIP(hipMemsetAsync(flag_.ptr, 0, sizeof(int), st));
  for (int kb = 0; kb < R1; kb += kT) {
    const int nb = std::min(kT, R1 - kb);
    chol_diag_kernel<<<1, 64, 0, st>>>(C_.as<double>(), ldc_, kb, nb, flag_.as<int>());
    KQR_LAUNCH_CHECK();
    const int rest = R1 - kb - nb;
    if (rest > 0) {
      chol_panel_kernel<<<(rest + 63) / 64, 64, 0, st>>>(C_.as<double>(), ldc_, kb, nb, R1);
      KQR_LAUNCH_CHECK();
      const int mt = (rest + kT - 1) / kT;
      chol_update_kernel<<<mt * (mt + 1) / 2, 256, 0, st>>>(C_.as<double>(), ldc_, kb, nb, R1);
      KQR_LAUNCH_CHECK();
    }
  }
  KQR_CHECK_HIP(hipMemcpyAsync(hflag_.ptr, flag_.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
  KQR_CHECK_HIP(hipStreamSynchronize(st));
  return *hflag_.as<int>() == 0;
}

void Woodbury::apply(const double* w, double* out, const double* dot_with, double* dot_out, Workspace& ws,
                     hipStream_t st) {
  const int R1 = int(R1_);
  const int64_t chunk = (n_ + kGtBlocks - 1) / kGtBlocks;
  wood_gt_kernel<<<kGtBlocks, 256, 0, st>>>(
      F_, n_, int(r_), ldf_, R1, L_, w, g_.as<double>(), chunk, part_.as<double>());
  KQR_LAUNCH_CHECK();
  wood_solve_kernel<<<1, 256, 0, st>>>(part_.as<double>(), kGtBlocks, R1, C_.as<double>(), ldc_,
                                       s_.as<double>());
  KQR_LAUNCH_CHECK();
  wood_out_kernel<<<kRedBlocks, 256, size_t(R1) * sizeof(double), st>>>(
      F_, n_, int(r_), ldf_, L_, g_.as<double>(), s_.as<double>(), out, dot_with,
      dot_with ? ws.partials : nullptr);
  KQR_LAUNCH_CHECK();
  if (dot_with) reduce_finalize(ws.partials, kRedBlocks, 1, dot_out, st);
}

}  // namespace kqr
