// Preconditioner (3.2) applied through Lemma 1 (Sherman-Morrison-Woodbury):
//   P = F F^T + c 1 1^T + L,  U = [F 1],  C = diag(I_r, 1/c) + U^T L^{-1} U,
//   P^{-1} w = L^{-1} w - L^{-1} U C^{-1} U^T L^{-1} w.
//
// Device-side, all FP64:
//  * the core C is formed by a split-n SYRK of the FP32 factor (FP64
//    products).  In the Newton systems (3.1) L takes two values,
//    l_in = lambda eps_t on the interior set E and l_out = lambda sigma +
//    lambda eps_t elsewhere, so U^T L^{-1} U = G_all / l_out +
//    (1/l_in - 1/l_out) U_E^T U_E with G_all = U^T U formed once per fit; a
//    Newton step then only sums over the |E| interior rows.
//  * C = Lc Lc^T by a blocked right-looking Cholesky (64-column panels; the
//    diagonal block is factored by one wave, one row per lane, with the
//    panel columns finished in registers);
//    W = Lc^{-1} is formed explicitly by recursive doubling
//    (W21 = -W22 L21 W11), so an application needs two triangular mat-vecs
//    over many workgroups instead of sequential substitutions, and
//    s = W^T (W t) stays a symmetric positive definite map.
//  * U s uses a skinny streamed mat-vec with F as the matrix.
#include "pstep.h"
#include "reduce.h"
#include "vec.h"

#include <algorithm>
#include <atomic>
#include <cmath>

namespace kqr {

namespace {
constexpr int kT = 64;        // SYRK / update / GEMM tile edge
constexpr int kSubRows = 32;  // rows staged per LDS step of the SYRK
constexpr int kNb = 64;       // Cholesky panel width = inverse leaf block
constexpr int kLt = 32;       // output tile edge of the Cholesky update and the doubling GEMMs
constexpr int kGtBlocks = 512;
constexpr int kGtStage = 256;
}  // namespace

// U(i, a) = F(i, a) for a < r, 1 for a == r, 0 beyond.
__device__ __forceinline__ double u_at(const float* __restrict__ F, int64_t ldf, int r, int64_t i, int a) {
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

// *p if ok, else 0, with the load issued unconditionally (p must be a valid
// address either way): a load under a data-dependent branch is followed by a
// full wait, so a loop of them runs one memory latency per element.
__device__ __forceinline__ double load_or_zero(const double* p, bool ok) {
  const double v = *p;
  return ok ? v : 0.0;
}

// part[s][tile][64x64] = sum over rows of chunk s of w_i U_ia U_ib, where the
// rows are idx[k] (or k itself when idx is null) and w_i = 1/L_i (or 1).
__global__ __launch_bounds__(256) void syrk_kernel(const float* __restrict__ F, int64_t nrows, int r,
                                                   int64_t ldf, const double* __restrict__ L,
                                                   const int* __restrict__ idx, int ntile, int64_t chunk,
                                                   double* __restrict__ part) {
  __shared__ double A[kSubRows][kT + 1];
  __shared__ double B[kSubRows][kT + 1];
  __shared__ int64_t rows[kSubRows];
  __shared__ double wts[kSubRows];
  int ta, tb;
  tile_coords(blockIdx.x, ta, tb);
  const int s = blockIdx.y;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  const int64_t k0 = int64_t(s) * chunk;
  const int64_t k1 = min(nrows, k0 + chunk);
  for (int64_t kb = k0; kb < k1; kb += kSubRows) {
    // the stage's rows and weights first (one lane per row), then every
    // element load issued unconditionally at a clamped address
    if (threadIdx.x < kSubRows) {
      const int64_t kk = kb + threadIdx.x;
      const int64_t i = kk < k1 ? (idx ? int64_t(idx[kk]) : kk) : -1;
      rows[threadIdx.x] = i;
      wts[threadIdx.x] = i < 0 ? 0.0 : (L ? 1.0 / L[i] : 1.0);
    }
    __syncthreads();
    double fa[kSubRows * kT / 256], fb[kSubRows * kT / 256];
    if (r > 0) {  // the same in every lane; an empty factor (r = 0, F may be null) is never read
#pragma unroll
      for (int t = 0; t < kSubRows * kT / 256; ++t) {
        const int e = int(threadIdx.x) + 256 * t;
        const int ii = e / kT, k = e % kT;
        const int64_t ic = rows[ii] < 0 ? 0 : rows[ii];
        fa[t] = double(F[ic * ldf + min(ta * kT + k, r - 1)]);
        fb[t] = double(F[ic * ldf + min(tb * kT + k, r - 1)]);
      }
    } else {
#pragma unroll
      for (int t = 0; t < kSubRows * kT / 256; ++t) fa[t] = fb[t] = 0.0;
    }
#pragma unroll
    for (int t = 0; t < kSubRows * kT / 256; ++t) {
      const int e = int(threadIdx.x) + 256 * t;
      const int ii = e / kT, k = e % kT;
      const int64_t i = rows[ii];
      const int ca = ta * kT + k, cb = tb * kT + k;
      const double ua = ca < r ? fa[t] : (ca == r ? 1.0 : 0.0);
      const double ub = cb < r ? fb[t] : (cb == r ? 1.0 : 0.0);
      A[ii][k] = i < 0 ? 0.0 : ua * wts[ii];
      B[ii][k] = i < 0 ? 0.0 : ub;
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

// C[a][b] (b <= a < R1) = diag(I_r, 1/c)[a][b] + alpha G[a][b] + beta sum_s part[s][tile]
// G (optional) is a lower-triangular R1 x R1 matrix with leading dimension ldc.
__global__ __launch_bounds__(256) void syrk_combine_kernel(const double* __restrict__ part, int nsplit, int ntile,
                                                           int r, int R1, double diag_r, double diag_last,
                                                           const double* __restrict__ G, double alpha, double beta,
                                                           double* __restrict__ C, int64_t ldc) {
  int ta, tb;
  tile_coords(blockIdx.x, ta, tb);
  for (int e = threadIdx.x; e < kT * kT; e += 256) {
    const int a = ta * kT + e / kT, b = tb * kT + e % kT;
    if (a >= R1 || b > a) continue;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t(k) * ntile + blockIdx.x) * (kT * kT) + e];
    double v = beta * s;
    if (G) v = fma(alpha, G[int64_t(a) * ldc + b], v);
    if (a == b) v += (a < r) ? diag_r : diag_last;
    C[int64_t(a) * ldc + b] = v;
  }
}

// ---------------------------------------------------------------- interior index list
__global__ __launch_bounds__(256) void flag_count_kernel(const uint8_t* __restrict__ S, int64_t n, int64_t chunk,
                                                         int* __restrict__ counts) {
  __shared__ int sh[256];
  const int64_t i0 = int64_t(blockIdx.x) * chunk, i1 = min(n, i0 + chunk);
  int c = 0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) c += S[i] ? 1 : 0;
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = sh[0];
}

// Exclusive scan of nblk <= 256 counts in place by one wave (4 per lane).
__global__ __launch_bounds__(64) void flag_scan_kernel(int* __restrict__ counts, int nblk, int* __restrict__ total) {
  const int l = threadIdx.x;
  int c[4];
  int s = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = l * 4 + q;
    c[q] = b < nblk ? counts[b] : 0;
    s += c[q];
  }
  int incl = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off);
    if (l >= off) incl += t;
  }
  int excl = incl - s;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = l * 4 + q;
    if (b < nblk) counts[b] = excl;
    excl += c[q];
  }
  if (l == 63) total[0] = incl;
}

// Each block writes the indices of its chunk in increasing order (one wave scans).
__global__ __launch_bounds__(64) void flag_scatter_kernel(const uint8_t* __restrict__ S, int64_t n, int64_t chunk,
                                                          const int* __restrict__ offsets, int* __restrict__ idx) {
  const int lane = threadIdx.x;
  const int64_t i0 = int64_t(blockIdx.x) * chunk, i1 = min(n, i0 + chunk);
  int base = offsets[blockIdx.x];
  for (int64_t b = i0; b < i1; b += 64) {
    const int64_t i = b + lane;
    const bool f = i < i1 && S[i];
    const unsigned long long m = __ballot(f);
    if (f) idx[base + __popcll(m & ((1ull << lane) - 1ull))] = int(i);
    base += __popcll(m);
  }
}

// ---------------------------------------------------------------- blocked Cholesky (lower)
__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// 1 / sqrt(a) for a normal a > 0: v_rsq_f64 and two Newton steps
// y <- y + y (1 - a y^2) / 2.
__device__ __forceinline__ double rsqrt_f64(double a) {
  double y = __builtin_amdgcn_rsq(a);
  y = fma(0.5 * y, fma(-a * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-a * y, y, 1.0), y);
  return y;
}

// Diagonal block (nb <= 64), one wave.  The block sits in LDS column-major
// (Ac[k][i] = A[i][k]) and lane l owns row l.  Columns go in panels of
// eight: every lane first subtracts sum_{k<j0} L[l][k] L[j][k] from its row's
// eight panel entries (per earlier column k: its own L[l][k], a
// conflict-free read, and the panel rows' L[j0..j0+7][k], contiguous
// broadcast reads), then finishes the panel in registers column by column:
// the pivot comes from lane j (readlane), its reciprocal square root from
// rsqrt_f64, and the multipliers L[j0+c2][j] of the later panel columns from
// their lanes, so the panel needs no LDS traffic and no barrier until it is
// written back.  The loop over panels is not unrolled, so the kernel stays
// small in the instruction cache.
__global__ __launch_bounds__(64) void chol_diag_kernel(double* __restrict__ C, int64_t ldc, int kb, int nb,
                                                       int* __restrict__ flag) {
  __shared__ __align__(16) double Ac[kNb][kNb + 2];  // row stride 528 bytes: 16-byte aligned, banks spread
  const int l = threadIdx.x;
  // coalesced: one row of the block per step, lane l reads column l (the
  // address clamped into the block's lower triangle, so all 64 loads are in
  // flight at once)
  {
    double t[kNb];
#pragma unroll
    for (int i = 0; i < kNb; ++i) {
      const int ic = min(i, nb - 1);
      t[i] = C[int64_t(kb + ic) * ldc + kb + min(l, ic)];
    }
#pragma unroll
    for (int i = 0; i < kNb; ++i) Ac[l][i] = (i < nb && l <= i) ? t[i] : (i == l ? 1.0 : 0.0);
  }
  __syncthreads();
  bool bad = false;
  constexpr int PW = 8;
  for (int j0 = 0; j0 < kNb; j0 += PW) {
    double v[PW];
#pragma unroll
    for (int c = 0; c < PW; ++c) v[c] = Ac[j0 + c][l];
#pragma unroll 4
    for (int k = 0; k < j0; ++k) {
      const double a = Ac[k][l];
      const double2 b01 = *reinterpret_cast<const double2*>(&Ac[k][j0]);
      const double2 b23 = *reinterpret_cast<const double2*>(&Ac[k][j0 + 2]);
      const double2 b45 = *reinterpret_cast<const double2*>(&Ac[k][j0 + 4]);
      const double2 b67 = *reinterpret_cast<const double2*>(&Ac[k][j0 + 6]);
      v[0] = fma(-a, b01.x, v[0]);
      v[1] = fma(-a, b01.y, v[1]);
      v[2] = fma(-a, b23.x, v[2]);
      v[3] = fma(-a, b23.y, v[3]);
      v[4] = fma(-a, b45.x, v[4]);
      v[5] = fma(-a, b45.y, v[5]);
      v[6] = fma(-a, b67.x, v[6]);
      v[7] = fma(-a, b67.y, v[7]);
    }
#pragma unroll
    for (int c = 0; c < PW; ++c) {
      const int j = j0 + c;
      double piv = readlane_f64(v[c], j);
      if (!(piv > 0.0) || !isfinite(piv)) {  // the same in every lane
        bad = true;
        piv = 1e-300;
      }
      const double y = rsqrt_f64(piv);
      v[c] = (l == j) ? piv * y : v[c] * y;  // rows above j hold unused entries
#pragma unroll
      for (int c2 = c + 1; c2 < PW; ++c2) v[c2] = fma(-v[c], readlane_f64(v[c], j0 + c2), v[c2]);
    }
#pragma unroll
    for (int c = 0; c < PW; ++c) Ac[j0 + c][l] = v[c];
    __syncthreads();
  }
  if (bad && l == 0) flag[0] = 1;
  for (int i = 0; i < nb; ++i)
    if (l <= i) C[int64_t(kb + i) * ldc + kb + l] = Ac[l][i];
}

// Panel: rows i >= kb+nb solve x L_kk^T = C[i, kb:kb+nb].  One wave per row,
// lane k owns x_k; column j is finished by lane j (times the reciprocal of
// the pivot) and broadcast by readlane.
__global__ __launch_bounds__(256) void chol_panel_kernel(double* __restrict__ C, int64_t ldc, int kb, int nb,
                                                         int R1) {
  __shared__ double Lk[kNb][kNb + 1];
  __shared__ double rinv[kNb];
#pragma unroll
  for (int t = 0; t < kNb * kNb / 256; ++t) {
    const int e = int(threadIdx.x) + 256 * t;
    const int i = e / kNb, k = e % kNb;
    const int ic = min(i, nb - 1);
    const double v = load_or_zero(C + int64_t(kb + ic) * ldc + kb + min(k, ic), i < nb && k <= i);
    Lk[i][k] = (i >= nb && i == k) ? 1.0 : v;
  }
  __syncthreads();
  if (threadIdx.x < kNb) rinv[threadIdx.x] = 1.0 / Lk[threadIdx.x][threadIdx.x];
  __syncthreads();
  const int k = threadIdx.x & 63;
  const int64_t i = int64_t(kb) + nb + int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const bool ok = i < R1;
  double* row = C + (ok ? i : 0) * ldc + kb;
  double x = (ok && k < nb) ? row[k] : 0.0;
  for (int j = 0; j < kNb; ++j) {
    if (k == j) x *= rinv[j];
    const double xj = readlane_f64(x, j);
    if (k > j) x = fma(-xj, Lk[k][j], x);
  }
  if (ok && k < nb) row[k] = x;
}

// Trailing update of the lower part: C[i][j] -= sum_k P[i][k] P[j][k], j <= i,
// over the 64-wide panel P.  One workgroup per 32 x 32 lower tile (2 x 2
// outputs per thread), K in two chunks of 32: the second chunk's global loads
// are in flight while the first is multiplied.
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ C, int64_t ldc, int kb, int nb,
                                                          int R1) {
  __shared__ double Pi[2][kLt][kLt + 1];  // Pi[buf][a][k] = P[i0 + a][k]
  __shared__ double Pj[2][kLt][kLt + 1];  // Pj[buf][k][b] = P[j0 + b][k]
  int ta, tb;
  tile_coords(blockIdx.x, ta, tb);
  const int base = kb + nb;
  const int i0 = base + ta * kLt, j0 = base + tb * kLt;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double ri[4], rj[4];
  auto load = [&](int h) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int a = e >> 5, k = e & 31;  // row a of the tile, column h + k of the panel
      const bool kk = h + k < nb;
      const int kc = kb + min(h + k, nb - 1);
      ri[q] = load_or_zero(C + int64_t(min(i0 + a, R1 - 1)) * ldc + kc, i0 + a < R1 && kk);
      rj[q] = load_or_zero(C + int64_t(min(j0 + a, R1 - 1)) * ldc + kc, j0 + a < R1 && kk);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int a = e >> 5, k = e & 31;
      Pi[buf][a][k] = ri[q];
      Pj[buf][k][a] = rj[q];
    }
  };
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int h = 0; h < nb; h += kLt, buf ^= 1) {
    const bool next = h + kLt < nb;
    if (next) load(h + kLt);
#pragma unroll 8
    for (int k = 0; k < kLt; ++k) {
      const double a0 = Pi[buf][ty * 2][k], a1 = Pi[buf][ty * 2 + 1][k];
      const double b0 = Pj[buf][k][tx * 2], b1 = Pj[buf][k][tx * 2 + 1];
      acc[0][0] = fma(a0, b0, acc[0][0]);
      acc[0][1] = fma(a0, b1, acc[0][1]);
      acc[1][0] = fma(a1, b0, acc[1][0]);
      acc[1][1] = fma(a1, b1, acc[1][1]);
    }
    if (next) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int i = i0 + ty * 2 + p, j = j0 + tx * 2 + q;
      if (i < R1 && j <= i) C[int64_t(i) * ldc + j] -= acc[p][q];
    }
}

// ---------------------------------------------------------------- W = Lc^{-1}
// Inverse of each 64 x 64 diagonal block: lane j forms column j of the
// inverse, X[i][j] = (delta_ij - sum_{k<i} L[i][k] X[k][j]) / L[i][i], in
// panels of eight rows: every lane first subtracts the earlier rows'
// contributions (per earlier row k: its own X[k][j], a conflict-free read,
// and the panel rows' L[i0..i0+7][k] from the transposed factor, contiguous
// broadcast reads), then finishes the panel in registers.  Entries above the
// diagonal come out as exact zeros.  Blocks are independent (one workgroup
// each).  W must be zero outside the blocks written here before the doubling
// steps run.
__global__ __launch_bounds__(64) void trinv_diag_kernel(const double* __restrict__ C, int64_t ldc, int R1,
                                                        double* __restrict__ W) {
  __shared__ __align__(16) double Lt[kNb][kNb + 2];  // Lt[k][i] = L[i][k]
  __shared__ __align__(16) double X[kNb][kNb];
  __shared__ double rinv[kNb];
  const int kb = blockIdx.x * kNb;
  const int nb = min(kNb, R1 - kb);
  const int j = threadIdx.x;
  // coalesced: one row of the block per step, lane j reads column j (the
  // address clamped into the block's lower triangle, so all 64 loads are in
  // flight at once)
  {
    double t[kNb];
#pragma unroll
    for (int i = 0; i < kNb; ++i) {
      const int ic = min(i, nb - 1);
      t[i] = C[int64_t(kb + ic) * ldc + kb + min(j, ic)];
    }
#pragma unroll
    for (int i = 0; i < kNb; ++i) Lt[j][i] = (i < nb && j <= i) ? t[i] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  rinv[j] = 1.0 / Lt[j][j];
  __syncthreads();
  constexpr int PW = 8;
  for (int i0 = 0; i0 < kNb; i0 += PW) {
    double x[PW];
#pragma unroll
    for (int c = 0; c < PW; ++c) x[c] = (i0 + c == j) ? 1.0 : 0.0;
#pragma unroll 4
    for (int k = 0; k < i0; ++k) {
      const double xk = X[k][j];
      const double2 l01 = *reinterpret_cast<const double2*>(&Lt[k][i0]);
      const double2 l23 = *reinterpret_cast<const double2*>(&Lt[k][i0 + 2]);
      const double2 l45 = *reinterpret_cast<const double2*>(&Lt[k][i0 + 4]);
      const double2 l67 = *reinterpret_cast<const double2*>(&Lt[k][i0 + 6]);
      x[0] = fma(-l01.x, xk, x[0]);
      x[1] = fma(-l01.y, xk, x[1]);
      x[2] = fma(-l23.x, xk, x[2]);
      x[3] = fma(-l23.y, xk, x[3]);
      x[4] = fma(-l45.x, xk, x[4]);
      x[5] = fma(-l45.y, xk, x[5]);
      x[6] = fma(-l67.x, xk, x[6]);
      x[7] = fma(-l67.y, xk, x[7]);
    }
#pragma unroll
    for (int c = 0; c < PW; ++c) {
#pragma unroll
      for (int c1 = 0; c1 < c; ++c1) x[c] = fma(-Lt[i0 + c1][i0 + c], x[c1], x[c]);
      x[c] *= rinv[i0 + c];
    }
#pragma unroll
    for (int c = 0; c < PW; ++c) X[i0 + c][j] = x[c];  // the lane's own column: no barrier needed
  }
  if (j < nb)
    for (int i = 0; i < nb; ++i) W[int64_t(kb + i) * ldc + kb + j] = X[i][j];
}

// One doubling level with blocks of s rows: for every pair (top = [i0, i0+s),
// bottom = [i0+s, min(i0+2s, R1))), computes Out[bottom, top] =
// alpha * A[bottom, A-cols] * B[B-rows, top] where
//   stage 0: A = Lc[bottom, top]   (K = s),        B = W[top, top],   Out = T
//   stage 1: A = W[bottom, bottom] (K = |bottom|),  B = T[bottom, top], Out = W (alpha = -1)
// Grid: (pair, 32 x 32 output tile), 2 x 2 outputs per thread; K goes in
// chunks of 32 with the next chunk's global loads in flight while the
// current one is multiplied (double-buffered LDS).
__global__ __launch_bounds__(256) void trinv_level_kernel(const double* __restrict__ Lc, const double* __restrict__ W,
                                                          const double* __restrict__ T, double* __restrict__ out,
                                                          int64_t ldc, int R1, int s, int stage, int tiles_per_pair) {
  __shared__ double As[2][kLt][kLt + 1];  // As[buf][row][k]
  __shared__ double Bs[2][kLt][kLt + 1];  // Bs[buf][k][col]
  const int pair = blockIdx.x / tiles_per_pair;
  const int tile = blockIdx.x % tiles_per_pair;
  const int i0 = pair * 2 * s;
  const int bot0 = i0 + s;
  const int bot_len = min(s, R1 - bot0);
  if (bot_len <= 0) return;
  const int tiles_n = s / kLt;  // columns of the output block (top) in tiles
  const int tm = tile / tiles_n, tn = tile % tiles_n;
  const int r0 = tm * kLt;  // row offset inside bottom
  const int c0 = tn * kLt;  // column offset inside top
  if (r0 >= bot_len) return;
  const int K = stage == 0 ? s : bot_len;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double ra[4], rb[4];
  auto load = [&](int kb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int hi = e >> 5, lo = e & 31;
      // A: row hi of the tile, column kb + lo;  B: row kb + hi, column lo of the tile
      const int row = r0 + hi, ka = kb + lo, kbr = kb + hi, col = c0 + lo;
      const int rowc = min(row, bot_len - 1), kac = min(ka, K - 1), kbc = min(kbr, K - 1);
      const double* pa = stage == 0 ? Lc + int64_t(bot0 + rowc) * ldc + i0 + kac
                                    : W + int64_t(bot0 + rowc) * ldc + bot0 + kac;
      const double* pb = stage == 0 ? W + int64_t(i0 + kbc) * ldc + i0 + col : T + int64_t(bot0 + kbc) * ldc + i0 + col;
      ra[q] = load_or_zero(pa, row < bot_len && ka < K);
      rb[q] = load_or_zero(pb, kbr < K);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      As[buf][e >> 5][e & 31] = ra[q];
      Bs[buf][e >> 5][e & 31] = rb[q];
    }
  };
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int kb = 0; kb < K; kb += kLt, buf ^= 1) {
    const bool next = kb + kLt < K;
    if (next) load(kb + kLt);
#pragma unroll 8
    for (int k = 0; k < kLt; ++k) {
      const double a0 = As[buf][ty * 2][k], a1 = As[buf][ty * 2 + 1][k];
      const double b0 = Bs[buf][k][tx * 2], b1 = Bs[buf][k][tx * 2 + 1];
      acc[0][0] = fma(a0, b0, acc[0][0]);
      acc[0][1] = fma(a0, b1, acc[0][1]);
      acc[1][0] = fma(a1, b0, acc[1][0]);
      acc[1][1] = fma(a1, b1, acc[1][1]);
    }
    if (next) store(buf ^ 1);
    __syncthreads();
  }
  const double alpha = stage == 0 ? 1.0 : -1.0;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int row = r0 + ty * 2 + p, col = c0 + tx * 2 + q;
      if (row < bot_len) out[int64_t(bot0 + row) * ldc + i0 + col] = alpha * acc[p][q];
    }
}

// WT = W^T (lower triangle of W, R1 x R1)
__global__ void transpose_lower_kernel(const double* __restrict__ W, int64_t ldc, int R1, double* __restrict__ WT) {
  __shared__ double tileb[32][33];
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int k = ty; k < 32; k += 8) {
    const int i = bi + k, j = bj + tx;
    tileb[k][tx] = (i < R1 && j < R1 && j <= i) ? W[int64_t(i) * ldc + j] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int j = bj + k, i = bi + tx;  // WT[j][i] = W[i][j]
    if (i < R1 && j < R1) WT[int64_t(j) * ldc + i] = tileb[tx][k];
  }
}

// ---------------------------------------------------------------- apply
// g = w / L ; part[blk][a] = sum_{rows of this block} U_ia g_i.  Thread t owns
// the columns a = t + 256 q (R1 <= 1024) and reads eight rows of each per
// step, all loads issued before any is used (columns past r read column
// r - 1 and are dropped), so enough bytes are in flight to stream F.
// (Workgroup blk of the pass; the body also serves the batched PCG steps.)
template <int NQ>  // NQ = ceil(R1 / 256)
__device__ __forceinline__ void wood_gt_body(const float* __restrict__ F, int64_t n, int r, int64_t ldf, int R1,
                                             const double* __restrict__ L, const double* __restrict__ w,
                                             double* __restrict__ g, int64_t chunk, double* __restrict__ part,
                                             int blk) {
  constexpr int RU = 8;  // rows per step
  constexpr int nq = NQ;
  __shared__ double gs[kGtStage];
  const int64_t i0 = int64_t(blk) * chunk;
  const int64_t i1 = min(n, i0 + chunk);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // column a = tid + 256 q
  int col[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) col[q] = min(int(threadIdx.x) + 256 * q, max(r - 1, 0));
  for (int64_t sb = i0; sb < i1; sb += kGtStage) {
    const int cnt = int(min<int64_t>(kGtStage, i1 - sb));
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += 256) {
      const double gi = w[sb + k] / L[sb + k];
      g[sb + k] = gi;
      gs[k] = gi;
    }
    __syncthreads();
    double s[4][2];
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q][0] = s[q][1] = 0.0;
    if (r > 0) {  // the same in every lane; an empty factor (F may be null) is never read
      const float* base = F + sb * ldf;
      int k = 0;
      for (; k + RU <= cnt; k += RU) {
        float f[4][RU];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < nq)
#pragma unroll
            for (int u = 0; u < RU; ++u) f[q][u] = base[int64_t(k + u) * ldf + col[q]];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < nq)
#pragma unroll
            for (int u = 0; u < RU; ++u) s[q][u & 1] = fma(double(f[q][u]), gs[k + u], s[q][u & 1]);
      }
      for (; k < cnt; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < nq) s[q][0] = fma(double(base[int64_t(k) * ldf + col[q]]), gs[k], s[q][0]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = threadIdx.x + 256 * q;
      if (a < r) {
        acc[q] += s[q][0] + s[q][1];
      } else if (a == r) {
        double t = 0.0;
        for (int k = 0; k < cnt; ++k) t += gs[k];
        acc[q] += t;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = threadIdx.x + 256 * q;
    if (a < R1) part[int64_t(blk) * R1 + a] = acc[q];
  }
}

template <int NQ>
__global__ __launch_bounds__(256) void wood_gt_kernel(const float* __restrict__ F, int64_t n, int r,
                                                      int64_t ldf, int R1, const double* __restrict__ L,
                                                      const double* __restrict__ w, double* __restrict__ g,
                                                      int64_t chunk, double* __restrict__ part) {
  wood_gt_body<NQ>(F, n, r, ldf, R1, L, w, g, chunk, part, int(blockIdx.x));
}

// t[a] = sum_b part[b][a]: a block per 64 columns, 16 thread rows split the
// partials, then a fixed-order sum over the 16 rows.
__global__ __launch_bounds__(1024) void wood_treduce_kernel(const double* __restrict__ part, int nblk, int R1,
                                                            double* __restrict__ t) {
  __shared__ double sh[16][65];
  const int ca = threadIdx.x & 63, rb = threadIdx.x >> 6;
  const int a = blockIdx.x * 64 + ca;
  double s0 = 0.0, s1 = 0.0;
  if (a < R1) {
    int b = rb;
    for (; b + 16 < nblk; b += 32) {
      s0 += part[int64_t(b) * R1 + a];
      s1 += part[int64_t(b + 16) * R1 + a];
    }
    for (; b < nblk; b += 16) s0 += part[int64_t(b) * R1 + a];
  }
  sh[rb][ca] = s0 + s1;
  __syncthreads();
  if (rb == 0 && a < R1) {
    double s = 0.0;
    for (int k = 0; k < 16; ++k) s += sh[k][ca];
    t[a] = s;
  }
}

// out[i] = sum_{k in [lo(i), hi(i)]} M[i][k] x[k]  for a triangular M (one wave per row).
template <bool LOWER>
__global__ __launch_bounds__(256) void trmv_kernel(const double* __restrict__ M, int64_t ldm, int R1,
                                                   const double* __restrict__ x, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= R1) return;
  const int lo = LOWER ? 0 : row, hi = LOWER ? row : R1 - 1;
  const double* mr = M + int64_t(row) * ldm;
  double s = 0.0;
  for (int k = lo + lane; k <= hi; k += 64) s = fma(mr[k], x[k], s);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) out[row] = s;
}

// Small cores (R1 <= kFusedCore): t = sum of the wood_gt partials, then
// s = C^{-1} t = W^T (W t), in one workgroup of 1024 threads.  Each of the R1
// columns (and then rows) gets H = 1024 / C threads, C the power of two at or
// above R1; their H partial sums are added in a fixed order through LDS.
__device__ __forceinline__ void core_solve_body(const double* __restrict__ part, int nblk, int R1,
                                                const double* __restrict__ W, const double* __restrict__ WT,
                                                int64_t ldc, double* __restrict__ s) {
  __shared__ double red[1024];
  __shared__ double t[kFusedCore], y[kFusedCore];
  int C = 1;
  while (C < R1) C <<= 1;
  const int H = 1024 / C;
  const int a = threadIdx.x & (C - 1), h = threadIdx.x / C;
  auto gather = [&](double v, double* dst) {  // dst[a] = sum over h of v(a, h), h in order
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < R1) {
      double sum = 0.0;
      for (int k = 0; k < H; ++k) sum += red[k * C + threadIdx.x];
      dst[threadIdx.x] = sum;
    }
    __syncthreads();
  };
  double acc = 0.0;
  if (a < R1)
    for (int b = h; b < nblk; b += H) acc += part[int64_t(b) * R1 + a];
  gather(acc, t);
  // y = W t (W lower triangular): row a, columns k = h, h + H, ... <= a
  acc = 0.0;
  if (a < R1) {
    const double* w = W + int64_t(a) * ldc;
    for (int k = h; k <= a; k += H) acc = fma(w[k], t[k], acc);
  }
  gather(acc, y);
  // s = W^T y (WT upper triangular): row a, columns k >= a
  acc = 0.0;
  if (a < R1) {
    const double* w = WT + int64_t(a) * ldc;
    for (int k = a + h; k < R1; k += H) acc = fma(w[k], y[k], acc);
  }
  gather(acc, t);
  if (threadIdx.x < R1) s[threadIdx.x] = t[threadIdx.x];
}

__global__ __launch_bounds__(1024) void core_solve_kernel(const double* __restrict__ part, int nblk, int R1,
                                                          const double* __restrict__ W,
                                                          const double* __restrict__ WT, int64_t ldc,
                                                          double* __restrict__ s) {
  core_solve_body(part, nblk, R1, W, WT, ldc, s);
}

// out_i = g_i - (Fs_i + s_r) / L_i ; with dot_with, the sum of dot_with . out
// (one workgroup up to kOneBlockN rows, else partials for reduce_finalize)
// (Block blk of a grid of nblk; the body also serves the batched PCG steps.)
__device__ __forceinline__ void wood_out_body(int64_t n, int r, const double* __restrict__ L,
                                              const double* __restrict__ g, const double* __restrict__ Fs,
                                              const double* __restrict__ s, double* __restrict__ out,
                                              const double* __restrict__ dot_with, double* __restrict__ partials,
                                              double* __restrict__ dot_out, int blk, int nblk) {
  const double sr = s[r];
  double acc[1] = {0.0};
  for (int64_t i = blk * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(nblk) * blockDim.x) {
    const double fs = r > 0 ? Fs[i] : 0.0;
    const double o = g[i] - (fs + sr) / L[i];
    out[i] = o;
    if (dot_with) acc[0] = fma(o, dot_with[i], acc[0]);
  }
  if (dot_with) block_sums_at<1>(acc, partials, dot_out, blk, nblk);
}

__global__ __launch_bounds__(1024) void wood_out_kernel(int64_t n, int r, const double* __restrict__ L,
                                                       const double* __restrict__ g, const double* __restrict__ Fs,
                                                       const double* __restrict__ s, double* __restrict__ out,
                                                       const double* __restrict__ dot_with,
                                                       double* __restrict__ partials, double* __restrict__ dot_out) {
  wood_out_body(n, r, L, g, Fs, s, out, dot_with, partials, dot_out, int(blockIdx.x), int(gridDim.x));
}

// One workgroup (n <= kOneBlockN): wood_out with its dot product, then PCG's
// direction update p = out + beta p (beta = the new dot over sc[rz_old]),
// p32, sum(p) -- the same per-thread order and block sums as wood_out_kernel
// followed by pcg_p_kernel.
__device__ __forceinline__ void wood_out_p_one_body(int64_t n, int r, const double* __restrict__ L,
                                                    const double* __restrict__ g, const double* __restrict__ Fs,
                                                    const double* __restrict__ s, double* __restrict__ out,
                                                    const double* __restrict__ dot_with, double* sc, int rz_old,
                                                    int rz_new, int sump, int first, double* __restrict__ p,
                                                    float* __restrict__ p32) {
  const double sr = s[r];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double fs = r > 0 ? Fs[i] : 0.0;
    const double o = g[i] - (fs + sr) / L[i];
    out[i] = o;
    acc = fma(o, dot_with[i], acc);
  }
  const double rz = block_sum_all(acc);
  if (threadIdx.x == 0) sc[rz_new] = rz;
  const double beta = first ? 0.0 : rz / sc[rz_old];
  acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {  // out[i] was written by this thread
    const double pi = first ? out[i] : fma(beta, p[i], out[i]);
    p[i] = pi;
    if (p32) p32[i] = float(pi);
    acc += pi;
  }
  const double sum = block_sum_all(acc);
  if (threadIdx.x == 0) sc[sump] = sum;
}

__global__ __launch_bounds__(1024) void wood_out_p_one_kernel(int64_t n, int r, const double* __restrict__ L,
                                                             const double* __restrict__ g,
                                                             const double* __restrict__ Fs,
                                                             const double* __restrict__ s, double* __restrict__ out,
                                                             const double* __restrict__ dot_with, double* sc,
                                                             int rz_old, int rz_new, int sump, int first,
                                                             double* __restrict__ p, float* __restrict__ p32) {
  wood_out_p_one_body(n, r, L, g, Fs, s, out, dot_with, sc, rz_old, rz_new, sump, first, p, p32);
}

// ---------------------------------------------------------------- batched PCG steps
// The bodies above, one fit per workgroup (core, output) or per range of
// workgroups (F^T g); zz = P^{-1} r with r as dot_with, then the direction update.
__global__ __launch_bounds__(256) void wood_gt_steps_kernel(const PcgStepDesc* __restrict__ d,
                                                            const int* __restrict__ first, int nf) {
  const int f = step_of_block(first, nf, int(blockIdx.x));
  const PcgStepDesc& e = d[f];
  wood_gt_body<1>(e.F, e.n, e.rank, e.ldf, e.R1, e.Lw, e.r, e.g, e.chunk, e.part, int(blockIdx.x) - first[f]);
}

__global__ __launch_bounds__(1024) void core_solve_steps_kernel(const PcgStepDesc* __restrict__ d) {
  const PcgStepDesc& e = d[blockIdx.x];
  core_solve_body(e.part, e.nblk, e.R1, e.W, e.WT, e.ldc, e.s);
}

__global__ __launch_bounds__(1024) void wood_out_p_steps_kernel(const PcgStepDesc* __restrict__ d) {
  const PcgStepDesc& e = d[blockIdx.x];
  wood_out_p_one_body(e.n, e.rank, e.Lw, e.g, e.Fs, e.s, e.zz, e.r, e.sc, e.rz, e.rz_new, e.sump, 0, e.p, e.p32);
  if (e.status) {  // the fit's host thread reads these, then resumes the fit
    __syncthreads();  // every thread's part of the step is written
    if (threadIdx.x == 0) {
      __threadfence_system();
      e.status[0] = e.sc[e.pq];
      e.status[1] = e.sc[e.rr];
      __threadfence_system();
      *static_cast<volatile double*>(e.status + 2) = 1.0;
    }
  }
}

void launch_wood_gt_steps(const PcgStepDesc* d, const int* gt_first, int nf, int total, hipStream_t st) {
  if (nf <= 0 || total <= 0) return;
  wood_gt_steps_kernel<<<total, 256, 0, st>>>(d, gt_first, nf);
  KQR_LAUNCH_CHECK();
}

void launch_core_solve_steps(const PcgStepDesc* d, int nf, hipStream_t st) {
  if (nf <= 0) return;
  core_solve_steps_kernel<<<nf, 1024, 0, st>>>(d);
  KQR_LAUNCH_CHECK();
}

// Several workgroups per fit: zz = P^{-1} r and the partials of r . zz.
__global__ __launch_bounds__(256) void wood_out_steps_kernel(const PcgStepDesc* __restrict__ d,
                                                             const int* __restrict__ first, int nf) {
  const int f = step_of_block(first, nf, int(blockIdx.x));
  const PcgStepDesc& e = d[f];
  wood_out_body(e.n, e.rank, e.Lw, e.g, e.Fs, e.s, e.zz, e.r, e.partials, e.sc + e.rz_new, int(blockIdx.x) - first[f],
                e.nred);
}

void launch_wood_out_steps(const PcgStepDesc* d, const int* first, int nf, int total, hipStream_t st) {
  if (nf <= 0 || total <= 0) return;
  wood_out_steps_kernel<<<total, kRedThreads, 0, st>>>(d, first, nf);
  KQR_LAUNCH_CHECK();
}

void launch_wood_out_p_steps(const PcgStepDesc* d, int nf, hipStream_t st) {
  if (nf <= 0) return;
  wood_out_p_steps_kernel<<<nf, kOneBlockThreads, 0, st>>>(d);
  KQR_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- class
Woodbury::Woodbury(const float* F, int64_t n, int64_t r, int64_t ldf)
    : F_(F), n_(n), r_(r), ldf_(ldf), R1_(r + 1) {
  if (R1_ > 1024) fail(KQR_EINVAL, "preconditioner rank %lld exceeds 1023", (long long)r);
  ldc_ = R1_;
  const size_t core = size_t(R1_) * ldc_ * sizeof(double);
  C_.alloc(core);
  W_.alloc(core);
  WT_.alloc(core);
  T_.alloc(core);
  const int nt = int((R1_ + kT - 1) / kT);
  const int ntile = nt * (nt + 1) / 2;
  nsplit_ = std::max(1, std::min(32, 1024 / ntile));
  const size_t syrk_part = size_t(nsplit_) * ntile * kT * kT;
  const size_t gt_part = size_t(kGtBlocks) * R1_;
  part_.alloc(std::max(syrk_part, gt_part) * sizeof(double));
  g_.alloc(size_t(std::max<int64_t>(n, 1)) * sizeof(double));
  Fs_.alloc(size_t(std::max<int64_t>(n, 1)) * sizeof(double));
  t_.alloc(size_t(R1_) * sizeof(double));
  y_.alloc(size_t(R1_) * sizeof(double));
  s_.alloc(size_t(R1_) * sizeof(double));
  flag_.alloc(4 * sizeof(int));
}

void Woodbury::syrk(const double* L, const int* idx, int64_t nrows, double* G, double alpha, double beta,
                    double diag_r, double diag_last, double* out, hipStream_t st) {
  const int R1 = int(R1_);
  const int nt = (R1 + kT - 1) / kT;
  const int ntile = nt * (nt + 1) / 2;
  int nsplit = 0;
  if (nrows > 0) {
    nsplit = nsplit_;
    if (nrows < int64_t(nsplit) * kSubRows) nsplit = int(std::max<int64_t>(1, (nrows + kSubRows - 1) / kSubRows));
    int64_t chunk = (nrows + nsplit - 1) / nsplit;
    chunk = std::max<int64_t>(kSubRows, (chunk + kSubRows - 1) / kSubRows * kSubRows);
    nsplit = int(std::max<int64_t>(1, (nrows + chunk - 1) / chunk));
    syrk_kernel<<<dim3(ntile, nsplit), 256, 0, st>>>(F_, nrows, int(r_), ldf_, L, idx, ntile, chunk,
                                                     part_.as<double>());
    KQR_LAUNCH_CHECK();
  }
  syrk_combine_kernel<<<ntile, 256, 0, st>>>(part_.as<double>(), nsplit, ntile, int(r_), R1, diag_r, diag_last, G,
                                             alpha, beta, out, ldc_);
  KQR_LAUNCH_CHECK();
}

void spd_factor_inverse(double* C, int64_t ldc, int R1, double* W, double* WT, double* T, int* flag, hipStream_t st) {
  KQR_CHECK_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  for (int kb = 0; kb < R1; kb += kNb) {
    const int nb = std::min(kNb, R1 - kb);
    chol_diag_kernel<<<1, 64, 0, st>>>(C, ldc, kb, nb, flag);
    KQR_LAUNCH_CHECK();
    const int rest = R1 - kb - nb;
    if (rest > 0) {
      chol_panel_kernel<<<(rest + 3) / 4, 256, 0, st>>>(C, ldc, kb, nb, R1);
      KQR_LAUNCH_CHECK();
      const int mt = (rest + kLt - 1) / kLt;
      chol_update_kernel<<<mt * (mt + 1) / 2, 256, 0, st>>>(C, ldc, kb, nb, R1);
      KQR_LAUNCH_CHECK();
    }
  }
  // W = Lc^{-1}: diagonal blocks, then doubling levels
  KQR_CHECK_HIP(hipMemsetAsync(W, 0, size_t(R1) * ldc * sizeof(double), st));
  const int nib = (R1 + kNb - 1) / kNb;
  trinv_diag_kernel<<<nib, 64, 0, st>>>(C, ldc, R1, W);
  KQR_LAUNCH_CHECK();
  for (int s = kNb; s < R1; s *= 2) {
    const int pairs = (R1 + 2 * s - 1) / (2 * s);
    const int tiles = (s / kLt) * (s / kLt);
    for (int stage = 0; stage < 2; ++stage) {
      double* out = stage == 0 ? T : W;
      trinv_level_kernel<<<pairs * tiles, 256, 0, st>>>(C, W, T, out, ldc, R1, s, stage, tiles);
      KQR_LAUNCH_CHECK();
    }
  }
  transpose_lower_kernel<<<dim3((R1 + 31) / 32, (R1 + 31) / 32), 256, 0, st>>>(W, ldc, R1, WT);
  KQR_LAUNCH_CHECK();
}

int64_t index_list(const uint8_t* S, int64_t n, int* idx, int* cnt, hipStream_t st) {
  constexpr int nblk = 256;
  const int64_t chunk = (n + nblk - 1) / nblk;
  flag_count_kernel<<<nblk, 256, 0, st>>>(S, n, chunk, cnt);
  KQR_LAUNCH_CHECK();
  flag_scan_kernel<<<1, 64, 0, st>>>(cnt, nblk, cnt + nblk);
  KQR_LAUNCH_CHECK();
  flag_scatter_kernel<<<nblk, 64, 0, st>>>(S, n, chunk, cnt, idx);
  KQR_LAUNCH_CHECK();
  int m = 0;
  KQR_CHECK_HIP(hipMemcpyAsync(&m, cnt + nblk, sizeof(int), hipMemcpyDeviceToHost, st));
  KQR_CHECK_HIP(hipStreamSynchronize(st));
  return m;
}

void spd_solve(const double* W, const double* WT, int64_t ldc, int R1, const double* t, double* y, double* s,
               hipStream_t st) {
  trmv_kernel<true><<<(R1 + 3) / 4, 256, 0, st>>>(W, ldc, R1, t, y);
  KQR_LAUNCH_CHECK();
  trmv_kernel<false><<<(R1 + 3) / 4, 256, 0, st>>>(WT, ldc, R1, y, s);
  KQR_LAUNCH_CHECK();
}

namespace {
std::atomic<int> g_force_skip{0}, g_force_count{0};
}  // namespace

void set_forced_core_breakdowns(int skip, int count) {
  g_force_skip.store(std::max(skip, 0));
  g_force_count.store(std::max(count, 0));
}

Co<bool> Woodbury::factor(Exec& ex) {
  spd_factor_inverse(C_.as<double>(), ldc_, int(R1_), W_.as<double>(), WT_.as<double>(), T_.as<double>(),
                     flag_.as<int>(), ex.st);
  int flag = 1;
  co_await read_back(ex, flag_.ptr, sizeof(int), &flag);
  if (g_force_count.load() > 0) {  // test hook: report a breakdown of a factorisation that ran normally
    if (g_force_skip.load() > 0) g_force_skip.fetch_sub(1);
    else if (g_force_count.fetch_sub(1) > 0) flag = 1;
  }
  co_return flag == 0;
}

Co<bool> Woodbury::build(const double* L, double c, Exec& ex) {
  L_ = L;
  syrk(L, nullptr, n_, nullptr, 0.0, 1.0, 1.0, 1.0 / c, C_.as<double>(), ex.st);
  co_return co_await factor(ex);
}

void Woodbury::prepare_gram(hipStream_t st) {
  if (G_.ptr) return;
  G_.alloc(size_t(R1_) * ldc_ * sizeof(double));
  syrk(nullptr, nullptr, n_, nullptr, 0.0, 1.0, 0.0, 0.0, G_.as<double>(), st);
}

Co<bool> Woodbury::build_scaled_identity(const double* L, double l, double c, Exec& ex, double shrink) {
  const hipStream_t st = ex.st;
  prepare_gram(st);
  L_ = L;
  syrk(nullptr, nullptr, 0, G_.as<double>(), 1.0 / l, 0.0, shrink, shrink / c, C_.as<double>(), st);
  co_return co_await factor(ex);
}

Co<bool> Woodbury::build_two_level(const double* L, const uint8_t* S, double l_in, double l_out, double c,
                                   Exec& ex) {
  const hipStream_t st = ex.st;
  L_ = L;
  const int64_t n = n_;
  constexpr int nblk = 256;
  const int64_t chunk = (n + nblk - 1) / nblk;
  if (!idx_.ptr) {
    idx_.alloc(size_t(std::max<int64_t>(n, 1)) * sizeof(int));
    cnt_.alloc((nblk + 1) * sizeof(int));
  }
  flag_count_kernel<<<nblk, 256, 0, st>>>(S, n, chunk, cnt_.as<int>());
  KQR_LAUNCH_CHECK();
  flag_scan_kernel<<<1, 64, 0, st>>>(cnt_.as<int>(), nblk, cnt_.as<int>() + nblk);
  KQR_LAUNCH_CHECK();
  int m32 = 0;
  co_await read_back(ex, cnt_.as<int>() + nblk, sizeof(int), &m32);
  const int64_t m = m32;
  if (m > n / 2) {  // the interior is most of the data: one weighted pass is cheaper
    syrk(L, nullptr, n, nullptr, 0.0, 1.0, 1.0, 1.0 / c, C_.as<double>(), st);
    co_return co_await factor(ex);
  }
  prepare_gram(st);
  flag_scatter_kernel<<<nblk, 64, 0, st>>>(S, n, chunk, cnt_.as<int>(), idx_.as<int>());
  KQR_LAUNCH_CHECK();
  // C = diag(I, 1/c) + G_all / l_out + (1/l_in - 1/l_out) U_E^T U_E
  syrk(nullptr, idx_.as<int>(), m, G_.as<double>(), 1.0 / l_out, 1.0 / l_in - 1.0 / l_out, 1.0, 1.0 / c,
       C_.as<double>(), st);
  co_return co_await factor(ex);
}

// Workgroups of the U^T g pass: 64 rows of F each, at most kGtBlocks.
static int gt_blocks(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>(kGtBlocks, (n + 63) / 64))); }

int pcg_step_gt_blocks(const PcgStepDesc& d) { return d.nblk; }

bool Woodbury::step_desc(PcgStepDesc& d) const {
  if (R1_ > kFusedCore || (r_ > 0 && (ldf_ & 3))) return false;
  const int nblk = gt_blocks(n_);
  d.Lw = L_;
  d.F = F_;
  d.ldf = ldf_;
  d.rank = int(r_);
  d.R1 = int(R1_);
  d.nblk = nblk;
  d.chunk = (n_ + nblk - 1) / nblk;
  d.g = g_.as<double>();
  d.part = part_.as<double>();
  d.W = W_.as<double>();
  d.WT = WT_.as<double>();
  d.ldc = ldc_;
  d.s = s_.as<double>();
  d.Fs = Fs_.as<double>();
  return true;
}

void Woodbury::apply(const double* w, double* out, const double* dot_with, double* dot_out, Workspace& ws,
                     hipStream_t st, const PUpdate* up) {
  const int R1 = int(R1_);
  const int nblk = gt_blocks(n_);
  const int64_t chunk = (n_ + nblk - 1) / nblk;
  switch ((R1 + 255) / 256) {
    case 1: wood_gt_kernel<1><<<nblk, 256, 0, st>>>(F_, n_, int(r_), ldf_, R1, L_, w, g_.as<double>(), chunk,
                                                    part_.as<double>()); break;
    case 2: wood_gt_kernel<2><<<nblk, 256, 0, st>>>(F_, n_, int(r_), ldf_, R1, L_, w, g_.as<double>(), chunk,
                                                    part_.as<double>()); break;
    case 3: wood_gt_kernel<3><<<nblk, 256, 0, st>>>(F_, n_, int(r_), ldf_, R1, L_, w, g_.as<double>(), chunk,
                                                    part_.as<double>()); break;
    default: wood_gt_kernel<4><<<nblk, 256, 0, st>>>(F_, n_, int(r_), ldf_, R1, L_, w, g_.as<double>(), chunk,
                                                     part_.as<double>()); break;
  }
  KQR_LAUNCH_CHECK();
  if (R1 <= kFusedCore) {
    core_solve_kernel<<<1, 1024, 0, st>>>(part_.as<double>(), nblk, R1, W_.as<double>(), WT_.as<double>(), ldc_,
                                         s_.as<double>());
    KQR_LAUNCH_CHECK();
  } else {
    wood_treduce_kernel<<<(R1 + 63) / 64, 1024, 0, st>>>(part_.as<double>(), nblk, R1, t_.as<double>());
    KQR_LAUNCH_CHECK();
    spd_solve(W_.as<double>(), WT_.as<double>(), ldc_, R1, t_.as<double>(), y_.as<double>(), s_.as<double>(), st);
  }
  if (r_ > 0) gemv_skinny(F_, ldf_, n_, r_, s_.as<double>(), Fs_.as<double>(), st);
  if (up && dot_with && n_ <= kOneBlockN) {
    wood_out_p_one_kernel<<<1, kOneBlockThreads, 0, st>>>(n_, int(r_), L_, g_.as<double>(), Fs_.as<double>(),
                                                          s_.as<double>(), out, dot_with, up->sc, up->rz_old,
                                                          up->rz_new, up->sump, up->first ? 1 : 0, up->p, up->p32);
    KQR_LAUNCH_CHECK();
    return;
  }
  const RedShape g = red_shape(n_);
  wood_out_kernel<<<g.blocks, g.threads, 0, st>>>(n_, int(r_), L_, g_.as<double>(), Fs_.as<double>(),
                                                  s_.as<double>(), out, dot_with, ws.partials, dot_out);
  KQR_LAUNCH_CHECK();
  if (dot_with && g.blocks > 1) reduce_finalize(ws.partials, int(g.blocks), 1, dot_out, st);
  if (up)
    pcg_update_p(n_, out, up->p, up->p32, up->sc, up->rz_old, up->rz_new, up->first, ws, up->sc + up->sump, st);
}

}  // namespace kqr
