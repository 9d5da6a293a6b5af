// Implicit gradient of a validation check loss with respect to log(gamma) and
// log(lambda) (not in the paper; derived from the KKT system of the dual (1.3)).
//
// At a solution with index sets R (alpha = tau), L (alpha = tau - 1) and the
// interior E, (alpha_E, beta) solve the bordered system
//     [K_EE/lambda 1; 1^T 0][alpha_E; beta] = [y_E - K_EN alpha_N/lambda; -1^T alpha_N].
// With the partition locally constant, differentiating it gives, for the
// validation loss J = rho_tau(y' - beta - K' alpha/lambda) (K' = K(X', X)),
//     dJ/dlog(lambda) =  mu_E^T (K alpha)_E/lambda - g^T K' alpha/lambda,
//     dJ/dlog(gamma)  = gamma [mu_E^T ((D o K) alpha)_E - g^T (D' o K') alpha]/lambda,
// where g = -rho_tau'(r') and [K_EE/lambda 1; 1^T 0][mu_E; mu_beta] =
// [K'_E^T g/lambda; 1^T g] (d/dlog gamma of exp(-gamma d) is -gamma d exp(-gamma d)).
// Both bordered systems are solved through the FP64 Cholesky of K_EE:
// a = K_EE^{-1} h, b = K_EE^{-1} 1, mu_beta = (lambda 1^T a - h_beta)/(lambda 1^T b),
// mu_E = lambda (a - mu_beta b).
//
// The gradient is sensitive to the conditioning of K_EE, so every kernel
// entry here is formed in FP64 from the FP32 inputs by direct differences
// (no norm expansion), with FP64 products and sums.
//
// The fitted iterate is first polished: E = {|z_i| <= thr} from the final
// multipliers z, alpha_N at its bound, (alpha_E, beta) from the bordered
// system; the polish is kept when alpha_E lies in the box and the residual
// signs agree with the partition.
#include "adjoint.h"

#include <cmath>
#include <cstring>

namespace kqr {

// ----------------------------------------------------------------- FP64 kernel entries
template <int PMAX, bool LAP>
__device__ __forceinline__ double dist64(const double* xi, const double* xj) {
  double d = 0.0;
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    const double t = xi[k] - xj[k];
    d = LAP ? d + fabs(t) : fma(t, t, d);
  }
  return d;
}

constexpr int kF64Tile = 32;

// part[slice][i] = sum over the slice's columns j of e(i, j) v_j with
// e = exp(-gamma d) (DK: d exp(-gamma d)); one thread per row, column tiles
// of Xc staged in LDS as FP64.
template <int PMAX, bool LAP, bool DK>
__global__ __launch_bounds__(256) void kapply64_kernel(const float* __restrict__ Xr, int64_t nr,
                                                       const float* __restrict__ Xc, int64_t nc, int p, double gamma,
                                                       const double* __restrict__ v, int64_t cols_per_slice,
                                                       double* __restrict__ part) {
  __shared__ double xs[kF64Tile][PMAX];
  __shared__ double vs[kF64Tile];
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const bool row_ok = i < nr;
  double xi[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) xi[k] = (row_ok && k < p) ? double(Xr[i * p + k]) : 0.0;
  const int64_t c0 = int64_t(blockIdx.y) * cols_per_slice;
  const int64_t c1 = min(nc, c0 + cols_per_slice);
  double acc = 0.0;
  for (int64_t jb = c0; jb < c1; jb += kF64Tile) {
    const int cnt = int(min<int64_t>(kF64Tile, c1 - jb));
    __syncthreads();
    for (int t = threadIdx.x; t < kF64Tile * PMAX; t += 256) {
      const int jj = t / PMAX, k = t % PMAX;
      xs[jj][k] = (jj < cnt && k < p) ? double(Xc[(jb + jj) * p + k]) : 0.0;
    }
    if (threadIdx.x < kF64Tile) vs[threadIdx.x] = int(threadIdx.x) < cnt ? v[jb + threadIdx.x] : 0.0;
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const double d = dist64<PMAX, LAP>(xi, xs[jj]);
      const double e = exp(-gamma * d);
      acc = fma(DK ? d * e : e, vs[jj], acc);
    }
  }
  if (row_ok) part[int64_t(blockIdx.y) * nr + i] = acc;
}

__global__ void slice_sum_kernel(const double* __restrict__ part, int nslice, int64_t nr, double scale, double shift,
                                 double* __restrict__ u) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= nr) return;
  double s = 0.0;
  for (int k = 0; k < nslice; ++k) s += part[int64_t(k) * nr + i];
  u[i] = shift + scale * s;
}

// lower triangle of K_EE in FP64
template <int PMAX, bool LAP>
__global__ void kee64_kernel(const float* __restrict__ XE, int64_t m, int p, double gamma, double* __restrict__ C,
                             int64_t ldc) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= m * m) return;
  const int64_t a = t / m, b = t % m;
  if (b > a) return;
  double xa[PMAX], xb[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    xa[k] = k < p ? double(XE[a * p + k]) : 0.0;
    xb[k] = k < p ? double(XE[b * p + k]) : 0.0;
  }
  C[a * ldc + b] = exp(-gamma * dist64<PMAX, LAP>(xa, xb));
}

namespace {
inline unsigned blocks_for(int64_t n) { return unsigned((n + 255) / 256); }

template <int PMAX>
void kapply64_p(const float* Xr, int64_t nr, const float* Xc, int64_t nc, int p, KernelSpec ks, const double* v,
                double* u, double scale, double shift, bool dk, hipStream_t st) {
  const int64_t rblk = (nr + 255) / 256;
  int64_t nslice = std::max<int64_t>(1, std::min<int64_t>(2048 / std::max<int64_t>(rblk, 1), (nc + 511) / 512));
  nslice = std::min<int64_t>(nslice, 65535);
  int64_t per = (nc + nslice - 1) / nslice;
  per = (per + kF64Tile - 1) / kF64Tile * kF64Tile;
  nslice = (nc + per - 1) / per;
  DevBuf part(size_t(nslice) * size_t(nr) * sizeof(double));
  const dim3 grid((unsigned)rblk, (unsigned)nslice);
  const bool lap = ks.kind == KQR_LAPLACIAN;
  double* pp = part.as<double>();
  if (lap && dk) kapply64_kernel<PMAX, true, true><<<grid, 256, 0, st>>>(Xr, nr, Xc, nc, p, ks.gamma, v, per, pp);
  else if (lap) kapply64_kernel<PMAX, true, false><<<grid, 256, 0, st>>>(Xr, nr, Xc, nc, p, ks.gamma, v, per, pp);
  else if (dk) kapply64_kernel<PMAX, false, true><<<grid, 256, 0, st>>>(Xr, nr, Xc, nc, p, ks.gamma, v, per, pp);
  else kapply64_kernel<PMAX, false, false><<<grid, 256, 0, st>>>(Xr, nr, Xc, nc, p, ks.gamma, v, per, pp);
  KQR_LAUNCH_CHECK();
  slice_sum_kernel<<<blocks_for(nr), 256, 0, st>>>(pp, int(nslice), nr, scale, shift, u);
  KQR_LAUNCH_CHECK();
  KQR_CHECK_HIP(hipStreamSynchronize(st));  // part is released on return
}

template <int PMAX>
void kee64_p(const float* XE, int64_t m, int p, KernelSpec ks, double* C, hipStream_t st) {
  if (ks.kind == KQR_LAPLACIAN) kee64_kernel<PMAX, true><<<blocks_for(m * m), 256, 0, st>>>(XE, m, p, ks.gamma, C, m);
  else kee64_kernel<PMAX, false><<<blocks_for(m * m), 256, 0, st>>>(XE, m, p, ks.gamma, C, m);
  KQR_LAUNCH_CHECK();
}

#define KQR_ADJ_DISPATCH_P(p, FN, ...)                               \
  do {                                                               \
    if ((p) <= 8) FN<8>(__VA_ARGS__);                                \
    else if ((p) <= 16) FN<16>(__VA_ARGS__);                         \
    else if ((p) <= 32) FN<32>(__VA_ARGS__);                         \
    else if ((p) <= 64) FN<64>(__VA_ARGS__);                         \
    else fail(KQR_EINVAL, "feature dimension p=%d exceeds 64", (p)); \
  } while (0)

// u = shift + scale * E(Xr, Xc) v with FP64 entries (E = K, or D o K when dk)
void kapply64(const float* Xr, int64_t nr, const float* Xc, int64_t nc, int p, KernelSpec ks, const double* v,
              double* u, double scale, double shift, bool dk, hipStream_t st) {
  if (nr <= 0) return;
  KQR_ADJ_DISPATCH_P(p, kapply64_p, Xr, nr, Xc, nc, p, ks, v, u, scale, shift, dk, st);
}
}  // namespace

// ----------------------------------------------------------------- small vector kernels
__global__ void gather_rows_kernel(const float* __restrict__ X, int p, const int* __restrict__ idx, int64_t m,
                                   float* __restrict__ XE) {
  const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (t >= m * p) return;
  const int64_t a = t / p;
  const int k = int(t % p);
  XE[t] = X[int64_t(idx[a]) * p + k];
}

__global__ void mask_kernel(const double* __restrict__ z, int64_t n, double thr, uint8_t* __restrict__ S) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) S[i] = fabs(z[i]) <= thr ? 1 : 0;
}

// partition state: 0 interior, +1 at tau, -1 at tau - 1
__global__ void state_init_kernel(const double* __restrict__ z, int64_t n, double thr, int8_t* __restrict__ s) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) s[i] = fabs(z[i]) <= thr ? 0 : (z[i] > 0.0 ? 1 : -1);
}

__global__ void mask_from_state_kernel(const int8_t* __restrict__ s, int64_t n, uint8_t* __restrict__ S) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) S[i] = s[i] == 0 ? 1 : 0;
}

// at = alpha on N set to its bound, 0 on E
__global__ void bound_from_state_kernel(const int8_t* __restrict__ s, int64_t n, double tau, double* __restrict__ at) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) at[i] = s[i] == 0 ? 0.0 : (s[i] > 0 ? tau : tau - 1.0);
}

// one active-set move per violator (see polish_check_kernel for the tests)
__global__ void repair_kernel(const double* __restrict__ alpha, const double* __restrict__ y,
                              const double* __restrict__ Ka, int8_t* __restrict__ s, int64_t n, double tau,
                              double beta, double lam, double slack_a, double slack_z) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int8_t si = s[i];
  if (si == 0) {
    if (alpha[i] > tau + slack_a) s[i] = 1;
    else if (alpha[i] < tau - 1.0 - slack_a) s[i] = -1;
  } else {
    const double r = y[i] - beta - Ka[i] / lam;
    if ((si > 0 && r < -slack_z) || (si < 0 && r > slack_z)) s[i] = 0;
  }
}

// alpha[idx[a]] = aE[a]
__global__ void scatter_vec_kernel(const double* __restrict__ aE, const int* __restrict__ idx, int64_t m,
                                   double* __restrict__ alpha) {
  const int64_t a = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (a < m) alpha[idx[a]] = aE[a];
}

// q[a] = y[idx[a]] - u[a] / lambda
__global__ void rhs_e_kernel(const double* __restrict__ y, const int* __restrict__ idx, const double* __restrict__ u,
                             int64_t m, double lam, double* __restrict__ q) {
  const int64_t a = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (a < m) q[a] = y[idx[a]] - u[a] / lam;
}

// out = lambda (a - c b)
__global__ void combine_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t m, double lam,
                               double c, double* __restrict__ out) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < m) out[i] = lam * (a[i] - c * b[i]);
}

// box / sign check of a polished point: an interior alpha must lie in the box,
// alpha = tau needs a residual >= 0 and alpha = tau - 1 one <= 0 (both up to
// slack); partials [#violations]
__global__ __launch_bounds__(256) void polish_check_kernel(const double* __restrict__ alpha, const double* __restrict__ y,
                                                           const double* __restrict__ Ka, const int8_t* __restrict__ s,
                                                           int64_t n, double tau, double beta, double lam,
                                                           double slack_a, double slack_z, double* __restrict__ part) {
  __shared__ double sh[4];
  double bad = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    if (s[i] == 0) {
      if (alpha[i] < tau - 1.0 - slack_a || alpha[i] > tau + slack_a) bad += 1.0;
    } else {
      const double zz = y[i] - beta - Ka[i] / lam;
      if (s[i] > 0 && zz < -slack_z) bad += 1.0;
      if (s[i] < 0 && zz > slack_z) bad += 1.0;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) bad += __shfl_xor(bad, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = bad;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ void clip_kernel(double* __restrict__ a, const uint8_t* __restrict__ S, int64_t n, double tau) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n && S[i]) a[i] = fmin(fmax(a[i], tau - 1.0), tau);
}

// validation: r = yv - f ; g = -tau (r > 0) else 1 - tau ; partials [rho_tau(r), sum g]
__global__ __launch_bounds__(256) void val_kernel(const double* __restrict__ yv, const double* __restrict__ f,
                                                  int64_t nv, double tau, double* __restrict__ g,
                                                  double* __restrict__ part) {
  __shared__ double sh[2][4];
  double loss = 0.0, sg = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < nv; i += int64_t(gridDim.x) * blockDim.x) {
    const double r = yv[i] - f[i];
    loss += r > 0.0 ? tau * r : -(1.0 - tau) * r;
    const double gi = r > 0.0 ? -tau : 1.0 - tau;
    g[i] = gi;
    sg += gi;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    loss += __shfl_xor(loss, off);
    sg += __shfl_xor(sg, off);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = loss;
    sh[1][threadIdx.x >> 6] = sg;
  }
  __syncthreads();
  if (threadIdx.x < 2)
    part[blockIdx.x * 2 + threadIdx.x] =
        ((sh[threadIdx.x][0] + sh[threadIdx.x][1]) + sh[threadIdx.x][2]) + sh[threadIdx.x][3];
}

namespace {
// Deterministic device sums read back to the host.
struct Dots {
  Workspace ws;
  explicit Dots(hipStream_t st) : ws(st) {}
  DevBuf dev{8 * sizeof(double)};
  // sum(a) when b is null, else a . b
  double run(int64_t n, const double* a, const double* b, hipStream_t st) {
    vec_dots(n, a, b, ws, dev.as<double>(), st);
    double h[3];
    KQR_CHECK_HIP(hipMemcpyAsync(h, dev.ptr, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    return b ? h[1] : h[0];
  }
  double finalize(const double* part, int nq, int q, hipStream_t st) {
    reduce_finalize(part, kRedBlocks, nq, dev.as<double>(), st);
    double h[2];
    KQR_CHECK_HIP(hipMemcpyAsync(h, dev.ptr, size_t(nq) * sizeof(double), hipMemcpyDeviceToHost, st));
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    return h[q];
  }
};

// Dense FP64 factor of K_EE and b = K_EE^{-1} 1 for one interior set.
struct InteriorFactor {
  int64_t m = 0;
  DevBuf XE, C, W, WT, T, flag, tmp, b, ones;
  double b_sum = 0.0;
  // false when K_EE is not positive definite in FP64
  bool build(const float* X, int p, KernelSpec ks, const int* idx, int64_t mm, Dots& dots, hipStream_t st) {
    m = mm;
    XE.alloc(size_t(m) * p * sizeof(float));
    gather_rows_kernel<<<blocks_for(m * p), 256, 0, st>>>(X, p, idx, m, XE.as<float>());
    KQR_LAUNCH_CHECK();
    const size_t mat = size_t(m) * size_t(m) * sizeof(double);
    C.alloc(mat);
    W.alloc(mat);
    WT.alloc(mat);
    T.alloc(mat);
    flag.alloc(sizeof(int));
    tmp.alloc(size_t(m) * sizeof(double));
    b.alloc(size_t(m) * sizeof(double));
    ones.alloc(size_t(m) * sizeof(double));
    KQR_ADJ_DISPATCH_P(p, kee64_p, XE.as<float>(), m, p, ks, C.as<double>(), st);
    spd_factor_inverse(C.as<double>(), m, int(m), W.as<double>(), WT.as<double>(), T.as<double>(), flag.as<int>(), st);
    int fl = 0;
    KQR_CHECK_HIP(hipMemcpyAsync(&fl, flag.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    if (fl != 0) return false;
    fill(m, 1.0, ones.as<double>(), st);
    solve(ones.as<double>(), b.as<double>(), st);
    b_sum = dots.run(m, b.as<double>(), nullptr, st);
    return true;
  }
  void solve(const double* rhs, double* out, hipStream_t st) {
    spd_solve(W.as<double>(), WT.as<double>(), m, int(m), rhs, tmp.as<double>(), out, st);
  }
};
}  // namespace

GradOutcome adjoint_gradient(const float* X, int64_t n, int p, KernelSpec ks, double tau, double lam, double* alpha,
                             double* beta, const double* z, const double* y, const float* Xv, int64_t nv,
                             const double* yv, double tol, hipStream_t st) {
  GradOutcome out;
  DevBuf S(static_cast<size_t>(n)), idx(size_t(n) * sizeof(int)), cnt(257 * sizeof(int));
  DevBuf at(size_t(n) * sizeof(double)), Ka(size_t(n) * sizeof(double));
  DevBuf part(size_t(kRedBlocks) * 2 * sizeof(double)), alpha_try(size_t(n) * sizeof(double));
  Dots dots(st);
  const double ynorm = std::sqrt(dots.run(n, y, y, st));
  InteriorFactor fe;
  DevBuf uE, aE;
  // ---------------- active-set polish
  // Partition from the multipliers (|z_i| <= thr interior, else the bound of
  // z's sign), then primal-dual active-set rounds: solve the bordered system
  // on the partition; an interior coefficient outside the box moves to the
  // bound it crossed, a bound coefficient whose residual has the wrong sign
  // moves to the interior set; stop when nothing moves.
  const double scale = tol * (1.0 + ynorm);
  const double slack_a = 1e-10, slack_z = 1e-9 * (1.0 + ynorm);
  DevBuf state(static_cast<size_t>(n));
  int8_t* s8 = state.as<int8_t>();
  state_init_kernel<<<blocks_for(n), 256, 0, st>>>(z, n, scale, s8);
  KQR_LAUNCH_CHECK();
  double beta_new = *beta;
  for (int round = 0; round < kPolishRounds; ++round) {
    mask_from_state_kernel<<<blocks_for(n), 256, 0, st>>>(s8, n, S.as<uint8_t>());
    KQR_LAUNCH_CHECK();
    const int64_t m = index_list(S.as<uint8_t>(), n, idx.as<int>(), cnt.as<int>(), st);
    out.polish_rounds = round + 1;
    if (m == 0 || m > kAdjointMaxInterior) break;
    if (!fe.build(X, p, ks, idx.as<int>(), m, dots, st)) break;
    uE.alloc(size_t(m) * sizeof(double));
    aE.alloc(size_t(m) * sizeof(double));
    // alpha_N on its bounds: q_E = y_E - (K at)_E / lambda, q_beta = -1^T at
    bound_from_state_kernel<<<blocks_for(n), 256, 0, st>>>(s8, n, tau, at.as<double>());
    KQR_LAUNCH_CHECK();
    kapply64(fe.XE.as<float>(), m, X, n, p, ks, at.as<double>(), uE.as<double>(), 1.0, 0.0, false, st);
    rhs_e_kernel<<<blocks_for(m), 256, 0, st>>>(y, idx.as<int>(), uE.as<double>(), m, lam, uE.as<double>());
    KQR_LAUNCH_CHECK();
    const double q_beta = -dots.run(n, at.as<double>(), nullptr, st);
    fe.solve(uE.as<double>(), aE.as<double>(), st);
    const double a_sum = dots.run(m, aE.as<double>(), nullptr, st);
    const double bt = (lam * a_sum - q_beta) / (lam * fe.b_sum);
    combine_kernel<<<blocks_for(m), 256, 0, st>>>(aE.as<double>(), fe.b.as<double>(), m, lam, bt, aE.as<double>());
    KQR_LAUNCH_CHECK();
    copy(n, at.as<double>(), alpha_try.as<double>(), st);
    scatter_vec_kernel<<<blocks_for(m), 256, 0, st>>>(aE.as<double>(), idx.as<int>(), m, alpha_try.as<double>());
    KQR_LAUNCH_CHECK();
    // box of alpha_E and residual signs on N, with the full K alpha
    kapply64(X, n, X, n, p, ks, alpha_try.as<double>(), Ka.as<double>(), 1.0, 0.0, false, st);
    polish_check_kernel<<<kRedBlocks, 256, 0, st>>>(alpha_try.as<double>(), y, Ka.as<double>(), s8, n, tau, bt, lam,
                                                    slack_a, slack_z, part.as<double>());
    KQR_LAUNCH_CHECK();
    if (dots.finalize(part.as<double>(), 1, 0, st) == 0.0) {
      clip_kernel<<<blocks_for(n), 256, 0, st>>>(alpha_try.as<double>(), S.as<uint8_t>(), n, tau);
      KQR_LAUNCH_CHECK();
      copy(n, alpha_try.as<double>(), alpha, st);
      beta_new = bt;
      out.polished = true;
      break;
    }
    repair_kernel<<<blocks_for(n), 256, 0, st>>>(alpha_try.as<double>(), y, Ka.as<double>(), s8, n, tau, bt, lam,
                                                 slack_a, slack_z);
    KQR_LAUNCH_CHECK();
  }
  if (!out.polished) {  // gradient at the fitted iterate with E = {|z| <= thr}
    mask_kernel<<<blocks_for(n), 256, 0, st>>>(z, n, scale, S.as<uint8_t>());
    KQR_LAUNCH_CHECK();
    const int64_t m = index_list(S.as<uint8_t>(), n, idx.as<int>(), cnt.as<int>(), st);
    if (m == 0) fail(KQR_ENUMERIC, "no interior coefficients: beta is not differentiable");
    if (m > kAdjointMaxInterior)
      fail(KQR_EINVAL, "interior set of %lld points exceeds the dense adjoint limit %lld", (long long)m,
           (long long)kAdjointMaxInterior);
    if (!fe.build(X, p, ks, idx.as<int>(), m, dots, st)) fail(KQR_ENUMERIC, "K_EE is not positive definite in FP64");
    uE.alloc(size_t(m) * sizeof(double));
    aE.alloc(size_t(m) * sizeof(double));
  }
  *beta = beta_new;
  const int64_t m = fe.m;
  out.n_interior = m;
  // ---------------- validation loss and its adjoint
  DevBuf fv(size_t(nv) * sizeof(double)), g(size_t(nv) * sizeof(double));
  kapply64(Xv, nv, X, n, p, ks, alpha, fv.as<double>(), 1.0 / lam, *beta, false, st);
  val_kernel<<<kRedBlocks, 256, 0, st>>>(yv, fv.as<double>(), nv, tau, g.as<double>(), part.as<double>());
  KQR_LAUNCH_CHECK();
  out.J = dots.finalize(part.as<double>(), 2, 0, st);
  const double h_beta = dots.finalize(part.as<double>(), 2, 1, st);
  // mu: h_E = K'_E^T g / lambda (rows of E against the validation points)
  kapply64(fe.XE.as<float>(), m, Xv, nv, p, ks, g.as<double>(), uE.as<double>(), 1.0 / lam, 0.0, false, st);
  fe.solve(uE.as<double>(), aE.as<double>(), st);
  const double a_sum = dots.run(m, aE.as<double>(), nullptr, st);
  const double mu_beta = (lam * a_sum - h_beta) / (lam * fe.b_sum);
  combine_kernel<<<blocks_for(m), 256, 0, st>>>(aE.as<double>(), fe.b.as<double>(), m, lam, mu_beta, aE.as<double>());
  KQR_LAUNCH_CHECK();  // aE = mu_E
  // (K alpha)_E, ((D o K) alpha)_E, K' alpha, (D' o K') alpha
  DevBuf kaE(size_t(m) * sizeof(double)), dkaE(size_t(m) * sizeof(double));
  DevBuf kav(size_t(nv) * sizeof(double)), dkav(size_t(nv) * sizeof(double));
  kapply64(fe.XE.as<float>(), m, X, n, p, ks, alpha, kaE.as<double>(), 1.0, 0.0, false, st);
  kapply64(fe.XE.as<float>(), m, X, n, p, ks, alpha, dkaE.as<double>(), 1.0, 0.0, true, st);
  kapply64(Xv, nv, X, n, p, ks, alpha, kav.as<double>(), 1.0, 0.0, false, st);
  kapply64(Xv, nv, X, n, p, ks, alpha, dkav.as<double>(), 1.0, 0.0, true, st);
  const double muKa = dots.run(m, aE.as<double>(), kaE.as<double>(), st);
  const double muDKa = dots.run(m, aE.as<double>(), dkaE.as<double>(), st);
  const double gKa = dots.run(nv, g.as<double>(), kav.as<double>(), st);
  const double gDKa = dots.run(nv, g.as<double>(), dkav.as<double>(), st);
  out.dlam = (muKa - gKa) / lam;
  out.dgam = ks.gamma * (muDKa - gDKa) / lam;
  return out;
}

}  // namespace kqr
