// Randomly pivoted Cholesky, F = RPCholesky(K, r), K_hat = F F^T (Section 3,
// preconditioner (3.2)), and the rank heuristic of Section 3.
//
// Step i of RPCholesky:
//   s    = first j with sum_{l<=j} d_l > u_i * sum(d)  (pivot ~ residual diagonal)
//   g    = K[:, s] - F[:, :i] F[s, :i]^T
//   F[:, i] = g / sqrt(g_s),  d <- max(d - F[:, i]^2, 0),  d_s <- 0
// Everything stays on the device: the pivot is found by a one-wave scan over
// block sums that the previous step's update kernel produced, the correction
// F[:, :i] F[s, :i]^T is the streamed mat-vec of the K-apply with F as the
// matrix, and the early stop (sum(d) <= 1e-14 tr K) is a device flag, so the
// host synchronises once at the end.
//
// Rank heuristic: r0 = ceil(sqrt n), eigenvalues of F0^T F0, r = smallest index
// with lambda_r <= xi lambda_1.  F0^T F0 is reduced to tridiagonal form by
// Householder reflections in one workgroup (FP64), lambda_1 is found by
// bisection with Sturm counts, and the number of eigenvalues above
// xi lambda_1 by one more Sturm count.
#include "kernel_entry.h"
#include "vec.h"

#include <cmath>
#include <cstring>

namespace kqr {

namespace {
constexpr int kSelBlocks = 256;
}

__global__ __launch_bounds__(256) void rpc_blocksum_kernel(const double* __restrict__ d, int64_t n, int64_t chunk,
                                                           double* __restrict__ bsum) {
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

// One wave.  state[0] = tr K (set at step 0), state[1] = stopped flag.
// Writes piv[step] = pivot, or -1 once the residual trace is negligible.
__global__ __launch_bounds__(64) void rpc_select_kernel(const double* __restrict__ d, int64_t n, int64_t chunk,
                                                        const double* __restrict__ bsum, int nblk, double u, int step,
                                                        int64_t* __restrict__ piv, double* __restrict__ state) {
  const int lane = threadIdx.x;
  // prefix sums of the block sums: lane l owns blocks [PER l, PER l + PER)
  constexpr int PER = kSelBlocks / 64;
  double bs[PER];
  double own = 0.0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = lane * PER + q;
    bs[q] = b < nblk ? bsum[b] : 0.0;
    own += bs[q];
  }
  double incl = own;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  const double total = __shfl(incl, 63);
  bool stop = state[1] != 0.0;
  if (step == 0) stop = false;
  const double tr0 = step == 0 ? total : state[0];
  if (!(total > 1e-14 * tr0)) stop = true;
  int64_t found = -1;
  if (!stop) {
    const double target = u * total;
    // first block whose running sum passes the target
    int mine = -1;
    double before = 0.0;
    double run_b = incl - own;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const double next = run_b + bs[q];
      if (mine < 0 && next > target && bs[q] > 0.0) {
        mine = lane * PER + q;
        before = run_b;
      }
      run_b = next;
    }
    const unsigned long long hitm = __ballot(mine >= 0);
    int bsel = -1;
    double pref_sel = 0.0;
    if (hitm) {
      const int src = __ffsll((long long)hitm) - 1;
      bsel = __shfl(mine, src);
      pref_sel = __shfl(before, src);
    }
    if (bsel >= 0) {
      // scan from the selected block on (a later block only when the rounding
      // of block sums and running sum disagree next to the target)
      double run = pref_sel;
      for (int64_t base = int64_t(bsel) * chunk; base < n && found < 0; base += 64) {
        const int64_t i = base + lane;
        const double di = i < n ? d[i] : 0.0;
        double incl = di;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const double t = __shfl_up(incl, off);
          if (lane >= off) incl += t;
        }
        const bool hit = (i < n) && (run + incl > target) && di > 0.0;
        const unsigned long long m = __ballot(hit);
        if (m) found = base + __ffsll((long long)m) - 1;
        else run += __shfl(incl, 63);
      }
    }
    if (found < 0) {  // u*total rounded to the very end: take the last positive entry
      for (int64_t base = ((n - 1) / 64) * 64; base >= 0 && found < 0; base -= 64) {
        const int64_t i = base + lane;
        const unsigned long long m = __ballot(i < n && d[i] > 0.0);
        if (m) found = base + 63 - __clzll((long long)m);
      }
    }
    if (found < 0) stop = true;
  }
  if (lane == 0) {
    piv[step] = stop ? -1 : found;
    if (step == 0) state[0] = tr0;
    state[1] = stop ? 1.0 : 0.0;
  }
}

// fs[k] = F[s][k] for k < i (FP64 copy of the pivot row of F)
__global__ void rpc_pivrow_kernel(const float* __restrict__ F, int64_t ldf, int i, const int64_t* __restrict__ piv,
                                  int step, double* __restrict__ fs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= i) return;
  const int64_t s = piv[step];
  fs[k] = s >= 0 ? double(F[s * ldf + k]) : 0.0;
}

// g_j = K[s][j] - u_j, F[j][i] = g_j / sqrt(g_s), d_j <- max(d_j - F[j][i]^2, 0),
// d_s <- 0, and the block sums of the new d for the next pivot draw.
__global__ __launch_bounds__(256) void rpc_update_kernel(const KMat km, const float* __restrict__ X,
                                                         const float* __restrict__ q, int p, int lap, float ng,
                                                         float* __restrict__ F, int64_t n, int64_t ldf, int i,
                                                         const int64_t* __restrict__ piv, int step,
                                                         const double* __restrict__ u, double* __restrict__ d,
                                                         int64_t chunk, double* __restrict__ bsum) {
  __shared__ double sh[4];
  const int64_t s = piv[step];
  const int64_t i0 = int64_t(blockIdx.x) * chunk;
  const int64_t i1 = min(n, i0 + chunk);
  double bs = 0.0;
  if (s < 0) {
    for (int64_t j = i0 + threadIdx.x; j < i1; j += 256) {
      F[j * ldf + i] = 0.f;
      bs += d[j];
    }
  } else {
    auto kentry = [&](int64_t j) -> double {
      if (km.K) {
        const size_t off = km.layout == 1 ? pk_offset(s, j, km.ld) : size_t(s * km.ld + j);
        if (km.dtype == KQR_BF16)
          return double(__uint_as_float(uint32_t(static_cast<const uint16_t*>(km.K)[off]) << 16));
        return double(static_cast<const float*>(km.K)[off]);
      }
      float dd = pair_dist_dyn(X + s * p, q ? q[s] : 0.f, X + j * p, q ? q[j] : 0.f, p, lap != 0);
      if (j == s) dd = 0.f;
      return double(kexp2(ng * dd));
    };
    const double gs = kentry(s) - (i > 0 ? u[s] : 0.0);
    const double inv = gs > 0.0 ? 1.0 / sqrt(gs) : 0.0;
    for (int64_t j = i0 + threadIdx.x; j < i1; j += 256) {
      const double g = kentry(j) - (i > 0 ? u[j] : 0.0);
      const double f = g * inv;
      F[j * ldf + i] = float(f);
      const double dj = (j == s) ? 0.0 : fmax(d[j] - f * f, 0.0);
      d[j] = dj;
      bs += dj;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) bs += __shfl_xor(bs, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = bs;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ void rpc_diag_kernel(const KMat km, int64_t n, double* __restrict__ d) {
  const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (j >= n) return;
  if (!km.K) { d[j] = 1.0; return; }  // k(x, x) = exp(0) for both kernels
  const size_t off = km.layout == 1 ? pk_offset(j, j, km.ld) : size_t(j * km.ld + j);
  if (km.dtype == KQR_BF16)
    d[j] = __uint_as_float(uint32_t(static_cast<const uint16_t*>(km.K)[off]) << 16);
  else
    d[j] = static_cast<const float*>(km.K)[off];
}

Co<std::vector<int64_t>> rpcholesky(KMat km, const float* X, const float* sqn, int64_t n, int p,
                                    KernelSpec ks, int64_t rank, const double* uniforms, float* F, int64_t ldf,
                                    Exec& ex) {
  const hipStream_t st = ex.st;
  std::vector<int64_t> pivots;
  if (rank <= 0 || n <= 0) co_return pivots;
  rank = std::min<int64_t>(rank, n);
  if (rank > 1024) fail(KQR_EINVAL, "RPCholesky rank %lld exceeds 1024", (long long)rank);
  DevBuf d(size_t(n) * sizeof(double)), u(size_t(n) * sizeof(double)), fs(1024 * sizeof(double));
  DevBuf bsum(kSelBlocks * sizeof(double)), piv(size_t(rank) * sizeof(int64_t)), state(2 * sizeof(double));
  rpc_diag_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, st>>>(km, n, d.as<double>());
  KQR_LAUNCH_CHECK();
  KQR_CHECK_HIP(hipMemsetAsync(state.ptr, 0, 2 * sizeof(double), st));
  const int64_t chunk = (n + kSelBlocks - 1) / kSelBlocks;
  rpc_blocksum_kernel<<<kSelBlocks, 256, 0, st>>>(d.as<double>(), n, chunk, bsum.as<double>());
  KQR_LAUNCH_CHECK();
  const float ng = -float(ks.gamma) * kLog2e;
  const bool lap = ks.kind == KQR_LAPLACIAN;
  for (int64_t i = 0; i < rank; ++i) {
    rpc_select_kernel<<<1, 64, 0, st>>>(d.as<double>(), n, chunk, bsum.as<double>(), kSelBlocks, uniforms[i],
                                        int(i), piv.as<int64_t>(), state.as<double>());
    KQR_LAUNCH_CHECK();
    if (i > 0) {
      rpc_pivrow_kernel<<<(unsigned)((i + 255) / 256), 256, 0, st>>>(F, ldf, int(i), piv.as<int64_t>(), int(i),
                                                                      fs.as<double>());
      KQR_LAUNCH_CHECK();
      gemv_skinny(F, ldf, n, i, fs.as<double>(), u.as<double>(), st);
    }
    rpc_update_kernel<<<kSelBlocks, 256, 0, st>>>(km, X, lap ? nullptr : sqn, p, lap ? 1 : 0, ng, F, n, ldf, int(i),
                                                  piv.as<int64_t>(), int(i), u.as<double>(), d.as<double>(), chunk,
                                                  bsum.as<double>());
    KQR_LAUNCH_CHECK();
  }
  std::vector<int64_t> h(size_t(rank), -1);
  co_await read_back(ex, piv.ptr, size_t(rank) * sizeof(int64_t), h.data());
  for (int64_t i = 0; i < rank; ++i) {
    if (h[size_t(i)] < 0) break;
    pivots.push_back(h[size_t(i)]);
  }
  co_return pivots;
}

// ================================================================= rank heuristic
// Householder tridiagonalisation of the symmetric m x m matrix whose lower
// triangle is G (ld ldg), in one workgroup; A is m x m scratch.  Writes the
// diagonal dg[m] and the off-diagonal eg[m-1].
__global__ __launch_bounds__(1024) void tridiag_kernel(const double* __restrict__ G, int64_t ldg, int m,
                                                       double* __restrict__ A, double* __restrict__ v,
                                                       double* __restrict__ w, double* __restrict__ dg,
                                                       double* __restrict__ eg) {
  __shared__ double red[32];
  __shared__ double bc[4];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
  auto block_sum = [&](double x) -> double {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    __syncthreads();
    if (lane == 0) red[wid] = x;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red[k];
    return s;
  };
  for (int64_t e = tid; e < int64_t(m) * m; e += nt) {
    const int i = int(e / m), j = int(e % m);
    A[e] = i >= j ? G[int64_t(i) * ldg + j] : G[int64_t(j) * ldg + i];
  }
  __syncthreads();
  for (int k = 0; k + 2 < m; ++k) {
    const int len = m - k - 1;  // trailing size
    double* col = A + int64_t(k + 1) * m + k;  // A[k+1+i][k], stride m
    double part = 0.0;
    for (int i = tid; i < len; i += nt) {
      const double x = col[int64_t(i) * m];
      part = fma(x, x, part);
    }
    const double xx = block_sum(part);
    const double x0 = col[0];
    if (tid == 0) dg[k] = A[int64_t(k) * m + k];
    if (!(xx > 0.0)) {
      if (tid == 0) eg[k] = 0.0;
      __syncthreads();
      continue;
    }
    const double alpha = x0 >= 0.0 ? -sqrt(xx) : sqrt(xx);
    const double vv = 2.0 * (xx - x0 * alpha);  // ||x - alpha e1||^2
    for (int i = tid; i < len; i += nt) v[i] = col[int64_t(i) * m] - (i == 0 ? alpha : 0.0);
    if (tid == 0) eg[k] = alpha;
    __syncthreads();
    // p = (2 / vv) A22 v  (one wave per row)
    const double* A22 = A + int64_t(k + 1) * m + (k + 1);
    for (int i = wid; i < len; i += nw) {
      const double* row = A22 + int64_t(i) * m;
      double s = 0.0;
      for (int j = lane; j < len; j += 64) s = fma(row[j], v[j], s);
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
      if (lane == 0) w[i] = s * (2.0 / vv);
    }
    __syncthreads();
    part = 0.0;
    for (int i = tid; i < len; i += nt) part = fma(v[i], w[i], part);
    const double Kc = block_sum(part) / vv;
    for (int i = tid; i < len; i += nt) w[i] = w[i] - Kc * v[i];
    __syncthreads();
    // A22 -= v w^T + w v^T
    double* A22w = A + int64_t(k + 1) * m + (k + 1);
    for (int64_t e = tid; e < int64_t(len) * len; e += nt) {
      const int i = int(e / len), j = int(e % len);
      A22w[int64_t(i) * m + j] -= v[i] * w[j] + w[i] * v[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (m >= 2) {
      dg[m - 2] = A[int64_t(m - 2) * m + (m - 2)];
      eg[m - 2] = A[int64_t(m - 1) * m + (m - 2)];
    }
    dg[m - 1] = A[int64_t(m - 1) * m + (m - 1)];
  }
  (void)bc;
}

// Number of eigenvalues below x of the symmetric tridiagonal (d, e) (Sturm count).
__device__ int sturm_below(const double* d, const double* e, int m, double x, double tiny) {
  int c = 0;
  double qv = d[0] - x;
  if (qv < 0.0) ++c;
  for (int i = 1; i < m; ++i) {
    if (fabs(qv) < tiny) qv = -tiny;
    qv = d[i] - x - e[i - 1] * e[i - 1] / qv;
    if (qv < 0.0) ++c;
  }
  return c;
}

// out[0] = r (as double), out[1] = lambda_1
__global__ void rank_from_tridiag_kernel(const double* __restrict__ d, const double* __restrict__ e, int m, double xi,
                                         double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double lo = 0.0, hi = 0.0;
  for (int i = 0; i < m; ++i) {
    const double rad = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < m ? fabs(e[i]) : 0.0);
    lo = fmin(lo, d[i] - rad);
    hi = fmax(hi, d[i] + rad);
  }
  const double tiny = 1e-300 + 1e-18 * fmax(fabs(lo), fabs(hi));
  // lambda_1: smallest x with no eigenvalue above it
  double a = lo, b = hi;
  for (int it = 0; it < 200 && b - a > 1e-15 * fmax(fabs(a), fabs(b)); ++it) {
    const double mid = 0.5 * (a + b);
    if (sturm_below(d, e, m, mid, tiny) >= m) b = mid;
    else a = mid;
  }
  const double lam1 = b;
  const int below = sturm_below(d, e, m, xi * lam1, tiny);  // #{lambda < xi lambda_1}
  int r = m - below + 1;                                     // smallest r with lambda_r <= xi lambda_1
  if (r > m) r = m;
  out[0] = double(r);
  out[1] = lam1;
}

Co<int64_t> adaptive_rank(const float* F0, int64_t n, int64_t r0, int64_t ldf, double xi, Exec& ex,
                          double* lambda1_out) {
  const hipStream_t st = ex.st;
  if (r0 <= 1) co_return r0;
  Woodbury W(F0, n, r0, ldf);
  const double* G = W.gram(st);  // (r0+1)^2 lower triangle of [F0 1]^T [F0 1]
  const int m = int(r0);
  DevBuf A(size_t(m) * m * sizeof(double)), v(size_t(m) * sizeof(double)), w(size_t(m) * sizeof(double));
  DevBuf dg(size_t(m) * sizeof(double)), eg(size_t(m) * sizeof(double)), out(2 * sizeof(double));
  tridiag_kernel<<<1, 1024, 0, st>>>(G, r0 + 1, m, A.as<double>(), v.as<double>(), w.as<double>(), dg.as<double>(),
                                     eg.as<double>());
  KQR_LAUNCH_CHECK();
  rank_from_tridiag_kernel<<<1, 64, 0, st>>>(dg.as<double>(), eg.as<double>(), m, xi, out.as<double>());
  KQR_LAUNCH_CHECK();
  double h[2];
  co_await read_back(ex, out.ptr, 2 * sizeof(double), h);
  if (lambda1_out) *lambda1_out = h[1];
  co_return int64_t(h[0]);
}

}  // namespace kqr
