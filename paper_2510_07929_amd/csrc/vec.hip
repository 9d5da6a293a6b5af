// Fused O(n) vector kernels of the solver, all with deterministic reductions:
// every kernel that produces sums writes one partial per block (the grid
// depends only on n, each thread sums in a fixed order); a single block
// writes its sums directly, several are added in a fixed order by
// `reduce_finalize`.  Runs are bitwise reproducible.
#include "kqr_internal.h"
#include "pstep.h"
#include "reduce.h"
#include "solver.h"

#include <algorithm>

namespace kqr {

__global__ __launch_bounds__(256) void finalize_kernel(const double* __restrict__ partials,
                                                       int nblocks, int nq, double* __restrict__ out) {
  finish_sums(partials, nblocks, nq, out);
}

void reduce_finalize(const double* partials, int nblocks, int nq, double* out, hipStream_t st) {
  finalize_kernel<<<1, 256, 0, st>>>(partials, nblocks, nq, out);
  KQR_LAUNCH_CHECK();
}

#define KQR_GRID_STRIDE(i, n) \
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)
// The same loop for block blk of a grid of nblk blocks (several grids sharing one launch).
#define KQR_GRID_STRIDE_AT(i, n, blk, nblk) \
  for (int64_t i = (blk) * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)(nblk) * blockDim.x)

// Elementwise kernels: one thread per element up to kRedBlocks workgroups.
static inline dim3 ew_grid(int64_t n) {
  return dim3(unsigned(std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, (n + 255) / 256))));
}

// The second pass of a reduction over the partials of a grid of g blocks.
static inline void finish(RedShape g, const double* partials, int nq, double* out, hipStream_t st) {
  if (g.blocks > 1) reduce_finalize(partials, int(g.blocks), nq, out, st);
}

// ----------------------------------------------------------------- generic sums
// out partials: [sum x, sum x*y (if y), sum x*x]
__global__ __launch_bounds__(1024) void dots_kernel(int64_t n, const double* __restrict__ x,
                                                   const double* __restrict__ y, double* partials, double* out) {
  double v[3] = {0.0, 0.0, 0.0};
  KQR_GRID_STRIDE(i, n) {
    const double a = x[i];
    v[0] += a;
    if (y) v[1] = fma(a, y[i], v[1]);
    v[2] = fma(a, a, v[2]);
  }
  block_sums<3>(v, partials, out);
}

void vec_dots(int64_t n, const double* x, const double* y, Workspace& ws, double* out3, hipStream_t st) {
  const RedShape g = red_shape(n);
  dots_kernel<<<g.blocks, g.threads, 0, st>>>(n, x, y, ws.partials, out3);
  KQR_LAUNCH_CHECK();
  finish(g, ws.partials, 3, out3, st);
}

// ----------------------------------------------------------------- PCG
// r = b - (Kx + c*sum(x) + L x) (or r = b when x = 0); Kx zeroed when x = 0.
__global__ __launch_bounds__(1024) void pcg_init_r_kernel(int64_t n, const double* __restrict__ b,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ Kx,
                                                         const double* __restrict__ L, double c,
                                                         const double* __restrict__ sc, int sum_x_slot,
                                                         double* __restrict__ r, double* partials, double* out) {
  const double cs = (x && sum_x_slot >= 0) ? c * sc[sum_x_slot] : 0.0;
  double v[1] = {0.0};
  KQR_GRID_STRIDE(i, n) {
    double ri = b[i];
    if (x) ri -= Kx[i] + cs + L[i] * x[i];
    r[i] = ri;
    v[0] = fma(ri, ri, v[0]);
  }
  block_sums<1>(v, partials, out);
}

void pcg_init_r(int64_t n, const double* b, const double* x, const double* Kx, const double* L,
                double c, const double* sc, int sum_x_slot, double* r, Workspace& ws, double* rr_out,
                hipStream_t st) {
  const RedShape g = red_shape(n);
  pcg_init_r_kernel<<<g.blocks, g.threads, 0, st>>>(n, b, x, Kx, L, c, sc, sum_x_slot, r, ws.partials, rr_out);
  KQR_LAUNCH_CHECK();
  finish(g, ws.partials, 1, rr_out, st);
}

// p = zz (+ beta p with beta = sc[rzn]/sc[rz]); p32 = float(p); partial sum p.
__device__ __forceinline__ void pcg_p_body(int64_t n, const double* __restrict__ zz, double* __restrict__ p,
                                           float* __restrict__ p32, const double* __restrict__ sc, int rz_slot,
                                           int rzn_slot, int first, double* partials, double* out, int blk,
                                           int nblk) {
  const double beta = first ? 0.0 : sc[rzn_slot] / sc[rz_slot];
  double v[1] = {0.0};
  KQR_GRID_STRIDE_AT(i, n, blk, nblk) {
    const double pi = first ? zz[i] : fma(beta, p[i], zz[i]);
    p[i] = pi;
    if (p32) p32[i] = float(pi);
    v[0] += pi;
  }
  block_sums_at<1>(v, partials, out, blk, nblk);
}

__global__ __launch_bounds__(1024) void pcg_p_kernel(int64_t n, const double* __restrict__ zz,
                                                    double* __restrict__ p, float* __restrict__ p32,
                                                    const double* __restrict__ sc, int rz_slot, int rzn_slot,
                                                    int first, double* partials, double* out) {
  pcg_p_body(n, zz, p, p32, sc, rz_slot, rzn_slot, first, partials, out, int(blockIdx.x), int(gridDim.x));
}

void pcg_update_p(int64_t n, const double* zz, double* p, float* p32, const double* sc, int rz_slot,
                  int rzn_slot, bool first, Workspace& ws, double* sump_out, hipStream_t st) {
  const RedShape g = red_shape(n);
  pcg_p_kernel<<<g.blocks, g.threads, 0, st>>>(n, zz, p, p32, sc, rz_slot, rzn_slot, first ? 1 : 0, ws.partials,
                                               sump_out);
  KQR_LAUNCH_CHECK();
  finish(g, ws.partials, 1, sump_out, st);
}

// q = Kp + c*sum(p) + L p ; partial p.q
__device__ __forceinline__ void pcg_q_body(int64_t n, const double* __restrict__ Kp, const double* __restrict__ p,
                                           const double* __restrict__ L, double c, const double* __restrict__ sc,
                                           int sump_slot, double* __restrict__ q, double* partials, double* out,
                                           int blk, int nblk) {
  const double cs = c * sc[sump_slot];
  double v[1] = {0.0};
  KQR_GRID_STRIDE_AT(i, n, blk, nblk) {
    const double pi = p[i];
    const double qi = Kp[i] + cs + L[i] * pi;
    q[i] = qi;
    v[0] = fma(pi, qi, v[0]);
  }
  block_sums_at<1>(v, partials, out, blk, nblk);
}

__global__ __launch_bounds__(1024) void pcg_q_kernel(int64_t n, const double* __restrict__ Kp,
                                                    const double* __restrict__ p,
                                                    const double* __restrict__ L, double c,
                                                    const double* __restrict__ sc, int sump_slot,
                                                    double* __restrict__ q, double* partials, double* out) {
  pcg_q_body(n, Kp, p, L, c, sc, sump_slot, q, partials, out, int(blockIdx.x), int(gridDim.x));
}

void pcg_q(int64_t n, const double* Kp, const double* p, const double* L, double c, const double* sc,
           int sump_slot, double* q, Workspace& ws, double* pq_out, hipStream_t st) {
  const RedShape g = red_shape(n);
  pcg_q_kernel<<<g.blocks, g.threads, 0, st>>>(n, Kp, p, L, c, sc, sump_slot, q, ws.partials, pq_out);
  KQR_LAUNCH_CHECK();
  finish(g, ws.partials, 1, pq_out, st);
}

// a = sc[rz]/sc[pq]; x += a p; r -= a q; Kx += a Kp (if Kx); partial r.r
__device__ __forceinline__ void pcg_xr_body(int64_t n, const double* __restrict__ p, const double* __restrict__ q,
                                            const double* __restrict__ Kp, double* __restrict__ x,
                                            double* __restrict__ r, double* __restrict__ Kx,
                                            const double* __restrict__ sc, int rz_slot, int pq_slot,
                                            double* partials, double* out, int blk, int nblk) {
  const double a = sc[rz_slot] / sc[pq_slot];
  double v[1] = {0.0};
  KQR_GRID_STRIDE_AT(i, n, blk, nblk) {
    x[i] = fma(a, p[i], x[i]);
    const double ri = fma(-a, q[i], r[i]);
    r[i] = ri;
    if (Kx) Kx[i] = fma(a, Kp[i], Kx[i]);
    v[0] = fma(ri, ri, v[0]);
  }
  block_sums_at<1>(v, partials, out, blk, nblk);
}

__global__ __launch_bounds__(1024) void pcg_xr_kernel(int64_t n, const double* __restrict__ p,
                                                     const double* __restrict__ q,
                                                     const double* __restrict__ Kp, double* __restrict__ x,
                                                     double* __restrict__ r, double* __restrict__ Kx,
                                                     const double* __restrict__ sc, int rz_slot,
                                                     int pq_slot, double* partials, double* out) {
  pcg_xr_body(n, p, q, Kp, x, r, Kx, sc, rz_slot, pq_slot, partials, out, int(blockIdx.x), int(gridDim.x));
}

void pcg_xr(int64_t n, const double* p, const double* q, const double* Kp, double* x, double* r,
            double* Kx, const double* sc, int rz_slot, int pq_slot, Workspace& ws, double* rr_out,
            hipStream_t st) {
  const RedShape g = red_shape(n);
  pcg_xr_kernel<<<g.blocks, g.threads, 0, st>>>(n, p, q, Kp, x, r, Kx, sc, rz_slot, pq_slot, ws.partials, rr_out);
  KQR_LAUNCH_CHECK();
  finish(g, ws.partials, 1, rr_out, st);
}

// One workgroup (n <= kOneBlockN): pcg_q and pcg_xr in one launch, with the
// same per-thread order and block sums as the two kernels (bitwise the same).
// The body also serves the batched PCG steps (one workgroup per fit).
__device__ __forceinline__ void pcg_qxr_one_body(int64_t n, const double* __restrict__ Kp,
                                                 const double* __restrict__ p, const double* __restrict__ L,
                                                 double c, double* sc, int sump_slot, int rz_slot, int pq_slot,
                                                 int rr_slot, double* __restrict__ q, double* __restrict__ x,
                                                 double* __restrict__ r, double* __restrict__ Kx) {
  const double cs = c * sc[sump_slot];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double pi = p[i];
    const double qi = Kp[i] + cs + L[i] * pi;
    q[i] = qi;
    acc = fma(pi, qi, acc);
  }
  const double pq = block_sum_all(acc);
  if (threadIdx.x == 0) sc[pq_slot] = pq;
  const double a = sc[rz_slot] / pq;
  acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {  // q[i] was written by this thread
    x[i] = fma(a, p[i], x[i]);
    const double ri = fma(-a, q[i], r[i]);
    r[i] = ri;
    if (Kx) Kx[i] = fma(a, Kp[i], Kx[i]);
    acc = fma(ri, ri, acc);
  }
  const double rr = block_sum_all(acc);
  if (threadIdx.x == 0) sc[rr_slot] = rr;
}

__global__ __launch_bounds__(1024) void pcg_qxr_one_kernel(int64_t n, const double* __restrict__ Kp,
                                                          const double* __restrict__ p,
                                                          const double* __restrict__ L, double c, double* sc,
                                                          int sump_slot, int rz_slot, int pq_slot, int rr_slot,
                                                          double* __restrict__ q, double* __restrict__ x,
                                                          double* __restrict__ r, double* __restrict__ Kx) {
  pcg_qxr_one_body(n, Kp, p, L, c, sc, sump_slot, rz_slot, pq_slot, rr_slot, q, x, r, Kx);
}

// Batched PCG steps: workgroup f runs fit f's pcg_qxr.
__global__ __launch_bounds__(1024) void pcg_qxr_steps_kernel(const PcgStepDesc* __restrict__ d) {
  const PcgStepDesc& e = d[blockIdx.x];
  pcg_qxr_one_body(e.n, e.Kp, e.p, e.L, e.c, e.sc, e.sump, e.rz, e.pq, e.rr, e.q, e.x, e.r, e.Kx);
}

void launch_pcg_qxr_steps(const PcgStepDesc* d, int nf, hipStream_t st) {
  if (nf <= 0) return;
  pcg_qxr_steps_kernel<<<nf, kOneBlockThreads, 0, st>>>(d);
  KQR_LAUNCH_CHECK();
}

// Batched PCG steps of fits whose vectors take several workgroups: each
// fit's nred blocks of kRedThreads, the blocks of fit f starting at first[f];
// the partial sums of each pass go to the fit's partials and a finishing
// launch (one workgroup per fit) adds them, as for the single-fit launches.
__global__ __launch_bounds__(256) void pcg_q_steps_kernel(const PcgStepDesc* __restrict__ d,
                                                          const int* __restrict__ first, int nf) {
  const int f = step_of_block(first, nf, int(blockIdx.x));
  const PcgStepDesc& e = d[f];
  pcg_q_body(e.n, e.Kp, e.p, e.L, e.c, e.sc, e.sump, e.q, e.partials, e.sc + e.pq, int(blockIdx.x) - first[f],
             e.nred);
}

__global__ __launch_bounds__(256) void pcg_xr_steps_kernel(const PcgStepDesc* __restrict__ d,
                                                           const int* __restrict__ first, int nf) {
  const int f = step_of_block(first, nf, int(blockIdx.x));
  const PcgStepDesc& e = d[f];
  pcg_xr_body(e.n, e.p, e.q, e.Kp, e.x, e.r, e.Kx, e.sc, e.rz, e.pq, e.partials, e.sc + e.rr,
              int(blockIdx.x) - first[f], e.nred);
}

__global__ __launch_bounds__(256) void pcg_p_steps_kernel(const PcgStepDesc* __restrict__ d,
                                                          const int* __restrict__ first, int nf) {
  const int f = step_of_block(first, nf, int(blockIdx.x));
  const PcgStepDesc& e = d[f];
  pcg_p_body(e.n, e.zz, e.p, e.p32, e.sc, e.rz, e.rz_new, 0, e.partials, e.sc + e.sump, int(blockIdx.x) - first[f],
             e.nred);
}

// which: 0 p.q, 1 r.r, 2 r.zz (the new rz), 3 sum p -- the last also hands
// (p.q, r.r) and the completion tag to the fit's status pair when it has one
__global__ __launch_bounds__(256) void finalize_steps_kernel(const PcgStepDesc* __restrict__ d, int which) {
  const PcgStepDesc& e = d[blockIdx.x];
  const int slot = which == 0 ? e.pq : which == 1 ? e.rr : which == 2 ? e.rz_new : e.sump;
  finish_sums(e.partials, e.nred, 1, e.sc + slot);
  if (which == 3 && e.status && threadIdx.x == 0) {
    __threadfence_system();
    e.status[0] = e.sc[e.pq];
    e.status[1] = e.sc[e.rr];
    __threadfence_system();
    *static_cast<volatile double*>(e.status + 2) = 1.0;
  }
}

void launch_pcg_q_steps(const PcgStepDesc* d, const int* first, int nf, int total, hipStream_t st) {
  if (nf <= 0 || total <= 0) return;
  pcg_q_steps_kernel<<<total, kRedThreads, 0, st>>>(d, first, nf);
  KQR_LAUNCH_CHECK();
}

void launch_pcg_xr_steps(const PcgStepDesc* d, const int* first, int nf, int total, hipStream_t st) {
  if (nf <= 0 || total <= 0) return;
  pcg_xr_steps_kernel<<<total, kRedThreads, 0, st>>>(d, first, nf);
  KQR_LAUNCH_CHECK();
}

void launch_pcg_p_steps(const PcgStepDesc* d, const int* first, int nf, int total, hipStream_t st) {
  if (nf <= 0 || total <= 0) return;
  pcg_p_steps_kernel<<<total, kRedThreads, 0, st>>>(d, first, nf);
  KQR_LAUNCH_CHECK();
}

void launch_finalize_steps(const PcgStepDesc* d, int nf, int which, hipStream_t st) {
  if (nf <= 0) return;
  finalize_steps_kernel<<<nf, 256, 0, st>>>(d, which);
  KQR_LAUNCH_CHECK();
}

void pcg_qxr(int64_t n, const double* Kp, const double* p, const double* L, double c, double* sc, int sump_slot,
             int rz_slot, int pq_slot, int rr_slot, double* q, double* x, double* r, double* Kx, Workspace& ws,
             hipStream_t st) {
  if (n <= kOneBlockN) {
    pcg_qxr_one_kernel<<<1, kOneBlockThreads, 0, st>>>(n, Kp, p, L, c, sc, sump_slot, rz_slot, pq_slot, rr_slot, q,
                                                       x, r, Kx);
    KQR_LAUNCH_CHECK();
    return;
  }
  pcg_q(n, Kp, p, L, c, sc, sump_slot, q, ws, sc + pq_slot, st);
  pcg_xr(n, p, q, Kp, x, r, Kx, sc, rz_slot, pq_slot, ws, sc + rr_slot, st);
}

// ----------------------------------------------------------------- ADMM / ALM
// b = lambda (y - beta - z + sigma v)
__global__ __launch_bounds__(256) void admm_rhs_kernel(int64_t n, const double* __restrict__ y,
                                                       const double* __restrict__ z,
                                                       const double* __restrict__ v, double beta,
                                                       double sigma, double lam, double* __restrict__ b) {
  KQR_GRID_STRIDE(i, n) b[i] = lam * (y[i] - beta - z[i] + sigma * v[i]);
}

void admm_rhs(int64_t n, const double* y, const double* z, const double* v, double beta, double sigma,
              double lam, double* b, hipStream_t st) {
  admm_rhs_kernel<<<ew_grid(n), 256, 0, st>>>(n, y, z, v, beta, sigma, lam, b);
  KQR_LAUNCH_CHECK();
}

// v = Pi_B(alpha + z/sigma); z += step*sigma*(alpha - v); then the KKT sums of
// Section 4 at (alpha, v, beta_new, z):
//   [0] ||z - y + beta 1 + K alpha/lam||^2  [1] ||alpha - v||^2  [2] ||alpha||^2
//   [3] ||v - Pi_B(z + v)||^2  [4] ||v||^2  [5] rho_tau(z)  [6] alpha.Kalpha
//   [7] y.alpha  [8] 1.alpha
__global__ __launch_bounds__(1024) void multiplier_kkt_kernel(
    int64_t n, const double* __restrict__ alpha, const double* __restrict__ Ka,
    const double* __restrict__ y, double* __restrict__ z, double* __restrict__ v, double beta_new,
    double sigma, double step, double tau, double lam, int update, double* partials, double* out) {
  double s[kKktSums];
#pragma unroll
  for (int q = 0; q < kKktSums; ++q) s[q] = 0.0;
  const double lo = tau - 1.0, hi = tau;
  const double inv_lam = 1.0 / lam;
  KQR_GRID_STRIDE(i, n) {
    const double a = alpha[i];
    double zi = z[i];
    double vi;
    if (update) {
      vi = fmin(fmax(a + zi / sigma, lo), hi);
      zi = fma(step * sigma, a - vi, zi);
      z[i] = zi;
      v[i] = vi;
    } else {
      vi = v[i];
    }
    const double kai = Ka[i];
    const double rp = zi - y[i] + beta_new + kai * inv_lam;
    s[0] = fma(rp, rp, s[0]);
    const double dv = a - vi;
    s[1] = fma(dv, dv, s[1]);
    s[2] = fma(a, a, s[2]);
    const double pc = vi - fmin(fmax(zi + vi, lo), hi);
    s[3] = fma(pc, pc, s[3]);
    s[4] = fma(vi, vi, s[4]);
    s[5] += zi > 0.0 ? tau * zi : -(1.0 - tau) * zi;
    s[6] = fma(a, kai, s[6]);
    s[7] = fma(y[i], a, s[7]);
    s[8] += a;
  }
  block_sums<kKktSums>(s, partials, out);
}

void multiplier_kkt(int64_t n, const double* alpha, const double* Ka, const double* y, double* z,
                    double* v, double beta_new, double sigma, double step, double tau, double lam,
                    bool update, Workspace& ws, double* out, hipStream_t st) {
  const RedShape g = red_shape(n);
  multiplier_kkt_kernel<<<g.blocks, g.threads, 0, st>>>(n, alpha, Ka, y, z, v, beta_new, sigma, step, tau,
                                                    lam, update ? 1 : 0, ws.partials, out);
  KQR_LAUNCH_CHECK();
  finish(g, ws.partials, kKktSums, out, st);
}

// ----------------------------------------------------------------- SSN (Algorithm 3)
// grad = Ka/lam - y + beta + sigma*sum(alpha) + sigma (w - Pi_B(w)),  w = alpha + z/sigma
// S = 1 strictly inside (tau-1, tau); partials [||grad||^2]
__global__ __launch_bounds__(1024) void ssn_grad_kernel(int64_t n, const double* __restrict__ alpha,
                                                       const double* __restrict__ Ka,
                                                       const double* __restrict__ y,
                                                       const double* __restrict__ z, double beta,
                                                       double sigma, double sum_alpha, double tau,
                                                       double lam, double* __restrict__ grad,
                                                       uint8_t* __restrict__ S, double* partials, double* out) {
  const double lo = tau - 1.0, hi = tau;
  const double base = beta + sigma * sum_alpha;
  const double inv_lam = 1.0 / lam;
  double v[1] = {0.0};
  KQR_GRID_STRIDE(i, n) {
    const double w = alpha[i] + z[i] / sigma;
    const double pw = fmin(fmax(w, lo), hi);
    const double g = Ka[i] * inv_lam - y[i] + base + sigma * (w - pw);
    grad[i] = g;
    S[i] = (w > lo && w < hi) ? 1 : 0;
    v[0] = fma(g, g, v[0]);
  }
  block_sums<1>(v, partials, out);
}

void ssn_grad(int64_t n, const double* alpha, const double* Ka, const double* y, const double* z,
              double beta, double sigma, double sum_alpha, double tau, double lam, double* grad,
              uint8_t* S, Workspace& ws, double* gg_out, hipStream_t st) {
  const RedShape g = red_shape(n);
  ssn_grad_kernel<<<g.blocks, g.threads, 0, st>>>(n, alpha, Ka, y, z, beta, sigma, sum_alpha, tau, lam, grad,
                                              S, ws.partials, gg_out);
  KQR_LAUNCH_CHECK();
  finish(g, ws.partials, 1, gg_out, st);
}

// L = lam sigma (1 - S) + lam eps_t ; rhs = -lam grad
__global__ __launch_bounds__(256) void ssn_system_kernel(int64_t n, const uint8_t* __restrict__ S,
                                                         const double* __restrict__ grad, double lam,
                                                         double sigma, double eps_t,
                                                         double* __restrict__ L, double* __restrict__ rhs) {
  const double ls = lam * sigma, le = lam * eps_t;
  KQR_GRID_STRIDE(i, n) {
    L[i] = (S[i] ? 0.0 : ls) + le;
    rhs[i] = -lam * grad[i];
  }
}

void ssn_system(int64_t n, const uint8_t* S, const double* grad, double lam, double sigma, double eps_t,
                double* L, double* rhs, hipStream_t st) {
  ssn_system_kernel<<<ew_grid(n), 256, 0, st>>>(n, S, grad, lam, sigma, eps_t, L, rhs);
  KQR_LAUNCH_CHECK();
}

// Line search sums for phi(alpha + c d) - phi(alpha) expanded from (2.2):
//   [0] d.Ka  [1] d.Kd  [2] y.d  [3] 1.d  [4] grad.d
//   [5 + j] sum_i dist^2(w_i + c_j d_i) - dist^2(w_i),  c_j = c0 shrink^j
__global__ __launch_bounds__(1024) void line_search_kernel(
    int64_t n, const double* __restrict__ alpha, const double* __restrict__ z,
    const double* __restrict__ d, const double* __restrict__ Ka, const double* __restrict__ Kd,
    const double* __restrict__ y, const double* __restrict__ grad, double sigma, double tau,
    double c0, double shrink, double* partials, double* out) {
  double s[5 + kLsTrials];
#pragma unroll
  for (int q = 0; q < 5 + kLsTrials; ++q) s[q] = 0.0;
  const double lo = tau - 1.0, hi = tau;
  KQR_GRID_STRIDE(i, n) {
    const double di = d[i];
    s[0] = fma(di, Ka[i], s[0]);
    s[1] = fma(di, Kd[i], s[1]);
    s[2] = fma(di, y[i], s[2]);
    s[3] += di;
    s[4] = fma(di, grad[i], s[4]);
    const double w = alpha[i] + z[i] / sigma;
    const double r0 = w - fmin(fmax(w, lo), hi);
    double c = c0;
#pragma unroll
    for (int j = 0; j < kLsTrials; ++j) {
      const double wc = fma(c, di, w);
      const double r1 = wc - fmin(fmax(wc, lo), hi);
      s[5 + j] += (r1 - r0) * (r1 + r0);
      c *= shrink;
    }
  }
  block_sums<5 + kLsTrials>(s, partials, out);
}

void line_search_sums(int64_t n, const double* alpha, const double* z, const double* d, const double* Ka,
                      const double* Kd, const double* y, const double* grad, double sigma, double tau,
                      double c0, double shrink, Workspace& ws, double* out, hipStream_t st) {
  const RedShape g = red_shape(n);
  line_search_kernel<<<g.blocks, g.threads, 0, st>>>(n, alpha, z, d, Ka, Kd, y, grad, sigma, tau, c0, shrink,
                                                 ws.partials, out);
  KQR_LAUNCH_CHECK();
  finish(g, ws.partials, 5 + kLsTrials, out, st);
}

// x += c d ; Kx += c Kd
__global__ __launch_bounds__(256) void axpy2_kernel(int64_t n, double c, const double* __restrict__ d,
                                                    double* __restrict__ x, const double* __restrict__ Kd,
                                                    double* __restrict__ Kx) {
  KQR_GRID_STRIDE(i, n) {
    x[i] = fma(c, d[i], x[i]);
    if (Kx) Kx[i] = fma(c, Kd[i], Kx[i]);
  }
}

void axpy2(int64_t n, double c, const double* d, double* x, const double* Kd, double* Kx, hipStream_t st) {
  axpy2_kernel<<<ew_grid(n), 256, 0, st>>>(n, c, d, x, Kd, Kx);
  KQR_LAUNCH_CHECK();
}

// Non-finite check: partial [count of non-finite entries]
__global__ __launch_bounds__(1024) void nonfinite_kernel(int64_t n, const double* __restrict__ x,
                                                        double* partials, double* out) {
  double v[1] = {0.0};
  KQR_GRID_STRIDE(i, n) {
    if (!isfinite(x[i])) v[0] += 1.0;
  }
  block_sums<1>(v, partials, out);
}

void count_nonfinite(int64_t n, const double* x, Workspace& ws, double* out, hipStream_t st) {
  const RedShape g = red_shape(n);
  nonfinite_kernel<<<g.blocks, g.threads, 0, st>>>(n, x, ws.partials, out);
  KQR_LAUNCH_CHECK();
  finish(g, ws.partials, 1, out, st);
}

__global__ void fill_kernel(int64_t n, double val, double* __restrict__ x) {
  KQR_GRID_STRIDE(i, n) x[i] = val;
}

void fill(int64_t n, double val, double* x, hipStream_t st) {
  fill_kernel<<<ew_grid(n), 256, 0, st>>>(n, val, x);
  KQR_LAUNCH_CHECK();
}

__global__ void copy_kernel(int64_t n, const double* __restrict__ s, double* __restrict__ d) {
  KQR_GRID_STRIDE(i, n) d[i] = s[i];
}

void copy(int64_t n, const double* src, double* dst, hipStream_t st) {
  copy_kernel<<<ew_grid(n), 256, 0, st>>>(n, src, dst);
  KQR_LAUNCH_CHECK();
}

// count of tau-1 < alpha_i < tau : partial
__global__ __launch_bounds__(1024) void interior_kernel(int64_t n, const double* __restrict__ a, double tau,
                                                       double* partials, double* out) {
  double v[1] = {0.0};
  KQR_GRID_STRIDE(i, n) {
    if (a[i] > tau - 1.0 && a[i] < tau) v[0] += 1.0;
  }
  block_sums<1>(v, partials, out);
}

void count_interior(int64_t n, const double* a, double tau, Workspace& ws, double* out, hipStream_t st) {
  const RedShape g = red_shape(n);
  interior_kernel<<<g.blocks, g.threads, 0, st>>>(n, a, tau, ws.partials, out);
  KQR_LAUNCH_CHECK();
  finish(g, ws.partials, 1, out, st);
}

}  // namespace kqr

namespace kqr {
// dst = src ; partial src . dst
__global__ __launch_bounds__(1024) void copy_dot_kernel(int64_t n, const double* __restrict__ s,
                                                       double* __restrict__ d, double* partials, double* out) {
  double v[1] = {0.0};
  KQR_GRID_STRIDE(i, n) {
    const double a = s[i];
    d[i] = a;
    v[0] = fma(a, a, v[0]);
  }
  block_sums<1>(v, partials, out);
}

void copy_dot(int64_t n, const double* src, double* dst, Workspace& ws, double* out, hipStream_t st) {
  const RedShape g = red_shape(n);
  copy_dot_kernel<<<g.blocks, g.threads, 0, st>>>(n, src, dst, ws.partials, out);
  KQR_LAUNCH_CHECK();
  finish(g, ws.partials, 1, out, st);
}
}  // namespace kqr
