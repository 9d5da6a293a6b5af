// The fit drivers: one problem, a batch of quantile levels on one K, and a
// batch of independent problems.
#pragma once

#include "kmulti.h"
#include "solver.h"

namespace kqr {

void validate_options(const kqr_options& o);  // fails with KQR_EINVAL

// Kernel matrix (materialised or not) and RPCholesky factor of one problem.
struct Prepared {
  DevBuf K;
  int64_t ldk = 0;
  int dtype = KQR_FP32;
  int layout = 0;  // 0 full n x ldk; 1 upper-triangle tiles (ldk = tiles per side)
  DevBuf K32;  // FP32 copy beside a BF16 K (exact applies), when requested
  DevBuf F;
  int64_t ldf = 4;
  int64_t rank = 0;
  double t_kbuild = 0.0, t_precond = 0.0;
  KMat kmat() const { return KMat{K.ptr, dtype, ldk, layout}; }
  KMat kmat_exact() const { return KMat{K32.ptr, KQR_FP32, ldk, layout}; }
  // Operator over this K (and its FP32 copy for the exact applies, if any).
  void attach(Operator& op) const {
    if (K32.ptr) op.set_exact(kmat_exact());
  }
};

// Materialises K (per o.kmode / o.k_dtype) and builds F (fixed rank, the
// Section 3 heuristic, or none) on ex's stream.  `op` is created by the
// caller afterwards.
Co<Prepared> prepare_fit(const float* X, int64_t n, int p, KernelSpec ks, kqr_options o, Exec& ex);

struct FitOutcome {
  bool converged = false;
  double beta = 0.0;
  kqr_info info{};
};

// Runs Phase I, Phase II and the final residuals on ex's stream; copies
// alpha to alpha_out and, when z_out / v_out are given, the final multipliers
// z and the final consensus vector v to them (device, n).
Co<FitOutcome> run_fit(Operator& op, const Prepared& pr, const double* y, int64_t n, double tau, double lam,
                       kqr_options o, double* alpha_out, Exec& ex, double* z_out = nullptr,
                       double* v_out = nullptr);

// Batches run as coroutines on the calling thread (coro.h): one scheduler,
// a few streams, and one batched launch per round of K-apply requests.
//
// tau batch: every level shares K and F; fast K-applies of all levels are
// coalesced into one K V launch on the matrix cores.
void fit_multi_tau(const float* X, const double* y, int64_t n, int p, KernelSpec ks, const double* taus, int ntau,
                   double lam, const kqr_options& o, double* alpha, double* beta, kqr_info* info, int* status,
                   hipStream_t st);

// lambda path: nlam values of lambda on one (X, y, tau, kernel); K and F are
// built once, every value is a cold start, and up to kKvMaxCols values run at
// once with their fast K-applies coalesced into K V launches (a worker that
// finishes one value takes the next).
void fit_path(const float* X, const double* y, int64_t n, int p, KernelSpec ks, double tau, const double* lams,
              int nlam, const kqr_options& o, double* alpha, double* beta, kqr_info* info, int* status,
              hipStream_t st);

// independent problems: fast K-applies of all running problems go out in one
// launch over (problem, row block) pairs.
void fit_batch(int nprob, const float* const* X, const double* const* y, const int64_t* n, int p, KernelSpec ks,
               const double* tau, const double* lam, const double* gamma, const kqr_options& o,
               double* const* alpha, double* beta, kqr_info* info, int* status, hipStream_t st);

std::vector<double> default_uniforms(uint64_t seed, int64_t count);
void set_batch_threads(int t);  // host threads of the batched fits (0: min(16, cores))
void set_batch_steps(bool on);   // kqr_fit_batch runs PCG iterations' vector work batched (default on)
double wall_seconds();

}  // namespace kqr
