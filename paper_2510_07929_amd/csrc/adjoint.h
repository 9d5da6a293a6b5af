// Implicit gradient of the validation check loss with respect to log(gamma)
// and log(lambda) at a fitted KQR solution.
#pragma once

#include "vec.h"

namespace kqr {

struct GradOutcome {
  double J = 0.0;     // validation check loss
  double dgam = 0.0;  // dJ / dlog(gamma)
  double dlam = 0.0;  // dJ / dlog(lambda)
  int64_t n_interior = 0;
  bool polished = false;
  int polish_rounds = 0;  // active-set rounds used by the polish
};

// Largest interior set whose FP64 K_EE is factored densely.
constexpr int64_t kAdjointMaxInterior = 8192;
// Active-set rounds of the polish before giving up.
constexpr int kPolishRounds = 12;

// X (n x p, device FP32); alpha (device, n) and
// *beta are the fitted coefficients and are replaced by the polished ones when
// the active-set polish succeeds; z (device, n) are the final ALM multipliers;
// y (device FP64).  Xv (nv x p) and yv are the validation set.  tol is the
// KKT level the fit reached (scales the |z| thresholds of the polish).
GradOutcome adjoint_gradient(const float* X, int64_t n, int p, KernelSpec ks, double tau, double lam, double* alpha,
                             double* beta, const double* z, const double* y, const float* Xv, int64_t nv,
                             const double* yv, double tol, hipStream_t st);

}  // namespace kqr
