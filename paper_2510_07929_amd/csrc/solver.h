// Host-side driver objects of the fit.
#pragma once

#include <memory>

#include "coro.h"
#include "vec.h"

namespace kqr {

// The kernel operator K v: materialised (FP32 / BF16 storage) or on the fly.
class Operator {
 public:
  Operator(const float* X, int64_t n, int p, KernelSpec ks, KMat km, hipStream_t st);
  // Route the applies through the scheduler's batched launches (fast ones
  // always, exact ones when the scheduler's launcher serves them).
  void attach_batching(bool on) { batched_ = on; }
  // FP32 copy of K for the exact applies when the fast operator is stored in BF16.
  void set_exact(KMat k) { kexact_ = k; }
  // Fast apply: FP32 products (from v32 when given, else a rounded copy of v).
  // In a batch the request goes to ex's scheduler and the returned awaitable
  // suspends until the batched launch has been enqueued.
  [[nodiscard]] ApplyAwait apply_fast(const double* v, const float* v32, double* u, Exec& ex);
  // Exact apply: FP32 entries (stored FP32 or recomputed) with FP64 vector and sums.
  [[nodiscard]] ApplyAwait apply_exact(const double* v, double* u, Exec& ex);
  // Whether ex's batched launches can also run the rest of a PCG iteration
  // (pstep.h); then apply_fast_step hands the fast apply u = K v together with
  // that iteration's descriptor.
  bool steps_batched(const Exec& ex) const { return batched_ && ex.sched && ex.sched->steps_ok(); }
  [[nodiscard]] ApplyAwait apply_fast_step(const double* v, double* u, const PcgStepDesc* step, bool clean,
                                           Exec& ex);
  bool materialized() const { return km_.K != nullptr; }
  int64_t calls() const { return calls_; }
  const KMat& kmat() const { return km_; }
  const float* sqn() const { return sqn_.as<float>(); }
  const float* X() const { return X_; }
  int p() const { return p_; }
  KernelSpec spec() const { return ks_; }
  // Record HIP events around every K-apply kernel (for kqr_info.t_kapply_*).
  void enable_profile(bool on) { profile_ = on; }
  // Sums the recorded kernel times (synchronises the events); seconds.
  void profile_totals(int64_t& nfast, double& tfast, int64_t& nexact, double& texact);
  ~Operator();

 private:
  struct Span { hipEvent_t a, b; bool fast; };
  void mark(bool begin, bool fast, hipStream_t st);
  const float* X_;
  int64_t n_;
  int p_;
  KernelSpec ks_;
  KMat km_;
  KMat kexact_;
  DevBuf sqn_, v32_;
  DevBuf scr_;  // partial sums of the materialised and symmetric on-the-fly applies (allocated on first use)
  DevBuf lin_;  // linear kernel: block partials and X^T v
  DevBuf xq_;   // Laplacian: fixed-point X (entries recomputed on every apply)
  int shift_ = -1;
  double* scratch(const KMat& k, size_t& doubles);
  double* scratch(size_t doubles);  // at least that many doubles, kept for later applies
  int64_t calls_ = 0;
  bool profile_ = false;
  std::vector<Span> spans_;
  bool batched_ = false;
};

struct PcgBuffers {
  DevBuf r, zz, p, q, Kp, p32, sc;
  explicit PcgBuffers(int64_t n);
};

struct PcgStats {
  int iters = 0;
  double resnorm = 0.0;
  bool breakdown = false;
};

struct Kkt {
  double eta_p = 1, eta_d = 1, eta_c = 1, eta_kkt = 1, eta_gap = 1, err = 1;
  double obj_p = 0, obj_d = 0, sum_alpha = 0;
};

// Section 4 residuals and objectives from the nine sums of multiplier_kkt.
Kkt kkt_from_sums(const double* s, double ynorm, double lam);

// Left-preconditioned conjugate gradients on (K + c 1 1^T + diag(L)) x = b.
class Pcg {
 public:
  Pcg(Operator& op, Workspace& ws, int64_t n, Exec& ex);
  // x holds the start (ignored when x_zero); Kx, when given, holds K x on entry
  // (ignored when x_zero) and is advanced with the same steps as x.
  Co<PcgStats> solve(double c, const double* L, Woodbury* P, const double* b, double* x, double* Kx, bool x_zero,
                     double tol, int maxit, bool fast);

 private:
  Operator& op_;
  Workspace& ws_;
  int64_t n_;
  Exec& ex_;
  PcgBuffers pb_;
};

class Solver {
 public:
  Solver(Operator& op, Exec& ex, const double* y, int64_t n, double tau, double lam, const kqr_options& o,
         const float* F, int64_t rank, int64_t ldf);
  Co<Unit> init();  // reads ||y|| (fails on non-finite y)
  Co<Unit> phase1(kqr_info& info);
  // Instead of phase1: (alpha, v, beta, z, sigma) from the options' warm start.
  Co<Unit> warm_start(kqr_info& info);
  Co<Unit> phase2(kqr_info& info);
  Co<Unit> finish(kqr_info& info);
  const double* alpha() const { return alpha_.as<double>(); }
  const double* z() const { return z_.as<double>(); }  // ALM multipliers
  const double* v() const { return v_.as<double>(); }  // consensus copy of alpha (1.4)
  double beta() const { return beta_; }
  bool converged() const { return converged_; }
  Workspace& ws() { return ws_; }

 private:
  Co<PcgStats> linsolve(double c, const double* L, const double* b, double* x, double* Kx, bool x_zero, double tol,
                        bool refine, kqr_info& info);
  Co<Unit> ssn(double stop, kqr_info& info);
  Kkt kkt_from_sums(const double* s) const;
  Co<Kkt> update_and_kkt(double beta_new, double sigma, double step, bool update);
  void record(int phase, int it, double err);
  Co<double> sum_of(const double* x);

  Operator& op_;
  Exec& ex_;
  const double* y_;
  int64_t n_;
  double tau_, lam_;
  kqr_options o_;
  hipStream_t st_;
  Workspace ws_;
  Pcg pcg_;
  DevBuf alpha_, v_, z_, Ka_, b_, L_, grad_, d_, Kd_, S_, red_;
  DevBuf rf_r_, rf_dx_, rf_kdx_;  // refinement workspace (BF16 storage)
  std::unique_ptr<Woodbury> P_;
  double beta_ = 0.0, sigma_ = 1.0, ynorm_ = 0.0, eta_d_prev_ = 1.0;
  double eps_floor_ = 0.0;  // floor of eps_t, raised after a Woodbury core breakdown
  double t_start_ = 0.0;
  int ntrace_ = 0;
  Kkt last_;
  bool converged_ = false;
};

// copy src -> dst and dot_with . dst into *out (device)
void copy_dot(int64_t n, const double* src, double* dst, Workspace& ws, double* out, hipStream_t st);

}  // namespace kqr
