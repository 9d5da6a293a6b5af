// Host driver of PALM-KQR on one stream: PCG (Section 3), Phase I inexact
// ADMM (Algorithm 1), Phase II semismooth Newton ALM (Algorithms 2 and 3),
// stopping rules of Section 4.  Every O(n) and O(n^2) step runs in device
// kernels; the host only sequences launches and reads back the scalars that
// decide convergence (a few doubles per iteration).
#include "solver.h"
#include "reduce.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>

namespace kqr {

// ================================================================= operator
Operator::Operator(const float* X, int64_t n, int p, KernelSpec ks, KMat km, hipStream_t st)
    : X_(X), n_(n), p_(p), ks_(ks), km_(km), sqn_(size_t(std::max<int64_t>(n, 1)) * sizeof(float)),
      v32_(size_t(std::max<int64_t>(n, 1)) * sizeof(float)) {
  if (ks.kind == KQR_LINEAR) {
    if (km.K) fail(KQR_EINVAL, "the linear kernel is applied in factored form (no materialised K)");
    lin_.alloc(lin_scratch_doubles(p) * sizeof(double));
  }
  row_sqnorms(X, n, p, sqn_.as<float>(), st);
  // Laplacian entries recomputed on every apply (on the fly, or the exact
  // operator beside a BF16 K): exact integer L1 distances of fixed-point X
  // when the quantum 2^-s keeps the entries at FP32 accuracy (s >= 20)
  if (ks.kind == KQR_LAPLACIAN && !(km.K && km.dtype == KQR_FP32) && n > 0) {
    xq_.alloc(size_t(n) * size_t(p) * sizeof(uint32_t));
    shift_ = quantize_columns(X, n, p, xq_.as<uint32_t>(), st);
    if (shift_ < 20) {
      xq_ = DevBuf();
      shift_ = -1;
    }
  }
}

Operator::~Operator() {
  for (auto& s : spans_) {
    (void)hipEventDestroy(s.a);
    (void)hipEventDestroy(s.b);
  }
}

void Operator::mark(bool begin, bool fast, hipStream_t st) {
  if (!profile_) return;
  if (begin) {
    Span s{};
    KQR_CHECK_HIP(hipEventCreate(&s.a));
    KQR_CHECK_HIP(hipEventCreate(&s.b));
    s.fast = fast;
    spans_.push_back(s);
    KQR_CHECK_HIP(hipEventRecord(spans_.back().a, st));
  } else {
    KQR_CHECK_HIP(hipEventRecord(spans_.back().b, st));
  }
}

void Operator::profile_totals(int64_t& nfast, double& tfast, int64_t& nexact, double& texact) {
  nfast = nexact = 0;
  tfast = texact = 0.0;
  for (auto& s : spans_) {
    KQR_CHECK_HIP(hipEventSynchronize(s.b));
    float ms = 0.f;
    KQR_CHECK_HIP(hipEventElapsedTime(&ms, s.a, s.b));
    if (s.fast) { ++nfast; tfast += 1e-3 * ms; }
    else { ++nexact; texact += 1e-3 * ms; }
  }
}

double* Operator::scratch(size_t doubles) {
  if (scr_.bytes < doubles * sizeof(double)) {
    scr_ = DevBuf();
    scr_.alloc(doubles * sizeof(double));
  }
  return scr_.as<double>();
}

double* Operator::scratch(const KMat& k, size_t& doubles) {
  doubles = kapply_scratch_doubles(k, n_);
  return scratch(doubles);
}

ApplyAwait Operator::apply_fast(const double* v, const float* v32, double* u, Exec& ex) {
  ++calls_;
  const hipStream_t st = ex.st;
  if (batched_) return ApplyAwait{&ex, ApplyReq{v, u, false}};
  if (ks_.kind == KQR_LINEAR) {  // X (X^T v), FP64: the fast and the exact operator coincide
    mark(true, true, st);
    lin_apply(X_, n_, p_, v, u, 1, lin_.as<double>(), st);
    mark(false, true, st);
    return {};
  }
  if (km_.K) {
    if (!v32) {
      to_f32(v, n_, 1, 1, v32_.as<float>(), 1, st);
      v32 = v32_.as<float>();
    }
    size_t nd = 0;
    double* scr = scratch(km_, nd);
    mark(true, true, st);
    kapply_dense(km_, n_, n_, v32, nullptr, u, 1, false, st, nullptr, scr, nd);
    mark(false, true, st);
  } else if (xq_.ptr) {
    const size_t nd = otf_sym_scratch_doubles(n_);
    double* scr = scratch(nd);
    mark(true, true, st);
    kapply_otf_l1q(xq_.as<uint32_t>(), n_, p_, ks_.gamma, shift_, v, u, 1, false, st, scr, nd);
    mark(false, true, st);
  } else {
    const size_t nd = otf_sym_scratch_doubles(n_);
    double* scr = scratch(nd);
    mark(true, true, st);
    kapply_otf(X_, sqn_.as<float>(), n_, X_, sqn_.as<float>(), n_, p_, ks_, v, u, 1, 1.0, 0.0, st, false, scr, nd);
    mark(false, true, st);
  }
  return {};
}

ApplyAwait Operator::apply_fast_step(const double* v, double* u, const PcgStepDesc* step, bool clean, Exec& ex) {
  if (!steps_batched(ex)) fail(KQR_EHIP, "internal: batched PCG step without a launcher that runs it");
  ++calls_;
  return ApplyAwait{&ex, ApplyReq{v, u, false, step, clean}};
}

ApplyAwait Operator::apply_exact(const double* v, double* u, Exec& ex) {
  ++calls_;
  const hipStream_t st = ex.st;
  if (batched_ && ex.sched->exact_ok()) return ApplyAwait{&ex, ApplyReq{v, u, true}};  // rides along in the shared pass over K
  size_t nd = 0;
  double* scr = nullptr;
  if (km_.K) scr = scratch(km_.dtype == KQR_FP32 || !kexact_.K ? km_ : kexact_, nd);
  else if (xq_.ptr) scr = scratch(nd = otf_sym_scratch_doubles(n_));
  mark(true, false, st);
  if (ks_.kind == KQR_LINEAR) {
    lin_apply(X_, n_, p_, v, u, 1, lin_.as<double>(), st);
  } else if (km_.K && km_.dtype == KQR_FP32) {
    kapply_dense(km_, n_, n_, nullptr, v, u, 1, true, st, nullptr, scr, nd);
  } else if (kexact_.K) {
    kapply_dense(kexact_, n_, n_, nullptr, v, u, 1, true, st, nullptr, scr, nd);
  } else if (xq_.ptr) {
    kapply_otf_l1q(xq_.as<uint32_t>(), n_, p_, ks_.gamma, shift_, v, u, 1, true, st, scr, nd);
  } else {
    // BF16 storage is not the exact operator: recompute FP32 entries from X.
    scr = scratch(nd = otf_sym_scratch_doubles(n_));
    kapply_otf(X_, sqn_.as<float>(), n_, X_, sqn_.as<float>(), n_, p_, ks_, v, u, 1, 1.0, 0.0, st, true, scr, nd);
  }
  mark(false, false, st);
  return {};
}

// ================================================================= PCG
PcgBuffers::PcgBuffers(int64_t n)
    : r(n * sizeof(double)), zz(n * sizeof(double)), p(n * sizeof(double)), q(n * sizeof(double)),
      Kp(n * sizeof(double)), p32(n * sizeof(float)), sc(16 * sizeof(double)) {}

Pcg::Pcg(Operator& op, Workspace& ws, int64_t n, Exec& ex) : op_(op), ws_(ws), n_(n), ex_(ex), pb_(n) {}

// Solves (K + c 1 1^T + diag(L)) x = b.  x holds the start (ignored when
// x_zero); Kx, when given, holds K x on entry (ignored when x_zero) and is
// advanced with the same steps as x, so on return Kx = K x up to rounding
// without an extra K-apply.
Co<PcgStats> Pcg::solve(double c, const double* L, Woodbury* P, const double* b, double* x, double* Kx,
                        bool x_zero, double tol, int maxit, bool fast) {
  const int64_t n = n_;
  const hipStream_t st = ex_.st;
  double* sc = pb_.sc.as<double>();
  enum { RZ0 = 0, RZ1 = 1, PQ = 2, RR = 3, SUMP = 4, SUMX = 5, TMP = 8 };
  if (x_zero) {
    fill(n, 0.0, x, st);
    if (Kx) fill(n, 0.0, Kx, st);
    pcg_init_r(n, b, nullptr, nullptr, L, c, sc, -1, pb_.r.as<double>(), ws_, sc + RR, st);
  } else {
    vec_dots(n, x, nullptr, ws_, sc + TMP, st);  // sc[TMP] = sum(x)
    const double* Kx0 = Kx;
    if (!Kx0) {
      co_await op_.apply_exact(x, pb_.Kp.as<double>(), ex_);
      Kx0 = pb_.Kp.as<double>();
    }
    pcg_init_r(n, b, x, Kx0, L, c, sc, TMP, pb_.r.as<double>(), ws_, sc + RR, st);
  }
  double rr = 0.0;
  co_await read_back(ex_, sc + RR, sizeof(double), &rr);
  PcgStats stats;
  stats.resnorm = std::sqrt(rr);
  if (!(stats.resnorm > tol)) co_return stats;
  int cur = 0;
  float* p32 = (fast && op_.materialized()) ? pb_.p32.as<float>() : nullptr;
  // zz = P^{-1} r, sc[rz_new] = r . zz, then p = zz + beta p (beta = sc[rz_new] / sc[rz_old])
  auto precond_p = [&](int rz_old, int rz_new, bool first) {
    if (P) {
      const Woodbury::PUpdate up{pb_.p.as<double>(), p32, sc, rz_old, rz_new, SUMP, first};
      P->apply(pb_.r.as<double>(), pb_.zz.as<double>(), pb_.r.as<double>(), sc + rz_new, ws_, st, &up);
    } else {
      copy_dot(n, pb_.r.as<double>(), pb_.zz.as<double>(), ws_, sc + rz_new, st);
      pcg_update_p(n, pb_.zz.as<double>(), pb_.p.as<double>(), p32, sc, rz_old, rz_new, first, ws_, sc + SUMP, st);
    }
  };
  // In a batch whose launcher runs the rest of the iteration after the K-apply
  // (pstep.h), the iteration is one request: K p, then q, x, r, K x and, before
  // this fit has read rr, the preconditioner and the direction update (dropped
  // when the solve stops here).  Same kernel bodies, same results.
  PcgStepDesc step;
  const bool batched_step = fast && P && op_.steps_batched(ex_) && P->step_desc(step);
  if (batched_step) {
    step.n = n;
    step.Kp = pb_.Kp.as<double>();
    step.L = L;
    step.c = c;
    step.sc = sc;
    step.sump = SUMP;
    step.pq = PQ;
    step.rr = RR;
    step.q = pb_.q.as<double>();
    step.x = x;
    step.r = pb_.r.as<double>();
    step.Kx = Kx;
    step.p = pb_.p.as<double>();
    step.p32 = p32;
    step.zz = pb_.zz.as<double>();
    step.nred = int(red_shape(n).blocks);
    step.partials = ws_.partials;
    // resumed only after the launch has completed: (p . q, r . r) come with it
    if (ex_.sched->complete_on_resume()) step.status = ex_.hbuf.as<double>();
  }
  precond_p(RZ0, RZ0, true);
  for (int it = 1; it <= maxit; ++it) {
    if (batched_step) {
      step.rz = cur == 0 ? RZ0 : RZ1;
      step.rz_new = cur == 0 ? RZ1 : RZ0;
      if (step.status) step.status[2] = 0.0;  // the launch sets it when this fit's step is complete
      // from the second iteration on, nothing of this solve runs on the fit's
      // stream between two batched steps (the status comes in host memory)
      co_await op_.apply_fast_step(pb_.p.as<double>(), pb_.Kp.as<double>(), &step, it > 1 && step.status, ex_);
    } else {
      if (fast) co_await op_.apply_fast(pb_.p.as<double>(), p32, pb_.Kp.as<double>(), ex_);
      else co_await op_.apply_exact(pb_.p.as<double>(), pb_.Kp.as<double>(), ex_);
      pcg_qxr(n, pb_.Kp.as<double>(), pb_.p.as<double>(), L, c, sc, SUMP, cur == 0 ? RZ0 : RZ1, PQ, RR,
              pb_.q.as<double>(), x, pb_.r.as<double>(), Kx, ws_, st);
    }
    double two[2];
    if (batched_step && step.status) memcpy(two, step.status, sizeof(two));
    else co_await read_back(ex_, sc + PQ, 2 * sizeof(double), two);  // [PQ, RR]
    stats.iters = it;
    stats.resnorm = std::sqrt(std::max(two[1], 0.0));
    if (!(two[0] > 0.0)) {  // curvature lost: the step just taken is unreliable, stop here
      stats.breakdown = true;
      break;
    }
    if (stats.resnorm <= tol) break;
    const int nxt = 1 - cur;
    if (!batched_step) precond_p(cur == 0 ? RZ0 : RZ1, nxt == 0 ? RZ0 : RZ1, false);
    cur = nxt;
  }
  co_return stats;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ================================================================= solver
Solver::Solver(Operator& op, Exec& ex, const double* y, int64_t n, double tau, double lam, const kqr_options& o,
               const float* F, int64_t rank, int64_t ldf)
    : op_(op), ex_(ex), y_(y), n_(n), tau_(tau), lam_(lam), o_(o), st_(ex.st), ws_(ex.st), pcg_(op, ws_, n, ex),
      alpha_(n * sizeof(double)), v_(n * sizeof(double)), z_(n * sizeof(double)), Ka_(n * sizeof(double)),
      b_(n * sizeof(double)), L_(n * sizeof(double)), grad_(n * sizeof(double)), d_(n * sizeof(double)),
      Kd_(n * sizeof(double)), S_(n), red_(64 * sizeof(double)) {
  if (rank > 0) P_.reset(new Woodbury(F, n, rank, ldf));
  eps_floor_ = o.eps_floor;
}

Co<Unit> Solver::init() {
  double t3[3];
  vec_dots(n_, y_, nullptr, ws_, red_.as<double>(), st_);
  co_await read_back(ex_, red_.as<double>(), 3 * sizeof(double), t3);
  ynorm_ = std::sqrt(t3[2]);
  if (!std::isfinite(ynorm_)) fail(KQR_ENUMERIC, "y contains NaN or Inf");
  t_start_ = now_s();
  co_return Unit{};
}

void Solver::record(int phase, int it, double err) {
  if (!o_.trace || ntrace_ >= o_.trace_cap) return;
  double* r = o_.trace + 4 * int64_t(ntrace_);
  r[0] = phase;
  r[1] = it;
  r[2] = err;
  r[3] = now_s() - t_start_;
  ++ntrace_;
}

// Section 4 stopping measures from the sums of multiplier_kkt (FP64):
// s = [||r_p||^2, ||alpha - v||^2, ||alpha||^2, ||v - Pi_B(z + v)||^2, ||v||^2,
//      rho_tau(z), alpha^T K alpha, y^T alpha, 1^T alpha].
Kkt kkt_from_sums(const double* s, double ynorm, double lam) {
  Kkt k;
  k.eta_p = std::sqrt(std::max(s[0], 0.0)) / (1.0 + ynorm);
  k.eta_d = std::sqrt(s[8] * s[8] + std::max(s[1], 0.0)) / (1.0 + std::sqrt(std::max(s[2], 0.0)));
  k.eta_c = std::sqrt(std::max(s[3], 0.0)) / (1.0 + std::sqrt(std::max(s[4], 0.0)));
  k.obj_p = s[5] + s[6] / (2.0 * lam);
  k.obj_d = -s[6] / (2.0 * lam) + s[7];
  k.eta_gap = std::fabs(k.obj_p - k.obj_d) / (1.0 + std::fabs(k.obj_p) + std::fabs(k.obj_d));
  k.eta_kkt = std::max(k.eta_p, std::max(k.eta_d, k.eta_c));
  k.err = std::max(k.eta_kkt, k.eta_gap);
  k.sum_alpha = s[8];
  return k;
}

Kkt Solver::kkt_from_sums(const double* s) const { return ::kqr::kkt_from_sums(s, ynorm_, lam_); }

Co<double> Solver::sum_of(const double* x) {
  double t3[3];
  vec_dots(n_, x, nullptr, ws_, red_.as<double>(), st_);
  co_await read_back(ex_, red_.as<double>(), 3 * sizeof(double), t3);
  co_return t3[0];
}

Co<Kkt> Solver::update_and_kkt(double beta_new, double sigma, double step, bool update) {
  double s[kKktSums];
  multiplier_kkt(n_, alpha_.as<double>(), Ka_.as<double>(), y_, z_.as<double>(), v_.as<double>(), beta_new, sigma,
                 step, tau_, lam_, update, ws_, red_.as<double>(), st_);
  co_await read_back(ex_, red_.as<double>(), kKktSums * sizeof(double), s);
  co_return kkt_from_sums(s);
}

// Linear solve of (K + c 1 1^T + diag(L)) x = b to ||b - A x|| <= tol, with K x
// kept in Kx.  With an FP32 (or on-the-fly) operator, or when refine is off,
// this is PCG on the fast operator itself.  With BF16 storage and refine on it
// is iterative refinement: the residual r = b - A x is formed with the exact
// operator (FP32 entries, stored or recomputed from X, FP64 vectors and sums),
// PCG on the BF16 operator solves A_bf16 dx = r to a relative accuracy matched
// to the contraction the previous step achieved, x += dx and K x += K_exact dx.
// When a refinement step fails to reduce the exact residual by a tenth, the
// solve finishes with PCG on the exact operator.
Co<PcgStats> Solver::linsolve(double c, const double* L, const double* b, double* x, double* Kx, bool x_zero,
                              double tol, bool refine, kqr_info& info) {
  if (!(refine && op_.materialized() && op_.kmat().dtype == KQR_BF16 && o_.refine)) {
    co_return co_await pcg_.solve(c, L, P_.get(), b, x, Kx, x_zero, tol, o_.pcg_max_iter, true);
  }
  const int64_t n = n_;
  if (!rf_r_.ptr) {
    rf_r_.alloc(size_t(n) * sizeof(double));
    rf_dx_.alloc(size_t(n) * sizeof(double));
    rf_kdx_.alloc(size_t(n) * sizeof(double));
  }
  double* r = rf_r_.as<double>();
  double* dx = rf_dx_.as<double>();
  double* kdx = rf_kdx_.as<double>();
  if (x_zero) {
    fill(n, 0.0, x, st_);
    fill(n, 0.0, Kx, st_);
  }
  double sums[3];
  auto residual = [&]() -> Co<double> {  // r = b - (Kx + c sum(x) + L x); returns ||r||
    vec_dots(n, x, nullptr, ws_, red_.as<double>(), st_);
    pcg_init_r(n, b, x, Kx, L, c, red_.as<double>(), 0, r, ws_, red_.as<double>() + 8, st_);
    co_await read_back(ex_, red_.as<double>() + 8, sizeof(double), sums);
    co_return std::sqrt(std::max(sums[0], 0.0));
  };
  PcgStats total;
  double rn = co_await residual();
  total.resnorm = rn;
  // relative accuracy of the inner solve: solving far below the contraction
  // the BF16 operator allows only costs iterations
  double inner_rel = 0.05;
  for (int step = 0; step < 30 && rn > tol; ++step) {
    const double inner_tol = std::max(0.5 * tol, inner_rel * rn);
    PcgStats ps = co_await pcg_.solve(c, L, P_.get(), r, dx, nullptr, true, inner_tol, o_.pcg_max_iter, true);
    total.iters += ps.iters;
    co_await op_.apply_exact(dx, kdx, ex_);
    axpy2(n, 1.0, dx, x, kdx, Kx, st_);
    ++info.refinements;
    const double rn_new = co_await residual();
    total.resnorm = rn_new;
    const bool stalled = !(rn_new < 0.9 * rn);
    inner_rel = std::min(0.3, std::max(0.05, 0.5 * rn_new / rn));
    rn = rn_new;
    if (stalled && rn > tol) {  // BF16 operator too far from the exact one here
      PcgStats pe = co_await pcg_.solve(c, L, P_.get(), b, x, Kx, false, tol, o_.pcg_max_iter, false);
      total.iters += pe.iters;
      total.resnorm = pe.resnorm;
      // exact K x after the exact solve (Kx was advanced with exact products)
      break;
    }
  }
  co_return total;
}

// Algorithm 1.  M = K + lambda sigma (I + 1 1^T) is fixed, so the Woodbury
// core (L = lambda sigma I) is formed once.
Co<Unit> Solver::phase1(kqr_info& info) {
  const double t0 = now_s();
  const int64_t n = n_;
  const double sigma = o_.admm_sigma, step = o_.admm_step, c = lam_ * sigma;
  fill(n, c, L_.as<double>(), st_);
  if (P_) {
    // a core breakdown (rounding, the core being near singular) is retried
    // with the low-rank part of P shrunk by 1e2, 1e4, 1e6: P stays
    // symmetric positive definite, only a weaker preconditioner
    bool ok = co_await P_->build_scaled_identity(L_.as<double>(), c, c, ex_);
    for (int k = 1; !ok && k <= 3; ++k) {
      ++info.core_retries;
      ok = co_await P_->build_scaled_identity(L_.as<double>(), c, c, ex_, std::pow(10.0, 2.0 * k));
    }
    if (!ok) fail(KQR_ENUMERIC, "ADMM preconditioner core not positive definite");
  }
  fill(n, 0.0, alpha_.as<double>(), st_);
  fill(n, 0.0, v_.as<double>(), st_);
  fill(n, 0.0, z_.as<double>(), st_);
  fill(n, 0.0, Ka_.as<double>(), st_);
  beta_ = 0.0;
  double b0 = 0.0;
  Kkt k;
  int it = 0;
  for (it = 0; it < o_.admm_max_iter; ++it) {
    admm_rhs(n, y_, z_.as<double>(), v_.as<double>(), beta_, sigma, lam_, b_.as<double>(), st_);
    if (it == 0) {
      double t3[3];
      vec_dots(n, b_.as<double>(), nullptr, ws_, red_.as<double>(), st_);
      co_await read_back(ex_, red_.as<double>(), 3 * sizeof(double), t3);
      b0 = std::sqrt(t3[2]);
    }
    const double eps_k = o_.admm_eps0 * b0 / std::pow(double(it + 1), 1.5);
    // Phase I is a warm start: with BF16 storage it runs on the BF16 operator
    // alone (K alpha is recomputed exactly when Phase II starts)
    PcgStats ps = co_await linsolve(c, L_.as<double>(), b_.as<double>(), alpha_.as<double>(), Ka_.as<double>(),
                                    it == 0, eps_k, false, info);
    info.admm_pcg_iters += ps.iters;
    const double sa = co_await sum_of(alpha_.as<double>());
    const double beta_new = beta_ + step * sigma * sa;
    k = co_await update_and_kkt(beta_new, sigma, step, true);
    beta_ = beta_new;
    if (o_.verbose)
      fprintf(stderr, "[kqr] admm %3d pcg %3d eta_p %.2e eta_d %.2e eta_c %.2e gap %.2e\n", it + 1, ps.iters,
              k.eta_p, k.eta_d, k.eta_c, k.eta_gap);
    if (!std::isfinite(k.err)) fail(KQR_ENUMERIC, "non-finite residual in Phase I");
    if (k.err <= o_.admm_tol && o_.admm_tol <= o_.tol) {
      // Phase I is the whole solve here: confirm with an exact K alpha (the
      // tracked products carry FP32 rounding) before stopping
      co_await op_.apply_exact(alpha_.as<double>(), Ka_.as<double>(), ex_);
      k = co_await update_and_kkt(beta_, sigma, step, false);
    }
    record(1, it + 1, k.err);
    if (k.err <= o_.admm_tol) { ++it; break; }
  }
  info.admm_iters = it;
  sigma_ = sigma;
  eta_d_prev_ = k.eta_d;
  last_ = k;
  info.t_admm = now_s() - t0;  // the last read-back drained the stream
  co_return Unit{};
}

// Warm start: Algorithm 2 begins from the iterate Phase I hands over; here
// that iterate is given (e.g. a fit stopped at a looser tolerance), so Phase I
// is skipped.  K alpha is formed exactly and the Section 4 measures of the
// given point seed the subproblem accuracy of the first outer iteration.
Co<Unit> Solver::warm_start(kqr_info& info) {
  const int64_t n = n_;
  copy(n, o_.warm_alpha, alpha_.as<double>(), st_);
  copy(n, o_.warm_v, v_.as<double>(), st_);
  copy(n, o_.warm_z, z_.as<double>(), st_);
  beta_ = o_.warm_beta;
  sigma_ = o_.warm_sigma > 0.0 ? o_.warm_sigma : o_.admm_sigma;
  co_await op_.apply_exact(alpha_.as<double>(), Ka_.as<double>(), ex_);
  last_ = co_await update_and_kkt(beta_, sigma_, 1.0, false);
  if (!std::isfinite(last_.err)) fail(KQR_ENUMERIC, "non-finite residual at the warm start");
  eta_d_prev_ = last_.eta_d;
  info.admm_iters = 0;
  co_return Unit{};
}

// Algorithm 3 on phi_k for the current (beta, z, sigma).
Co<Unit> Solver::ssn(double stop, kqr_info& info) {
  const int64_t n = n_;
  const double sigma = sigma_, c1 = lam_ * sigma;
  for (int t = 0; t < o_.ssn_max_iter; ++t) {
    const double sa = co_await sum_of(alpha_.as<double>());
    ssn_grad(n, alpha_.as<double>(), Ka_.as<double>(), y_, z_.as<double>(), beta_, sigma, sa, tau_, lam_,
             grad_.as<double>(), S_.as<uint8_t>(), ws_, red_.as<double>(), st_);
    double gg = 0.0;
    co_await read_back(ex_, red_.as<double>(), sizeof(double), &gg);
    const double gn = std::sqrt(gg);
    if (!std::isfinite(gn)) fail(KQR_ENUMERIC, "non-finite gradient in SSN");
    if (gn <= stop) break;
    double eps_t = std::max(o_.tau1 * std::min(o_.tau2, gn), eps_floor_);
    ssn_system(n, S_.as<uint8_t>(), grad_.as<double>(), lam_, sigma, eps_t, L_.as<double>(), b_.as<double>(), st_);
    if (P_) {
      // a core breakdown: the interior diagonal lambda eps_t is too small for
      // the core in FP64; raise the eps_t floor 100-fold (for the rest of the
      // fit) and form the Newton system again, up to four times
      bool ok = co_await P_->build_two_level(L_.as<double>(), S_.as<uint8_t>(), lam_ * eps_t,
                                             lam_ * sigma + lam_ * eps_t, c1, ex_);
      for (int k = 0; !ok && k < 4; ++k) {
        ++info.core_retries;
        eps_floor_ = std::max(100.0 * eps_t, 1e-10);
        eps_t = std::max(eps_t, eps_floor_);
        ssn_system(n, S_.as<uint8_t>(), grad_.as<double>(), lam_, sigma, eps_t, L_.as<double>(), b_.as<double>(),
                   st_);
        ok = co_await P_->build_two_level(L_.as<double>(), S_.as<uint8_t>(), lam_ * eps_t,
                                          lam_ * sigma + lam_ * eps_t, c1, ex_);
      }
      if (!ok) fail(KQR_ENUMERIC, "Newton preconditioner core not positive definite");
    }
    const double tol = lam_ * std::min(o_.etabar, std::pow(gn, 1.0 + o_.iota));
    PcgStats ps = co_await linsolve(c1, L_.as<double>(), b_.as<double>(), d_.as<double>(), Kd_.as<double>(), true,
                                    tol, true, info);
    info.pcg_iters += ps.iters;
    // Armijo backtracking, kLsTrials step lengths per pass
    const double s0 = sa + beta_ / sigma;
    double cstep = 0.0;
    double c0 = 1.0;
    int tried = 0;
    while (tried < o_.ls_max) {
      double s[5 + kLsTrials];
      line_search_sums(n, alpha_.as<double>(), z_.as<double>(), d_.as<double>(), Ka_.as<double>(), Kd_.as<double>(),
                       y_, grad_.as<double>(), sigma, tau_, c0, o_.ls_shrink, ws_, red_.as<double>(), st_);
      co_await read_back(ex_, red_.as<double>(), (5 + kLsTrials) * sizeof(double), s);
      const double dKa = s[0], dKd = s[1], yd = s[2], ed = s[3], gd = s[4];
      double cj = c0;
      bool ok = false;
      for (int j = 0; j < kLsTrials && tried < o_.ls_max; ++j, ++tried) {
        const double delta = cj * dKa / lam_ + 0.5 * cj * cj * dKd / lam_ - cj * yd +
                             0.5 * sigma * ((s0 + cj * ed) * (s0 + cj * ed) - s0 * s0) + 0.5 * sigma * s[5 + j];
        if (delta <= o_.armijo * cj * gd) { ok = true; break; }
        cj *= o_.ls_shrink;
        ++info.line_search_steps;
      }
      if (ok) { cstep = cj; break; }
      c0 = cj;
    }
    if (cstep == 0.0) cstep = c0;  // backtracking cap reached: take the last (tiny) step
    axpy2(n, cstep, d_.as<double>(), alpha_.as<double>(), Kd_.as<double>(), Ka_.as<double>(), st_);
    ++info.newton_iters;
    if (o_.verbose)
      fprintf(stderr, "[kqr]   newton %2d |grad| %.3e (stop %.1e) pcg %3d res %.2e tol %.2e step %.3g\n", t + 1, gn,
              stop, ps.iters, ps.resnorm, tol, cstep);
  }
  co_return Unit{};
}

Co<Unit> Solver::phase2(kqr_info& info) {
  const double t0 = now_s();
  // Subproblem accuracy: the summable tolerances of criterion (A) are taken
  // as a fraction of the previous outer residual, floored at the final target
  // (after the multiplier update ||grad phi_k|| = (1 + ||y||) eta_p).
  const double scale = 1.0 + ynorm_;
  Kkt k = last_;
  double e_prev = last_.err;
  int it = 0;
  bool done = false;
  if (k.err <= o_.tol) {  // Phase I already met the final target (ADMM run alone): confirm exactly
    co_await op_.apply_exact(alpha_.as<double>(), Ka_.as<double>(), ex_);
    k = co_await update_and_kkt(beta_, sigma_, 1.0, false);
    done = k.err <= o_.tol;
  }
  for (it = 0; !done && it < o_.alm_max_iter; ++it) {
    const double stop = scale * std::max(o_.ssn_rel * o_.tol, std::min(o_.ssn_adapt * e_prev, 1.0));
    co_await op_.apply_exact(alpha_.as<double>(), Ka_.as<double>(), ex_);  // reset drift of the tracked K alpha
    co_await ssn(stop, info);
    const double sa = co_await sum_of(alpha_.as<double>());
    const double beta_new = beta_ + sigma_ * sa;
    k = co_await update_and_kkt(beta_new, sigma_, 1.0, true);
    beta_ = beta_new;
    record(2, it + 1, k.err);
    if (o_.verbose)
      fprintf(stderr, "[kqr] alm %3d sigma %.1e eta_p %.2e eta_d %.2e eta_c %.2e gap %.2e\n", it + 1, sigma_,
              k.eta_p, k.eta_d, k.eta_c, k.eta_gap);
    if (!std::isfinite(k.err)) fail(KQR_ENUMERIC, "non-finite residual in Phase II");
    if (k.err <= o_.tol) {
      // confirm with an exact K alpha (tracked products drift by rounding)
      co_await op_.apply_exact(alpha_.as<double>(), Ka_.as<double>(), ex_);
      k = co_await update_and_kkt(beta_, sigma_, 1.0, false);
      if (k.err <= o_.tol) { ++it; done = true; break; }
    }
    if (k.eta_d > o_.sigma_stall * eta_d_prev_) sigma_ = std::min(o_.sigma_factor * sigma_, o_.sigma_max);
    eta_d_prev_ = k.eta_d;
    e_prev = k.err;
  }
  info.alm_iters = it;
  converged_ = done;
  last_ = k;
  info.t_alm = now_s() - t0;  // the last read-back drained the stream
  co_return Unit{};
}

Co<Unit> Solver::finish(kqr_info& info) {
  // final residuals with the exact operator
  co_await op_.apply_exact(alpha_.as<double>(), Ka_.as<double>(), ex_);
  Kkt k = co_await update_and_kkt(beta_, sigma_, 1.0, false);
  last_ = k;
  info.eta_p = k.eta_p;
  info.eta_d = k.eta_d;
  info.eta_c = k.eta_c;
  info.eta_kkt = k.eta_kkt;
  info.eta_gap = k.eta_gap;
  info.obj_p = k.obj_p;
  info.obj_d = k.obj_d;
  info.sigma = sigma_;
  info.trace_len = ntrace_;
  count_interior(n_, alpha_.as<double>(), tau_, ws_, red_.as<double>(), st_);
  double ni = 0.0;
  co_await read_back(ex_, red_.as<double>(), sizeof(double), &ni);
  info.n_interior = int64_t(ni);
  converged_ = converged_ && k.err <= o_.tol;
  co_return Unit{};
}

}  // namespace kqr
