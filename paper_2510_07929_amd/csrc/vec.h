// Solver-level declarations: vector kernels, the Woodbury preconditioner and
// randomly pivoted Cholesky.
#pragma once

#include "coro.h"
#include "pstep.h"

namespace kqr {

constexpr int kKktSums = 9;    // sums produced by multiplier_kkt
constexpr int kLsTrials = 24;  // step lengths evaluated per line-search pass
constexpr int kMaxPartialQ = 5 + kLsTrials;

// Scratch shared by the reduction kernels of one solve (per-block partial
// sums).  Kernels using one Workspace must be ordered (one stream).
struct Workspace {
  DevBuf part_buf;  // kRedBlocks * kMaxPartialQ doubles
  double* partials = nullptr;
  explicit Workspace(hipStream_t st) : part_buf(size_t(kRedBlocks) * kMaxPartialQ * sizeof(double)) {
    (void)st;
    partials = part_buf.as<double>();
  }
};

// ----------------------------------------------------------------- vector kernels (vec.hip)
void vec_dots(int64_t n, const double* x, const double* y, Workspace& ws, double* out3, hipStream_t st);
void pcg_init_r(int64_t n, const double* b, const double* x, const double* Kx, const double* L, double c,
                const double* sc, int sum_x_slot, double* r, Workspace& ws, double* rr_out, hipStream_t st);
void pcg_update_p(int64_t n, const double* zz, double* p, float* p32, const double* sc, int rz_slot,
                  int rzn_slot, bool first, Workspace& ws, double* sump_out, hipStream_t st);
void pcg_q(int64_t n, const double* Kp, const double* p, const double* L, double c, const double* sc,
           int sump_slot, double* q, Workspace& ws, double* pq_out, hipStream_t st);
void pcg_xr(int64_t n, const double* p, const double* q, const double* Kp, double* x, double* r, double* Kx,
            const double* sc, int rz_slot, int pq_slot, Workspace& ws, double* rr_out, hipStream_t st);
// pcg_q then pcg_xr (sc[pq_slot] and sc[rr_slot] written); one launch when
// n <= kOneBlockN.
void pcg_qxr(int64_t n, const double* Kp, const double* p, const double* L, double c, double* sc, int sump_slot,
             int rz_slot, int pq_slot, int rr_slot, double* q, double* x, double* r, double* Kx, Workspace& ws,
             hipStream_t st);
void admm_rhs(int64_t n, const double* y, const double* z, const double* v, double beta, double sigma,
              double lam, double* b, hipStream_t st);
void multiplier_kkt(int64_t n, const double* alpha, const double* Ka, const double* y, double* z, double* v,
                    double beta_new, double sigma, double step, double tau, double lam, bool update,
                    Workspace& ws, double* out, hipStream_t st);
void ssn_grad(int64_t n, const double* alpha, const double* Ka, const double* y, const double* z, double beta,
              double sigma, double sum_alpha, double tau, double lam, double* grad, uint8_t* S, Workspace& ws,
              double* gg_out, hipStream_t st);
void ssn_system(int64_t n, const uint8_t* S, const double* grad, double lam, double sigma, double eps_t,
                double* L, double* rhs, hipStream_t st);
void line_search_sums(int64_t n, const double* alpha, const double* z, const double* d, const double* Ka,
                      const double* Kd, const double* y, const double* grad, double sigma, double tau,
                      double c0, double shrink, Workspace& ws, double* out, hipStream_t st);
void axpy2(int64_t n, double c, const double* d, double* x, const double* Kd, double* Kx, hipStream_t st);
void count_nonfinite(int64_t n, const double* x, Workspace& ws, double* out, hipStream_t st);
void count_interior(int64_t n, const double* a, double tau, Workspace& ws, double* out, hipStream_t st);
void fill(int64_t n, double val, double* x, hipStream_t st);
void copy(int64_t n, const double* src, double* dst, hipStream_t st);

// ----------------------------------------------------------------- dense SPD (woodbury.hip)
// In place Cholesky C = Lc Lc^T of the lower triangle of an m x m FP64 matrix
// (leading dimension ldc), then W = Lc^{-1} and WT = W^T (both m x ldc; T is
// scratch of the same size).  *flag (device) becomes nonzero on a
// non-positive pivot.  Asynchronous.
void spd_factor_inverse(double* C, int64_t ldc, int m, double* W, double* WT, double* T, int* flag, hipStream_t st);
// idx[0..m) = increasing indices i with S[i] != 0; returns m (synchronises).
// cnt: device scratch of 257 ints.
int64_t index_list(const uint8_t* S, int64_t n, int* idx, int* cnt, hipStream_t st);
// s = C^{-1} t = W^T (W t); y is scratch of m doubles.
void spd_solve(const double* W, const double* WT, int64_t ldc, int m, const double* t, double* y, double* s,
               hipStream_t st);

// ----------------------------------------------------------------- Woodbury (woodbury.hip)
// P = F F^T + c 1 1^T + diag(L), applied by Lemma 1 with the (r+1)^2 core in FP64.
class Woodbury {
 public:
  Woodbury(const float* F, int64_t n, int64_t r, int64_t ldf);
  // Forms C = diag(I, 1/c) + U^T L^{-1} U for a general positive diagonal L,
  // factors it and forms W = Lc^{-1}.  Returns false when a pivot is not
  // positive (the factor is then unusable).
  Co<bool> build(const double* L, double c, Exec& ex);
  // Same for L = l I (Phase I), from the Gram matrix U^T U formed once;
  // shrink > 1 scales the low-rank part of P by 1 / shrink (the core's
  // diag(I, 1/c) by shrink).
  Co<bool> build_scaled_identity(const double* L, double l, double c, Exec& ex, double shrink = 1.0);
  // Same for the Newton systems: L_i = l_in where S_i = 1, l_out elsewhere.
  Co<bool> build_two_level(const double* L, const uint8_t* S, double l_in, double l_out, double c, Exec& ex);
  // out = P^{-1} w.  When dot_with != nullptr also writes dot_with . out to *dot_out (device).
  // With up (PCG's direction update after the preconditioner), also runs
  // pcg_update_p(out, up->p, ..., old slot, new slot = the slot of dot_out)
  // -- in the same launch as the last step when n <= kOneBlockN.
  struct PUpdate {
    double* p;
    float* p32;
    double* sc;
    int rz_old, rz_new, sump;
    bool first;
  };
  void apply(const double* w, double* out, const double* dot_with, double* dot_out, Workspace& ws,
             hipStream_t st, const PUpdate* up = nullptr);
  int64_t rank() const { return r_; }
  // The preconditioner's part of a batched PCG step (pstep.h): false when the
  // apply does not fit that form (n > kOneBlockN, r + 1 > kFusedCore).
  bool step_desc(PcgStepDesc& d) const;
  // Lower triangle of [F 1]^T [F 1] ((r+1) x (r+1), leading dimension r+1).
  const double* gram(hipStream_t st) {
    prepare_gram(st);
    return G_.as<double>();
  }

 private:
  void syrk(const double* L, const int* idx, int64_t nrows, double* G, double alpha, double beta, double diag_r,
            double diag_last, double* out, hipStream_t st);
  Co<bool> factor(Exec& ex);
  void prepare_gram(hipStream_t st);
  const float* F_;
  int64_t n_, r_, ldf_, R1_;
  int64_t ldc_;
  const double* L_ = nullptr;
  DevBuf C_, W_, WT_, T_, G_, part_, g_, Fs_, t_, y_, s_, flag_, idx_, cnt_;
  int nsplit_ = 1;
};

// Test hook (kqr_test_core_breakdowns): after `skip` more core
// factorisations, the next `count` report a non-positive pivot.
void set_forced_core_breakdowns(int skip, int count);

// ----------------------------------------------------------------- RPCholesky (rpchol.hip)
// Randomly pivoted Cholesky on K (materialised or from X).  Writes F (n x ldf
// FP32) and returns the pivots; stops early when sum(d) <= 1e-14 tr(K).
Co<std::vector<int64_t>> rpcholesky(KMat km, const float* X, const float* sqn, int64_t n, int p,
                                    KernelSpec ks, int64_t rank, const double* uniforms, float* F, int64_t ldf,
                                    Exec& ex);
// Rank heuristic of Section 3 on the r0 columns of F0: smallest r with
// lambda_r(F0^T F0) <= xi lambda_1 (r0 when none); lambda_1 optional output.
Co<int64_t> adaptive_rank(const float* F0, int64_t n, int64_t r0, int64_t ldf, double xi, Exec& ex,
                          double* lambda1_out);

}  // namespace kqr
