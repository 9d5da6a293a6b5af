/*
 * kqr.h -- C ABI of libkqr, an MI355X (gfx950) implementation of the hot path
 * of PALM-KQR, the two-phase preconditioned augmented Lagrangian method for
 * kernel quantile regression (Deng, Li, Zhang).
 *
 * Problem (Section 1, (1.1)-(1.3)): given X (n x p), y (n), quantile level
 * tau in (0,1), lambda > 0 and a kernel k (RBF exp(-gamma ||x-x'||_2^2) or
 * Laplacian exp(-gamma ||x-x'||_1)), find the dual optimum alpha of
 *     max  -alpha^T K alpha / (2 lambda) + y^T alpha
 *     s.t. alpha in [tau-1, tau]^n,  1^T alpha = 0,
 * and the intercept beta.  The fitted function is
 *     f(x) = beta + sum_j alpha_j k(x_j, x) / lambda
 * (representer form of Section 1 with theta = alpha at the optimum).
 *
 * Conventions shared by every entry point:
 *  - Pointers documented as "device" must point to device memory of the
 *    current HIP device; "host" pointers to host memory.  The caller owns all
 *    buffers passed in; the library never frees them.
 *  - Matrices are row-major.  A leading dimension (ld*) counts elements.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    kqr_kernel_build, kqr_kernel_apply and kqr_predict only enqueue work on
 *    `stream` and return; every other entry point synchronises `stream`
 *    before it returns.
 *  - Arguments are validated before any device work.  Invalid arguments give
 *    KQR_EINVAL and leave every output untouched.  Calls never throw.
 *  - On a negative status the contents of outputs are undefined.  On
 *    KQR_NOT_CONVERGED outputs hold the last iterate and `info` is filled.
 *  - kqr_last_error() returns a message describing the last failure on the
 *    calling thread.
 */
#ifndef KQR_H
#define KQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
  KQR_OK = 0,
  KQR_NOT_CONVERGED = 1, /* outputs valid, tolerance not reached */
  KQR_EINVAL = -1,       /* invalid argument */
  KQR_ENOMEM = -2,       /* device allocation failed */
  KQR_ENODEVICE = -3,    /* no HIP device available */
  KQR_EHIP = -4,         /* HIP runtime error */
  KQR_ENUMERIC = -5      /* NaN/Inf in inputs or a numerical breakdown */
};

/* kernels: RBF exp(-gamma ||x - x'||_2^2) and Laplacian exp(-gamma ||x - x'||_1)
 * (Section 1); linear x^T x' (Table 2; gamma unused, pass any positive value).
 * The linear kernel is never materialised: K v = X (X^T v) in FP64 on the FP32
 * entries of X, and the preconditioner factor is X itself (K = X X^T has
 * rank <= p, so RPCholesky would return X's column space exactly after p
 * steps).  Entry points that take a materialised K, RPCholesky and the
 * gradient (K_EE is singular once |E| > p) reject it with KQR_EINVAL. */
enum { KQR_RBF = 0, KQR_LAPLACIAN = 1, KQR_LINEAR = 2 };

/* storage type of a materialised kernel matrix */
enum { KQR_FP32 = 0, KQR_BF16 = 1 };

/* how kqr_fit obtains K */
enum {
  KQR_KMODE_AUTO = 0,        /* materialise if it fits in device memory */
  KQR_KMODE_MATERIALIZE = 1, /* always materialise (k_dtype storage) */
  KQR_KMODE_ON_THE_FLY = 2   /* recompute entries from X on every apply */
};

/* arithmetic of kqr_kernel_apply */
enum {
  KQR_APPLY_FAST = 0, /* V rounded to FP32, FP32 products, FP64 sums per segment */
  KQR_APPLY_EXACT = 1, /* V in FP64, products and sums in FP64 (K entries as stored) */
  KQR_APPLY_KV = 2     /* kqr_autotune_apply only: the multi-column K V launch on the matrix cores */
};

/* ---------------------------------------------------------------- options
 * Algorithm constants of Algorithms 1-3 and Section 4.  The paper fixes their
 * ranges, not their values; kqr_default_options fills the values the library
 * uses (each listed next to its field). */
typedef struct kqr_options {
  double tol;          /* Phase II stop: max(eta_kkt, eta_gap) <= tol (Section 4); 1e-6 */
  double admm_tol;     /* Phase I stop (Section 4); 1e-3 */
  int admm_max_iter;   /* Phase I cap (Section 4); 100 */
  int alm_max_iter;    /* Phase II cap (Section 4); 1000 */
  double admm_sigma;   /* sigma of Algorithm 1; 1 */
  double admm_step;    /* step length of Algorithm 1, in (0, (1+sqrt 5)/2); 1.618 */
  double admm_eps0;    /* eps_k = admm_eps0 ||b_0|| / (k+1)^1.5; 0.1 */
  double etabar;       /* Algorithm 3; 0.1 */
  double iota;         /* Algorithm 3; 0.5 */
  double armijo;       /* mu of Algorithm 3; 1e-4 */
  double ls_shrink;    /* r of Algorithm 3; 0.5 */
  int ls_max;          /* backtracking cap; 40 */
  double tau1, tau2;   /* eps_t = tau1 min(tau2, ||grad phi||); 0.1, 0.1 */
  double eps_floor;    /* lower bound of eps_t; 1e-12 */
  int ssn_max_iter;    /* Newton steps per ALM subproblem; 50 */
  double ssn_rel;      /* SSN stop ||grad phi|| <= ssn_rel tol (1+||y||); 0.5 */
  double sigma_factor; /* sigma <- min(sigma_factor sigma, sigma_max) ... ; 5 */
  double sigma_stall;  /* ... when eta_d > sigma_stall * previous eta_d; 0.25 */
  double sigma_max;    /* 1e8 */
  int rank;            /* preconditioner rank: >0 fixed, 0 adaptive (Section 3), <0 none; 0 */
  double xi;           /* adaptive-rank threshold (Section 3); 1e-7 */
  int pcg_max_iter;    /* per linear solve; 2000 */
  int k_dtype;         /* KQR_FP32 or KQR_BF16 storage of a materialised K; KQR_FP32 */
  int kmode;           /* KQR_KMODE_*; KQR_KMODE_AUTO */
  int refine;          /* BF16 K: 1 = every Phase II linear system is refined with FP64 residuals of the
                          exact operator (Phase I, a warm start, runs on the BF16 operator alone and
                          K alpha is recomputed exactly when Phase II starts); 1 */
  const double* pivot_uniforms; /* host, >= max(rank, ceil(sqrt n)) uniforms in [0,1) that
                                   drive RPCholesky's pivot draws; NULL = derive from `seed` */
  uint64_t seed;       /* used when pivot_uniforms is NULL; 0 */
  int verbose;         /* 1: one line per outer iteration on stderr; 0 */
  int profile;         /* 1: time every K-apply kernel with HIP events (kqr_info.t_kapply_*); 0 */
  int exact_k;         /* BF16 storage: source of the exact operator of the residuals and refinement.
                          0 = FP32 entries recomputed from X on every exact apply (no extra memory);
                          1 = an FP32 copy of K kept beside the BF16 one (n*ld*4 more bytes, streamed). 0 */
  double ssn_adapt;    /* Phase II subproblem accuracy (the summable tolerances of Algorithm 2's
                          criterion (A)): SSN of outer iteration k stops at ||grad phi_k|| <=
                          (1+||y||) max(ssn_rel tol, min(ssn_adapt e_{k-1}, 1)), e_{k-1} =
                          max(eta_kkt, eta_gap) of the previous outer iterate (Phase I's for k = 0);
                          0 = always ssn_rel tol.  0.3 */
  double* trace;       /* host, 4 * trace_cap doubles, or NULL: kqr_fit and kqr_fit_grad write one
                          record per outer iteration (Phase I ADMM iteration, Phase II ALM
                          iteration): {phase (1 or 2), iteration, max(eta_kkt, eta_gap) at that
                          iterate, seconds since the fit started}; records beyond trace_cap are
                          dropped.  The batched entry points ignore it.  NULL */
  int trace_cap;       /* records trace holds; 0 */
  int k_layout;        /* storage of a materialised K: 0 = full n x ld rows; 1 = K's symmetry used:
                          only the upper triangle of 128 x 128 tiles is stored (about half the
                          bytes, so half the HBM traffic per K-apply; see kqr_kernel_build_packed).
                          kqr_fit and kqr_fit_grad only; the joint and batched fits need 0.  0 */
  double* z_out;       /* device n FP64 or NULL: kqr_fit writes the final multipliers z of (1.4)
                          (the primal residual vector of Section 4).  NULL */
  double* v_out;       /* device n FP64 or NULL: kqr_fit writes the final consensus vector v of (1.4),
                          so that (alpha, v, beta, z) is the iterate the Section 4 measures in
                          kqr_info were taken at.  NULL */
  /* Warm start (resume): with warm_alpha non-NULL, kqr_fit and kqr_fit_grad skip
     Phase I and start Phase II (Algorithm 2) from (alpha, v, beta, z, sigma), the
     hand-off Algorithm 2 takes from Phase I -- e.g. the alpha, v_out, beta, z_out
     and kqr_info.sigma of an earlier fit of the same problem.  The batched entry
     points reject it (KQR_EINVAL). */
  const double* warm_alpha; /* device n FP64 or NULL (no warm start).  NULL */
  const double* warm_v;     /* device n FP64, required with warm_alpha.  NULL */
  const double* warm_z;     /* device n FP64, required with warm_alpha.  NULL */
  double warm_beta;         /* intercept of the warm start.  0 */
  double warm_sigma;        /* ALM penalty to resume with (> 0), or 0 = admm_sigma.  0 */
} kqr_options;

/* ---------------------------------------------------------------- report */
typedef struct kqr_info {
  double eta_p, eta_d, eta_c, eta_kkt, eta_gap; /* Section 4, exact K */
  double obj_p, obj_d;
  double sigma;                 /* final ALM penalty */
  int admm_iters, alm_iters, newton_iters, line_search_steps;
  int admm_pcg_iters, pcg_iters;
  int rank_used;
  int refinements;              /* BF16 outer refinement steps */
  int64_t kapply_calls;         /* K-applies of the whole fit (all precisions) */
  int64_t n_interior;           /* #{i : tau-1 < alpha_i < tau} */
  double t_kbuild, t_precond, t_admm, t_alm, t_total; /* seconds */
  /* with opt->profile: summed device time of the K-apply kernels (seconds) */
  int64_t kapply_fast_calls, kapply_exact_calls;
  double t_kapply_fast, t_kapply_exact;
  int trace_len;                /* records written to opt->trace */
  int core_retries;             /* Woodbury core factorisations repeated after a breakdown (a non-positive
                                   pivot): Newton systems with a 100x larger eps_t floor, the Phase I core
                                   with its low-rank part shrunk (both keep P symmetric positive definite) */
} kqr_info;

/* Fills *opt with the defaults listed above.  Returns KQR_OK or KQR_EINVAL (opt NULL). */
int kqr_default_options(kqr_options* opt);

/* Static text for a status code. */
const char* kqr_status_string(int status);

/* Message of the last failure on the calling thread ("" if none). */
const char* kqr_last_error(void);

/* Number of HIP devices (0 if none or the runtime is unusable). */
int kqr_device_count(void);

/* Test hook for the breakdown handling of Section 3's preconditioner core
 * (kqr_info.core_retries): after `skip` further Woodbury core factorisations,
 * the next `count` report a non-positive pivot although they ran normally
 * (process-wide; concurrent fits share the counters).  (0, 0) switches it off.
 * Returns KQR_OK, or KQR_EINVAL for negative arguments.  Touches no device. */
int kqr_test_core_breakdowns(int skip, int count);

/* Test hook for kqr_fit_batch: on = 0 makes the problems' PCG iterations run
 * their vector and preconditioner kernels one problem at a time after each
 * batched K-apply instead of in the batched launches, and the batch meet in
 * lock-step rounds instead of open ones (on = 1, the default); the results
 * are the same either way (process-wide; read when a batch starts and when a
 * solve starts).  Returns KQR_OK, or KQR_EINVAL unless on is 0 or 1.  Touches
 * no device. */
int kqr_test_batch_steps(int on);

/* ---------------------------------------------------------------- kernel matrix
 * kqr_kernel_build: materialise K_ij = k(x_i, x_j) (Section 1) into K.
 *  X      device, n x p FP32, row-major (ld = p).
 *  K      device, n x ldk, type k_dtype (FP32, or BF16 rounded to nearest even);
 *         ldk >= n and a multiple of 8.  Columns n..ldk-1 are written as 0.
 *  RBF distances use ||x_i||^2 + ||x_j||^2 - 2 x_i.x_j clamped at 0 with the
 *  diagonal set to exactly 0, so K_ii = 1.  Asynchronous on `stream`. */
int kqr_kernel_build(const float* X, int64_t n, int64_t p, int kernel, double gamma,
                     int k_dtype, void* K, int64_t ldk, void* stream);

/* Symmetric packed layout (kqr_options.k_layout = 1).  K is symmetric
 * (Section 1), so only the tiles (I, J), I <= J, of a tiling by 128 x 128
 * blocks are stored: tile-row by tile-row, tile (I, J) at tile index
 * I nt - I (I - 1) / 2 + (J - I) with nt = ceil(n / 128), each tile row-major
 * (128 x 128 entries, zero beyond n).  A K-apply reads about half the bytes of
 * the full layout.
 * kqr_packed_bytes: bytes of that layout for n rows and k_dtype, or -1 for
 *  invalid arguments.
 * kqr_kernel_build_packed: X device n x p FP32; K device, kqr_packed_bytes
 *  bytes (entries as in kqr_kernel_build).  Asynchronous on `stream`.
 * kqr_kernel_apply_packed: u = K v.  v, u device n FP64 (v 16-byte aligned);
 *  mode KQR_APPLY_FAST (v rounded to FP32, FP32 products, FP64 sums across
 *  16-byte chunks and tiles) or KQR_APPLY_EXACT (FP64 v, products and sums).
 *  Asynchronous on `stream`; allocates its partial sums (stream-ordered). */
int64_t kqr_packed_bytes(int64_t n, int k_dtype);
/* kqr_autotune_packed: times every launch shape of the packed K-apply (thread
 * map 0 = a tile row read contiguously by 256-thread workgroups, 2 = the same
 * with 512 threads (half the loads per lane), 3 = map 2 with a persistent grid
 * of 1024 workgroups walking the strips, 1 = each wave owns 32 columns of a
 * tile; strip = tiles per workgroup, 1..16; 4 and 5 = each workgroup a square
 * block of strip x strip tiles, strip 2 or 4, with far fewer partial sums
 * written: each wave owns 32 columns of a tile (4) or 64 columns of half its
 * rows (5)) on the packed K (device, from
 * kqr_kernel_build_packed) for mode KQR_APPLY_FAST or KQR_APPLY_EXACT, and
 * installs the fastest for k_dtype and that mode (all later packed applies of
 * the process use it; shapes are tried by map 0 to 5, strips ascending, and
 * a later shape wins only when at least 2 % faster than the best so far).  report: host buffer of cap bytes for a JSON summary,
 * or NULL.  Blocks until the timing is done.
 * kqr_set_packed_shape: installs a shape directly (map 0 to 3 with
 * 1 <= strip <= 32, or map 4 or 5 with strip 2 or 4). */
int kqr_autotune_packed(const void* K, int k_dtype, int64_t n, int mode, int reps, char* report, int64_t cap,
                        void* stream);
int kqr_set_packed_shape(int k_dtype, int mode, int map, int strip);

/* kqr_set_otf_symmetric_limit: the square on-the-fly apply K(X, X) v (RBF
 * with p <= 32, Laplacian in fixed point) evaluates each distinct pair once
 * (K is symmetric, Section 1) and keeps one FP64 partial sum per 128 x 128
 * tile and column, about n^2 / 32 bytes of device memory.  bytes (>= 0,
 * default 32 GiB) bounds that buffer for the whole process; at larger n the
 * applies stream all n^2 pairs with O(n) partial sums instead.  Host-only. */
int kqr_set_otf_symmetric_limit(int64_t bytes);

/* kqr_set_otf_shape: launch shape of the on-the-fly applies for the rest of
 * the process (every later apply, fit and prediction).  strip: 128 x 128
 * tiles per workgroup of the symmetric square applies, 1..32, or 0 = by size
 * (2 tiles below 64 tile-rows, 8 from 64, 16 from 256, 32 from 1024); the
 * partial-sum buffer grows as the strip shrinks.  wgs: workgroups a
 * row-streamed launch (rectangles: prediction; squares beyond the symmetric
 * limit) aims for by slicing its columns, 256..2^20, or 0 = 8192.
 * Host-only; KQR_EINVAL outside those ranges. */
int kqr_set_otf_shape(int strip, int64_t wgs);
int kqr_kernel_build_packed(const float* X, int64_t n, int64_t p, int kernel, double gamma, int k_dtype, void* K,
                            void* stream);
int kqr_kernel_apply_packed(const void* K, int k_dtype, int64_t n, const double* v, double* u, int mode,
                            void* stream);

/* kqr_kernel_apply: U = K(X, X) V (the operator K v of (1.2)-(3.1)).
 *  K      device matrix from kqr_kernel_build (type k_dtype, ld ldk), or NULL to
 *         compute entries on the fly from X (FP32 entries; Laplacian: the L1
 *         distance is the exact integer distance of X in 32-bit fixed point,
 *         round((x_ik - min_k) 2^s) with s <= 23 the largest scale whose sums
 *         fit 32 bits, one v_sad_u32 per coordinate, used when s >= 20; the
 *         call then blocks while it reads the column ranges).
 *  V      device, n x m FP64 row-major (ld ldv >= m);  U device, n x m FP64 (ld ldu >= m).
 *  mode   KQR_APPLY_FAST or KQR_APPLY_EXACT.  m > 1: FAST uses FP32 products with
 *         FP32 accumulation on the matrix cores (one pass over K); EXACT with an
 *         FP32 K and m <= 4 forms all columns in FP64 (vectors, products, sums)
 *         from one pass over K; every other EXACT case runs column by column in
 *         FP64 (so EXACT never drops to FP32 products).
 *  Needs 1 <= m <= 16.  Asynchronous on `stream`; allocates its device
 *  workspace on `stream` (stream-ordered) and frees it before returning. */
int kqr_kernel_apply(const float* X, int64_t n, int64_t p, int kernel, double gamma,
                     const void* K, int k_dtype, int64_t ldk, const double* V, int64_t m,
                     int64_t ldv, double* U, int64_t ldu, int mode, void* stream);

/* kqr_kernel_apply_static: u = K v on a materialised K (full layout, from
 * kqr_kernel_build), FAST or EXACT as kqr_kernel_apply with m = 1, that
 * allocates nothing.  For callers that cannot allocate device memory: code
 * under HIP graph capture, serving loops, harnesses that forbid allocation.
 *  K      device n x ldk, type k_dtype (ldk >= n, a multiple of 8, 16-byte aligned).
 *  v      device n FP64, element i at v[i * incv];  u device n FP64 at u[i * incu].
 *  Its scratch (the FP32 copy of v, an aligned FP64 copy when incv != 1, the
 *  partial sums of the column segments) lives in one fixed device array of
 *  64 MiB per device, held from the first call on that device until the
 *  process ends; n needs 20 n bytes of it plus alignment (n up to about
 *  3.3 million), else KQR_EINVAL.  The launch shape is kqr_kernel_apply's, with
 *  the column segments capped to fit the array.  Every call on a device
 *  shares that device's array: calls that overlap on one device (other
 *  streams, other threads) race.  Asynchronous on `stream`; no allocation, no
 *  memset, so the call can be captured into a HIP graph. */
int kqr_kernel_apply_static(const void* K, int k_dtype, int64_t n, int64_t ldk, const double* v, int64_t incv,
                            double* u, int64_t incu, int mode, void* stream);

/* kqr_predict: f = beta + K(Xnew, Xtrain) alpha / lambda, computed on the fly.
 *  Xtrain device n x p FP32; alpha device n FP64; Xnew device m x p FP32;
 *  f device m FP64.  Asynchronous on `stream`. */
int kqr_predict(const float* Xtrain, int64_t n, int64_t p, const double* alpha, double beta,
                double lambda, int kernel, double gamma, const float* Xnew, int64_t m,
                double* f, void* stream);

/* ---------------------------------------------------------------- preconditioner pieces
 * kqr_rpcholesky: randomly pivoted Cholesky F = RPCholesky(K, rank) (Section 3,
 * (3.2)).  Step i draws the pivot s = first index whose running sum of the
 * residual diagonal exceeds uniforms[i] times its total, then
 *     g = K[:, s] - F[:, :i] F[s, :i]^T,  F[:, i] = g / sqrt(g_s),
 *     d <- max(d - F[:, i]^2, 0),  d_s <- 0.
 * Stops early when sum(d) <= 1e-14 tr(K).
 *  K         device (as in kqr_kernel_build) or NULL for entries from X.
 *  uniforms  host, rank values in [0,1).
 *  F         device, n x ldf FP32 row-major, ldf >= rank (multiple of 4).
 *  pivots    host, rank int64 (filled up to *rank_out).
 *  rank_out  host, number of columns produced. */
int kqr_rpcholesky(const float* X, int64_t n, int64_t p, int kernel, double gamma,
                   const void* K, int k_dtype, int64_t ldk, int64_t rank,
                   const double* uniforms, float* F, int64_t ldf, int64_t* pivots,
                   int64_t* rank_out, void* stream);

/* kqr_adaptive_rank: the rank heuristic of Section 3.  Given the first r0
 * columns of an RPCholesky factor F0 (device, n x ldf FP32, ldf multiple of 4),
 * returns in *rank the smallest r with lambda_r(F0^T F0) <= xi lambda_1 (r0 if
 * none), eigenvalues in decreasing order, and lambda_1 in *lambda1 (may be
 * NULL).  F0^T F0 is formed in FP64 and reduced to tridiagonal form on the
 * device; eigenvalues are located by Sturm bisection.  r0 <= 1023, 0 < xi < 1. */
int kqr_adaptive_rank(const float* F0, int64_t n, int64_t r0, int64_t ldf, double xi, int64_t* rank,
                      double* lambda1, void* stream);

/* kqr_autotune_apply: times the materialised K-apply on the caller's K
 * (device, as in kqr_kernel_build) for every supported tile shape -- rows per
 * wave {2,4,8} x 16-byte loads in flight per row {1,2,4} x column segments
 * {1,2,4,8,16} -- with `reps` timed launches each, and keeps the fastest shape
 * for (k_dtype, mode, size class of n) for the rest of the process.  With
 * mode KQR_APPLY_KV it times the multi-column K V launch (16 columns) instead,
 * over {64-row tiles streamed through LDS} and {direct loads in the MFMA
 * layout: 16-byte loads per lane per step {4,8} x next-step prefetch {0,1}},
 * each with column segments {1,2,4,8} (20 shapes), and keeps the fastest for
 * (k_dtype, size class of n).  Writes a JSON report (every shape's average launch time and the
 * choice) into `report` (host, `cap` bytes, NUL-terminated; may be NULL).
 * Synchronises. */
int kqr_autotune_apply(const void* K, int k_dtype, int64_t n, int64_t ldk, int mode, int reps, char* report,
                       int64_t cap, void* stream);

/* kqr_set_apply_shape: installs a K-apply tile shape (e.g. one recorded by
 * kqr_autotune_apply) for (k_dtype, mode, size class of n).  rows in {2,4,8},
 * unroll in {1,2,4}, 1 <= segs <= 64; otherwise KQR_EINVAL. */
int kqr_set_apply_shape(int k_dtype, int mode, int64_t n, int rows, int unroll, int segs);

/* kqr_set_kv_shape: installs a K V launch shape (e.g. one recorded by
 * kqr_autotune_apply with KQR_APPLY_KV) for (k_dtype, size class of n).
 * nld = 0 (64-row tiles streamed through LDS; prefetch is ignored) or
 * nld in {4,8} (direct loads, 16-byte loads per lane per step) with prefetch
 * in {0,1}; 1 <= segs <= 8; otherwise KQR_EINVAL. */
int kqr_set_kv_shape(int k_dtype, int64_t n, int nld, int prefetch, int segs);

/* kqr_autotune_otf: times the on-the-fly applies on the caller's X (device,
 * n x p FP32) for mode KQR_APPLY_FAST or KQR_APPLY_EXACT: the square apply
 * K(X, X) v at every strip of its symmetric form (1, 2, 4, 8, 16, 32 tiles
 * per workgroup, where the partial sums fit the symmetric limit), keeping
 * the fastest for n's size class (as kqr_set_otf_shape would, for that class
 * only), then the column-slice target of the row-streamed form on the
 * rectangle K(X[0:n/4], X) v over 2048 .. 32768 workgroups, keeping the
 * fastest.  JSON report into `report` (host, cap bytes, or NULL).
 * Synchronises. */
int kqr_autotune_otf(const float* X, int64_t n, int64_t p, int kernel, double gamma, int mode, int reps,
                     char* report, int64_t cap, void* stream);

/* kqr_tune_save / kqr_tune_load: the launch shapes installed in this
 * process -- by kqr_autotune_apply (K-apply and K V), kqr_autotune_packed,
 * kqr_autotune_otf and the kqr_set_*_shape calls -- written to / read from a
 * JSON file at `path` (host string) keyed by the device architecture
 * (hipDeviceProp_t.gcnArchName): one entry per (kernel, storage type, mode,
 * size class of n, right-hand sides), with the measured launch time.
 * Loading installs the entries recorded for the current device's
 * architecture (none from another) and sets *count (host) to how many;
 * saving sets it to the entries written.  A process started with the
 * environment variable KQR_TUNE_FILE=<path> loads that file at its first
 * call that uses the device.  kqr_tune_load checks the whole file first
 * (KQR_EINVAL for an unreadable or malformed file, nothing installed), then
 * needs a device (KQR_ENODEVICE). */
int kqr_tune_save(const char* path, int* count);
int kqr_tune_load(const char* path, int* count);

/* kqr_woodbury_apply: out = P^{-1} w for P = F F^T + c 1 1^T + diag(Ldiag), by
 * Lemma 1 with U = [F 1] and the (r+1)x(r+1) core C = diag(I, 1/c) + U^T L^{-1} U
 * formed and Cholesky-factored in FP64 on the device.
 *  F device n x ldf FP32 (r columns used); Ldiag, w, out device n FP64; c > 0,
 *  Ldiag > 0.  r <= 1023.  Returns KQR_ENUMERIC if the core is not positive definite. */
int kqr_woodbury_apply(const float* F, int64_t n, int64_t r, int64_t ldf, double c,
                       const double* Ldiag, const double* w, double* out, void* stream);

/* kqr_pcg_solve: left-preconditioned CG (Section 3) on
 *     (K + c 1 1^T + diag(Ldiag)) x = b,
 * preconditioned by (3.2) with F (r columns; r = 0: no preconditioner).  Stops
 * when ||b - A x||_2 <= tol or after maxit iterations.
 *  K as in kqr_kernel_apply (NULL = on the fly from X); x device n FP64 holds
 *  the start on entry and the solution on return; iters, resnorm host. */
int kqr_pcg_solve(const float* X, int64_t n, int64_t p, int kernel, double gamma,
                  const void* K, int k_dtype, int64_t ldk, const float* F, int64_t r,
                  int64_t ldf, double c, const double* Ldiag, const double* b, double tol,
                  int maxit, double* x, int* iters, double* resnorm, void* stream);

/* kqr_ssn_gradient: the fused Newton set-up of Algorithm 3 at alpha:
 *     w = alpha + z/sigma,  grad = K alpha/lambda - y + beta 1 + sigma 1 (1^T alpha)
 *                                  + sigma (w - Pi_B(w))                      (2.3)
 *     S_ii = 1 if tau-1 < w_i < tau else 0 (boundary -> 0)          (Section 2.2)
 *     eps_t = max(tau1 min(tau2, ||grad||), eps_floor)
 *     Ldiag = lambda sigma (1 - S) + lambda eps_t,   rhs = -lambda grad      (3.1)
 *  alpha, Kalpha, y, z device n FP64; grad, Ldiag, rhs device n FP64 outputs;
 *  S device n uint8 output; gnorm, eps_t host outputs. */
int kqr_ssn_gradient(int64_t n, double tau, double lambda, double beta, double sigma,
                     double tau1, double tau2, double eps_floor, const double* alpha,
                     const double* Kalpha, const double* y, const double* z, double* grad,
                     uint8_t* S, double* Ldiag, double* rhs, double* gnorm, double* eps_t,
                     void* stream);

/* kqr_kkt_residuals: the multiplier step of Algorithms 1 and 2 and the
 * stopping measures of Section 4 at one iterate, by the kernel the fits use.
 *  update = 1: first v = Pi_B(alpha + z/sigma) and z += step sigma (alpha - v)
 *  (the z-part of the (beta, z) ascent of (2.1) and Algorithm 2, with v from
 *  its closed form; beta is the caller's, already updated); update = 0: z and
 *  v are used as given (sigma and step unused).  Then, with Kalpha = K alpha
 *  supplied by the caller (any precision):
 *    eta_p = ||z - y + beta 1 + Kalpha/lambda|| / (1 + ||y||)
 *    eta_d = sqrt((1^T alpha)^2 + ||alpha - v||^2) / (1 + ||alpha||)
 *    eta_c = ||v - Pi_B(z + v)|| / (1 + ||v||)
 *    obj_p = rho_tau(z) + alpha^T Kalpha / (2 lambda)
 *    obj_d = -alpha^T Kalpha / (2 lambda) + y^T alpha
 *    eta_gap = |obj_p - obj_d| / (1 + |obj_p| + |obj_d|)
 *  every product and sum in FP64, reduced in a fixed order.
 *  alpha, Kalpha, y device n FP64; z, v device n FP64 (overwritten when
 *  update = 1); out host double[7] = {eta_p, eta_d, eta_c, eta_kkt, eta_gap,
 *  obj_p, obj_d}.  Blocks until out is written. */
int kqr_kkt_residuals(int64_t n, double tau, double lambda, double beta, double sigma, double step, int update,
                      const double* alpha, const double* Kalpha, const double* y, double* z, double* v, double* out,
                      void* stream);

/* ---------------------------------------------------------------- the fit
 * kqr_fit: PALM-KQR -- Phase I inexact ADMM (Algorithm 1) warm start, Phase II
 * semismooth Newton ALM (Algorithms 2, 3) with PCG on (3.1) preconditioned by
 * (3.2) through Lemma 1, stopped by the rules of Section 4 with the residuals
 * measured with exact (FP32-entry, FP64-accumulated) K.
 *  X device n x p FP32; y device n FP64; alpha device n FP64 output;
 *  beta host output; info host (may be NULL); opt host (NULL = defaults).
 *  Returns KQR_OK, KQR_NOT_CONVERGED (caps reached), or an error.  Device
 *  workspace (K, F, vectors) is allocated inside and freed before return. */
int kqr_fit(const float* X, const double* y, int64_t n, int64_t p, double tau, double lambda,
            int kernel, double gamma, const kqr_options* opt, double* alpha, double* beta,
            kqr_info* info, void* stream);

/* Host threads the batched fits use from now on (process-wide): 1..16, or 0
 * for the default (min(16, host cores), or KQR_BATCH_THREADS when set).
 * Returns KQR_OK or KQR_EINVAL.  Touches no device. */
int kqr_set_batch_threads(int threads);

/* Batched fits (kqr_fit_multi_tau, kqr_fit_path, kqr_fit_batch) run every
 * fit's PALM-KQR iteration as a coroutine: a bounded pool of host threads
 * (min(fits, 16, host cores); environment variable KQR_BATCH_THREADS = 1..16
 * or kqr_set_batch_threads overrides), one scheduler and one stream each, resumes the fits between
 * their read-backs and K-apply requests.  Whenever every fit still running
 * waits for a K-apply, one batched launch serves them all (lock-step rounds
 * over the unfinished fits).  Results do not depend on the thread count.
 *
 * kqr_fit_multi_tau: kqr_fit for ntau quantile levels taus[0..ntau-1] on the
 * same (X, y, lambda, kernel, gamma), solved jointly.  K and the RPCholesky
 * factor are built once; each level runs its own PALM-KQR iteration and the
 * fast K-applies of all levels still running are coalesced into one K V
 * launch on the matrix cores (V: n x up to 16 columns), so one pass over K
 * serves every level.
 *  alpha   device, ntau x n FP64 (row t = alpha of taus[t]);  beta host ntau;
 *  info    host ntau (may be NULL); for the coalesced applies
 *          kapply_fast_calls / t_kapply_fast count the shared launches;
 *  status  host ntau: KQR_OK or KQR_NOT_CONVERGED per level.
 *  1 <= ntau <= 16.  Returns KQR_OK when every level ran (see status[]), else
 *  the first error. */
int kqr_fit_multi_tau(const float* X, const double* y, int64_t n, int64_t p, const double* taus, int ntau,
                      double lambda, int kernel, double gamma, const kqr_options* opt, double* alpha,
                      double* beta, kqr_info* info, int* status, void* stream);

/* kqr_fit_path: kqr_fit for nlam values of lambda, lambdas[0..nlam-1], on the
 * same (X, y, tau, kernel, gamma): the regularisation paths of Section 4.1.
 * K and the RPCholesky factor do not depend on lambda and are built once.
 * Every value is solved from the cold start of Algorithm 1 (each result is the
 * unique optimum for its lambda, independent of the order of lambdas); up to
 * 16 values run at once with their fast K-applies coalesced into K V launches
 * as in kqr_fit_multi_tau, and a fit slot that finishes one value takes the
 * next.
 *  alpha   device, nlam x n FP64 (row t = alpha of lambdas[t]);  beta host nlam;
 *  info    host nlam (may be NULL); status host nlam (KQR_OK or
 *          KQR_NOT_CONVERGED per value).
 *  1 <= nlam <= 4096, every lambda > 0.  Returns KQR_OK when every value ran
 *  (see status[]), else the first error. */
int kqr_fit_path(const float* X, const double* y, int64_t n, int64_t p, double tau, const double* lambdas,
                 int nlam, int kernel, double gamma, const kqr_options* opt, double* alpha, double* beta,
                 kqr_info* info, int* status, void* stream);

/* kqr_fit_batch: nprob independent fits (sizes n[i], common p and kernel
 * type, per-problem tau, lambda, gamma).  Each problem gets its own K and
 * preconditioner (built interleaved on the batch's streams); the fast
 * K-applies of all problems still running go out as one persistent launch
 * whose workgroups take (problem, 32-row block) items from a device queue,
 * largest problems first.  When a K-apply is a PCG iteration's (Algorithm 3's
 * solves with the Woodbury preconditioner of Lemma 1) of a problem with a
 * preconditioner rank below 128, the same launch sequence then runs the rest
 * of that iteration for all such problems in batched launches (five, and up
 * to eight more when some n[i] > 16384 need several workgroups per vector;
 * the single-problem kernels' code per problem, so the same results).
 *  X, y, alpha: host arrays of nprob device pointers (n[i] x p FP32, n[i] FP64,
 *  n[i] FP64); tau, lambda, gamma, n: host arrays; beta, status: host nprob;
 *  info: host nprob (may be NULL).  1 <= nprob <= 256. */
int kqr_fit_batch(int nprob, const float* const* X, const double* const* y, const int64_t* n, int64_t p,
                  const double* tau, const double* lambda, int kernel, const double* gamma,
                  const kqr_options* opt, double* const* alpha, double* beta, kqr_info* info, int* status,
                  void* stream);

/* kqr_fit_grad: kqr_fit followed by the implicit gradient of the validation
 * check loss J = sum_i rho_tau(yval_i - beta - K(Xval_i, X) alpha / lambda)
 * with respect to log(gamma) and log(lambda).  The gradient is not part of the
 * paper: it differentiates the KKT conditions of the dual (1.3) on the active
 * partition R (alpha = tau), L (alpha = tau - 1), E (interior), which requires
 * E to be non-empty (beta is otherwise not differentiable) and the partition
 * to be locally constant (strict complementarity); dK/dlog(gamma) = K o ln K
 * holds for both kernels.  Before the gradient the fit is polished: E is read
 * from the final multipliers (|z_i| below a threshold), alpha_N is put on its
 * bound and (alpha_E, beta) solve the bordered KKT system with the FP64
 * Cholesky of K_EE (entries formed in FP64 from the FP32 X); violators are
 * moved between the sets (an interior alpha outside the box to the bound it
 * crossed, a bound alpha with a residual of the wrong sign to the interior)
 * for up to 12 active-set rounds.  The polish is kept when alpha_E stays in
 * the box and every residual sign matches the partition, and alpha / beta are
 * then the polished values.
 *  Xval device nval x p FP32; yval device nval FP64; other arguments as kqr_fit.
 *  val_loss, grad (host, 2: dJ/dlog gamma, dJ/dlog lambda), n_interior and
 *  polished are host outputs (n_interior and polished may be NULL).
 *  Errors: KQR_ENUMERIC when E is empty or K_EE is not positive definite in
 *  FP64, KQR_EINVAL when |E| exceeds 8192 (the dense factor's limit).
 *  Returns KQR_OK or KQR_NOT_CONVERGED (gradient still computed). */
int kqr_fit_grad(const float* X, const double* y, int64_t n, int64_t p, double tau, double lambda, int kernel,
                 double gamma, const float* Xval, const double* yval, int64_t nval, const kqr_options* opt,
                 double* alpha, double* beta, double* val_loss, double* grad, int64_t* n_interior, int* polished,
                 kqr_info* info, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KQR_H */
