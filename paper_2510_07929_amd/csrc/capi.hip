// extern "C" entry points of libkqr: argument validation, workspace set-up and
// dispatch.  No exception crosses the ABI: every entry point returns a status.
#include "adjoint.h"
#include "fit.h"
#include "kernel_entry.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <memory>

namespace kqr {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

void fail(int status, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Error(status, buf);
}

void DevBuf::alloc(size_t b) {
  release();
  if (b == 0) b = 16;
  hipError_t e = hipMalloc(&ptr, b);
  if (e != hipSuccess) {
    ptr = nullptr;
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? KQR_ENOMEM : KQR_EHIP, "hipMalloc(%zu bytes): %s", b, hipGetErrorString(e));
  }
  bytes = b;
}

// hipFree waits for the whole device; inside a DeferFrees scope the frees
// wait for the scope's end instead, so a batch of fits running side by side
// does not drain the GPU whenever one of them releases a buffer.
static thread_local std::vector<void*>* g_deferred = nullptr;

void DevBuf::release() {
  if (ptr) {
    if (g_deferred) g_deferred->push_back(ptr);
    else (void)hipFree(ptr);
  }
  ptr = nullptr;
  bytes = 0;
}

DeferFrees::DeferFrees() : prev_(g_deferred) { g_deferred = &list_; }

DeferFrees::~DeferFrees() {
  g_deferred = prev_;
  for (void* p : list_) (void)hipFree(p);
}

void DeferFrees::hand_to(std::vector<void*>& out) {
  out.insert(out.end(), list_.begin(), list_.end());
  list_.clear();
}

HostPinned::HostPinned(size_t b) {
  hipError_t e = hipHostMalloc(&ptr, b, hipHostMallocDefault);
  if (e != hipSuccess) {
    ptr = nullptr;
    fail(KQR_EHIP, "hipHostMalloc(%zu bytes): %s", b, hipGetErrorString(e));
  }
}

HostPinned::~HostPinned() {
  if (ptr) (void)hipHostFree(ptr);
}

void ensure_device() {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    fail(KQR_ENODEVICE, "no HIP device available");
  }
  tune_autoload();  // launch shapes from KQR_TUNE_FILE, once per process
}

template <typename Fn>
static int guarded(Fn&& fn) {
  try {
    g_last_error.clear();
    fn();
    return KQR_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return KQR_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return KQR_EHIP;
  } catch (...) {
    g_last_error = "unknown failure";
    return KQR_EHIP;
  }
}

#define KQR_REQUIRE(cond, ...) \
  do {                         \
    if (!(cond)) fail(KQR_EINVAL, __VA_ARGS__); \
  } while (0)

static void check_kernel(int kernel, double gamma, bool linear_ok = true) {
  KQR_REQUIRE(kernel == KQR_RBF || kernel == KQR_LAPLACIAN || kernel == KQR_LINEAR,
              "kernel must be KQR_RBF, KQR_LAPLACIAN or KQR_LINEAR");
  KQR_REQUIRE(linear_ok || kernel != KQR_LINEAR,
              "the linear kernel is used in factored form only (no materialised K, RPCholesky or gradient)");
  KQR_REQUIRE(std::isfinite(gamma) && gamma > 0.0, "gamma must be positive and finite");
}

static void check_kmat(const void* K, int k_dtype, int64_t ldk, int64_t n) {
  if (!K) return;
  KQR_REQUIRE(k_dtype == KQR_FP32 || k_dtype == KQR_BF16, "k_dtype must be KQR_FP32 or KQR_BF16");
  KQR_REQUIRE(ldk >= n && ldk % 8 == 0, "ldk must be >= n and a multiple of 8");
  KQR_REQUIRE((reinterpret_cast<uintptr_t>(K) & 15) == 0, "K must be 16-byte aligned");
}

// Times every supported K V launch shape (16 right-hand sides) on K and
// installs the fastest for K's dtype and size bucket; JSON report.
static void autotune_kv(const KMat& km, int64_t n, int reps, char* report, int64_t cap, hipStream_t st) {
  DevBuf V16(size_t(n) * 16 * sizeof(float)), U(size_t(n) * 16 * sizeof(double));
  DevBuf part(kv_scratch_doubles(n) * sizeof(double)), ones(size_t(n) * 16 * sizeof(double));
  fill(n * 16, 1.0 / double(n), ones.as<double>(), st);
  kv_gather_strided(ones.as<double>(), 16, 16, n, n, V16.as<float>(), st);
  hipEvent_t e0, e1;
  KQR_CHECK_HIP(hipEventCreate(&e0));
  KQR_CHECK_HIP(hipEventCreate(&e1));
  std::string rep = "{\"n\": " + std::to_string(n) + ", \"k_dtype\": " + std::to_string(km.dtype) +
                    ", \"mode\": " + std::to_string(KQR_APPLY_KV) + ", \"shapes\": [";
  KvShape best;
  double best_us = 1e300;
  bool first = true;
  try {
    for (int nld : {0, 4, 8})
      for (int pf : {0, 1})
        for (int sg : {1, 2, 4, 8}) {
          if (nld == 0 && pf == 0) continue;  // the staged kernel always prefetches
          KvShape s;
          s.nld = nld;
          s.prefetch = pf;
          s.segs = sg;
          kapply_kv(km, n, V16.as<float>(), 16, U.as<double>(), 16, part.as<double>(), st, &s);  // warm-up
          KQR_CHECK_HIP(hipEventRecord(e0, st));
          for (int k = 0; k < reps; ++k)
            kapply_kv(km, n, V16.as<float>(), 16, U.as<double>(), 16, part.as<double>(), st, &s);
          KQR_CHECK_HIP(hipEventRecord(e1, st));
          KQR_CHECK_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          KQR_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
          const double us = 1e3 * ms / reps;
          char buf[128];
          snprintf(buf, sizeof(buf), "%s{\"nld\": %d, \"prefetch\": %d, \"segs\": %d, \"us\": %.2f}",
                   first ? "" : ", ", nld, pf, sg, us);
          first = false;
          rep += buf;
          if (us < best_us) { best_us = us; best = s; }
        }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  set_kv_shape(km.dtype, n, best);
  tune_record(TuneEntry{"kv", km.dtype, 0, n, 16, best.nld, best.prefetch, best.segs, 0, best_us});
  char buf[160];
  snprintf(buf, sizeof(buf), "], \"best\": {\"nld\": %d, \"prefetch\": %d, \"segs\": %d, \"us\": %.2f}}", best.nld,
           best.prefetch, best.segs, best_us);
  rep += buf;
  if (report && cap > 0) {
    const size_t nb = std::min<size_t>(size_t(cap) - 1, rep.size());
    memcpy(report, rep.data(), nb);
    report[nb] = '\0';
  }
}

// Times every supported packed K-apply shape (map x strip, with the reduction)
// on a packed K and installs the fastest for K's dtype and the mode; JSON report.
// Shapes are tried in order and a later one replaces the best so far only when
// it is at least 2 % faster, so timing noise between shapes of equal speed
// does not flip the choice (each shape rounds its FP32 partial sums in its
// own grouping, which a fit's iterates follow).
static void autotune_packed(const KMat& km, int64_t n, bool exact, int reps, char* report, int64_t cap,
                            hipStream_t st) {
  DevBuf v64(size_t(n) * sizeof(double)), v32(size_t(n) * sizeof(float)), u(size_t(n) * sizeof(double));
  DevBuf scratch(packed_scratch_doubles(n, 1) * sizeof(double));  // strip 1 needs the most
  fill(n, 1.0 / double(n), v64.as<double>(), st);
  to_f32(v64.as<double>(), n, 1, 1, v32.as<float>(), 1, st);
  hipEvent_t e0, e1;
  KQR_CHECK_HIP(hipEventCreate(&e0));
  KQR_CHECK_HIP(hipEventCreate(&e1));
  std::string rep = "{\"n\": " + std::to_string(n) + ", \"k_dtype\": " + std::to_string(km.dtype) +
                    ", \"exact\": " + std::to_string(int(exact)) + ", \"shapes\": [";
  PackedShape best;
  double best_us = 1e300;
  bool first = true;
  try {
    for (int map : {0, 1, 2, 3, 4, 5})
      for (int strip : {1, 2, 4, 8, 16}) {
        const PackedShape s{map, strip};
        if (!packed_shape_supported(s)) continue;  // maps 4 and 5: blocks of 2 x 2 or 4 x 4 tiles
        kapply_packed(km, n, v32.as<float>(), v64.as<double>(), u.as<double>(), 1, exact, st, &s,
                      scratch.as<double>());  // warm-up
        KQR_CHECK_HIP(hipEventRecord(e0, st));
        for (int k = 0; k < reps; ++k)
          kapply_packed(km, n, v32.as<float>(), v64.as<double>(), u.as<double>(), 1, exact, st, &s,
                        scratch.as<double>());
        KQR_CHECK_HIP(hipEventRecord(e1, st));
        KQR_CHECK_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        KQR_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
        const double us = 1e3 * ms / reps;
        char buf[128];
        snprintf(buf, sizeof(buf), "%s{\"map\": %d, \"strip\": %d, \"us\": %.2f}", first ? "" : ", ", map, strip,
                 us);
        first = false;
        rep += buf;
        if (us < 0.98 * best_us) { best_us = us; best = s; }
      }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  set_packed_shape(km.dtype, exact, best);
  tune_record(TuneEntry{"packed", km.dtype, exact ? 1 : 0, n, 1, best.map, best.strip, 0, 0, best_us});
  char buf[160];
  snprintf(buf, sizeof(buf), "], \"best\": {\"map\": %d, \"strip\": %d, \"us\": %.2f}}", best.map, best.strip,
           best_us);
  rep += buf;
  if (report && cap > 0) {
    const size_t nb = std::min<size_t>(size_t(cap) - 1, rep.size());
    memcpy(report, rep.data(), nb);
    report[nb] = '\0';
  }
}

// Times the square on-the-fly apply K(X, X) v at n for every strip of the
// symmetric form {1, 2, 4, 8, 16, 32} (those whose partial sums fit the
// budget) and installs the fastest for n's size class; then the column-slice
// target of the row-streamed form on a rectangle K(X[0:n/4], X) v, over
// {2048, 4096, 8192, 16384, 32768} workgroups.  JSON report.
static void autotune_otf(const float* X, int64_t n, int p, KernelSpec ks, bool exact, int reps, char* report,
                         int64_t cap, hipStream_t st) {
  DevBuf sqn(size_t(n) * sizeof(float)), v(size_t(n) * sizeof(double)), u(size_t(n) * sizeof(double));
  row_sqnorms(X, n, p, sqn.as<float>(), st);
  fill(n, 1.0 / double(n), v.as<double>(), st);
  DevBuf xq;
  int shift = -1;
  if (ks.kind == KQR_LAPLACIAN) {
    xq.alloc(size_t(n) * size_t(p) * sizeof(uint32_t));
    shift = quantize_columns(X, n, p, xq.as<uint32_t>(), st);
  }
  const bool sym = (ks.kind == KQR_RBF && p <= 32) || shift >= 20;
  const int keep_strip = otf_strip_for(n);
  const int64_t keep_wgs = otf_wgs();
  hipEvent_t e0, e1;
  KQR_CHECK_HIP(hipEventCreate(&e0));
  KQR_CHECK_HIP(hipEventCreate(&e1));
  auto time_us = [&](auto&& launch) {
    launch();  // warm-up
    KQR_CHECK_HIP(hipEventRecord(e0, st));
    for (int k = 0; k < reps; ++k) launch();
    KQR_CHECK_HIP(hipEventRecord(e1, st));
    KQR_CHECK_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    KQR_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
    return 1e3 * double(ms) / reps;
  };
  std::string rep = "{\"n\": " + std::to_string(n) + ", \"p\": " + std::to_string(p) +
                    ", \"exact\": " + std::to_string(int(exact)) + ", \"strips\": [";
  int best_strip = keep_strip;
  double best_us = 1e300;
  bool first = true;
  try {
    if (sym) {
      for (int strip : {1, 2, 4, 8, 16, 32}) {
        set_otf_strip_for(n, strip);
        const size_t need = otf_sym_scratch_doubles(n);
        if (need == 0) continue;  // partial sums beyond the budget at this strip
        DevBuf scr(need * sizeof(double));
        const double us = time_us([&] {
          if (shift >= 20)
            kapply_otf_l1q(xq.as<uint32_t>(), n, p, ks.gamma, shift, v.as<double>(), u.as<double>(), 1, exact, st,
                           scr.as<double>(), need);
          else
            kapply_otf(X, sqn.as<float>(), n, X, sqn.as<float>(), n, p, ks, v.as<double>(), u.as<double>(), 1, 1.0,
                       0.0, st, exact, scr.as<double>(), need);
        });
        char buf[96];
        snprintf(buf, sizeof(buf), "%s{\"strip\": %d, \"us\": %.2f}", first ? "" : ", ", strip, us);
        first = false;
        rep += buf;
        if (us < best_us) { best_us = us; best_strip = strip; }
      }
    }
    set_otf_strip_for(n, sym ? best_strip : keep_strip);
    rep += "], \"wgs\": [";
    const int64_t nr = std::max<int64_t>(1, n / 4);
    int64_t best_wgs = keep_wgs;
    double best_wus = 1e300;
    first = true;
    for (int64_t w : {int64_t(2048), int64_t(4096), int64_t(8192), int64_t(16384), int64_t(32768)}) {
      set_otf_wgs(w);
      const double us = time_us([&] {
        kapply_otf(X, sqn.as<float>(), nr, X, sqn.as<float>(), n, p, ks, v.as<double>(), u.as<double>(), 1, 1.0, 0.0,
                   st, exact);
      });
      char buf[96];
      snprintf(buf, sizeof(buf), "%s{\"wgs\": %lld, \"us\": %.2f}", first ? "" : ", ", (long long)w, us);
      first = false;
      rep += buf;
      if (us < best_wus) { best_wus = us; best_wgs = w; }
    }
    set_otf_wgs(best_wgs);
    tune_record(TuneEntry{"otf", 0, exact ? 1 : 0, n, 1, sym ? best_strip : 0, 0, 0, best_wgs, sym ? best_us : 0.0});
    char buf[160];
    snprintf(buf, sizeof(buf), "], \"best\": {\"strip\": %d, \"us\": %.2f, \"wgs\": %lld, \"wgs_us\": %.2f}}",
             sym ? best_strip : 0, sym ? best_us : 0.0, (long long)best_wgs, best_wus);
    rep += buf;
  } catch (...) {
    set_otf_strip_for(n, keep_strip);
    set_otf_wgs(keep_wgs);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (report && cap > 0) {
    const size_t nb = std::min<size_t>(size_t(cap) - 1, rep.size());
    memcpy(report, rep.data(), nb);
    report[nb] = '\0';
  }
}

}  // namespace kqr

using namespace kqr;

extern "C" {

int kqr_default_options(kqr_options* o) {
  if (!o) return KQR_EINVAL;
  memset(o, 0, sizeof(*o));
  o->tol = 1e-6;
  o->admm_tol = 1e-3;
  o->admm_max_iter = 100;
  o->alm_max_iter = 1000;
  o->admm_sigma = 1.0;
  o->admm_step = 1.618;
  o->admm_eps0 = 0.1;
  o->etabar = 0.1;
  o->iota = 0.5;
  o->armijo = 1e-4;
  o->ls_shrink = 0.5;
  o->ls_max = 40;
  o->tau1 = 0.1;
  o->tau2 = 0.1;
  o->eps_floor = 1e-12;
  o->ssn_max_iter = 50;
  o->ssn_rel = 0.5;
  o->sigma_factor = 5.0;
  o->sigma_stall = 0.25;
  o->sigma_max = 1e8;
  o->rank = 0;
  o->xi = 1e-7;
  o->pcg_max_iter = 2000;
  o->k_dtype = KQR_FP32;
  o->kmode = KQR_KMODE_AUTO;
  o->refine = 1;
  o->ssn_adapt = 0.3;
  o->pivot_uniforms = nullptr;
  o->seed = 0;
  o->verbose = 0;
  return KQR_OK;
}

const char* kqr_status_string(int s) {
  switch (s) {
    case KQR_OK: return "ok";
    case KQR_NOT_CONVERGED: return "not converged (iteration cap reached)";
    case KQR_EINVAL: return "invalid argument";
    case KQR_ENOMEM: return "device allocation failed";
    case KQR_ENODEVICE: return "no HIP device";
    case KQR_EHIP: return "HIP runtime error";
    case KQR_ENUMERIC: return "numerical failure (NaN/Inf or breakdown)";
    default: return "unknown status";
  }
}

const char* kqr_last_error(void) { return g_last_error.c_str(); }

int kqr_set_batch_threads(int threads) {
  if (threads < 0 || threads > 16) return KQR_EINVAL;
  set_batch_threads(threads);
  return KQR_OK;
}

int kqr_test_core_breakdowns(int skip, int count) {
  if (skip < 0 || count < 0) return KQR_EINVAL;
  set_forced_core_breakdowns(skip, count);
  return KQR_OK;
}

int kqr_test_batch_steps(int on) {
  if (on != 0 && on != 1) return KQR_EINVAL;
  set_batch_steps(on == 1);
  return KQR_OK;
}

int kqr_device_count(void) {
  int c = 0;
  if (hipGetDeviceCount(&c) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return c;
}

int kqr_kernel_build(const float* X, int64_t n, int64_t p, int kernel, double gamma, int k_dtype, void* K,
                     int64_t ldk, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(X && K, "X and K must be non-null");
    KQR_REQUIRE(n >= 1 && p >= 1 && p <= 64, "need n >= 1 and 1 <= p <= 64");
    check_kernel(kernel, gamma, false);
    check_kmat(K, k_dtype, ldk, n);
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    float* sqn = nullptr;
    KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&sqn), size_t(n) * sizeof(float), st));
    row_sqnorms(X, n, int(p), sqn, st);
    kbuild(X, sqn, n, int(p), KernelSpec{kernel, gamma}, k_dtype, K, ldk, st);
    KQR_CHECK_HIP(hipFreeAsync(sqn, st));
  });
}

int kqr_kernel_apply(const float* X, int64_t n, int64_t p, int kernel, double gamma, const void* K, int k_dtype,
                     int64_t ldk, const double* V, int64_t m, int64_t ldv, double* U, int64_t ldu, int mode,
                     void* stream) {
  return guarded([&] {
    KQR_REQUIRE(V && U, "V and U must be non-null");
    KQR_REQUIRE(n >= 1, "need n >= 1");
    KQR_REQUIRE(m >= 1 && m <= 16, "need 1 <= m <= 16");
    KQR_REQUIRE(ldv >= m && ldu >= m, "need ldv >= m and ldu >= m");
    KQR_REQUIRE(mode == KQR_APPLY_FAST || mode == KQR_APPLY_EXACT, "mode must be KQR_APPLY_FAST or KQR_APPLY_EXACT");
    if (!K) {
      KQR_REQUIRE(X != nullptr, "X must be non-null when K is NULL");
      KQR_REQUIRE(p >= 1 && p <= 64, "need 1 <= p <= 64");
      check_kernel(kernel, gamma);
    }
    check_kmat(K, k_dtype, ldk, n);
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    const KernelSpec ks{kernel, gamma};
    const KMat km{K, k_dtype, ldk};
    void* tmp = nullptr;
    // per column: contiguous FP64 copy (when strided) and its FP32 rounding
    const size_t bytes = size_t(n) * (sizeof(double) + sizeof(float)) + 256;
    KQR_CHECK_HIP(hipMallocAsync(&tmp, bytes, st));
    double* v64 = static_cast<double*>(tmp);
    float* v32 = reinterpret_cast<float*>(static_cast<char*>(tmp) + ((size_t(n) * sizeof(double) + 255) / 256) * 256);
    float* sqn = nullptr;
    double* lscr = nullptr;
    DevBuf xq;
    int shift = -1;
    if (!K && kernel == KQR_LINEAR) {
      KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&lscr), lin_scratch_doubles(int(p)) * sizeof(double), st));
    } else if (!K) {
      KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&sqn), size_t(n) * sizeof(float), st));
      row_sqnorms(X, n, int(p), sqn, st);
      if (kernel == KQR_LAPLACIAN) {  // exact integer L1 distances of fixed-point X, as in the fits
        xq.alloc(size_t(n) * size_t(p) * sizeof(uint32_t));
        shift = quantize_columns(X, n, int(p), xq.as<uint32_t>(), st);
      }
    }
    if (K && m > 1 && mode == KQR_APPLY_EXACT && k_dtype == KQR_FP32 && m <= kKvMaxExact) {
      // exact columns (FP64 vectors, products and sums) from one pass over K
      double* cols = nullptr;
      double* part = nullptr;
      KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&cols), size_t(2 * m) * size_t(n) * sizeof(double), st));
      KQR_CHECK_HIP(
          hipMallocAsync(reinterpret_cast<void**>(&part), kv_scratch_doubles(n) * sizeof(double), st));
      float* V16 = nullptr;  // no fast columns: zeros for the matrix-core half of the pass
      KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&V16), size_t(n) * 16 * sizeof(float), st));
      fill(n * 8, 0.0, reinterpret_cast<double*>(V16), st);  // 16 FP32 zeros per row, by a kernel (capturable)
      SrcTable16 xs{};
      DstTable16 xd{};
      for (int64_t j = 0; j < m; ++j) {
        double* cj = cols + size_t(j) * size_t(n);
        KQR_CHECK_HIP(hipMemcpy2DAsync(cj, sizeof(double), V + j, size_t(ldv) * sizeof(double), sizeof(double),
                                       size_t(n), hipMemcpyDeviceToDevice, st));
        xs.p[j] = cj;
        xd.p[j] = cols + size_t(m + j) * size_t(n);
      }
      kapply_kv_mixed(km, n, V16, 0, nullptr, 16, xs, int(m), xd, part, st);
      for (int64_t j = 0; j < m; ++j)
        KQR_CHECK_HIP(hipMemcpy2DAsync(U + j, size_t(ldu) * sizeof(double), xd.p[j], sizeof(double), sizeof(double),
                                       size_t(n), hipMemcpyDeviceToDevice, st));
      KQR_CHECK_HIP(hipFreeAsync(V16, st));
      KQR_CHECK_HIP(hipFreeAsync(part, st));
      KQR_CHECK_HIP(hipFreeAsync(cols, st));
      m = 0;  // done
    }
    if (K && m > 1 && mode == KQR_APPLY_FAST) {  // all columns in one pass over K on the matrix cores
      float* V16 = nullptr;
      double* part = nullptr;
      KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&V16), size_t(n) * 16 * sizeof(float), st));
      KQR_CHECK_HIP(
          hipMallocAsync(reinterpret_cast<void**>(&part), kv_scratch_doubles(n) * sizeof(double), st));
      kv_gather_strided(V, ldv, int(m), n, n, V16, st);
      kapply_kv(km, n, V16, int(m), U, ldu, part, st);
      KQR_CHECK_HIP(hipFreeAsync(part, st));
      KQR_CHECK_HIP(hipFreeAsync(V16, st));
      m = 0;  // done
    }
    for (int64_t j = 0; j < m; ++j) {
      const double* col = V + j;
      if (ldv != 1 || (reinterpret_cast<uintptr_t>(col) & 15) != 0) {  // kernels read 16-byte vectors
        KQR_CHECK_HIP(hipMemcpy2DAsync(v64, sizeof(double), V + j, size_t(ldv) * sizeof(double), sizeof(double),
                                       size_t(n), hipMemcpyDeviceToDevice, st));
        col = v64;
      }
      if (K) {
        if (mode == KQR_APPLY_EXACT) {
          kapply_dense(km, n, n, nullptr, col, U + j, ldu, true, st);
        } else {
          to_f32(col, n, 1, 1, v32, 1, st);
          kapply_dense(km, n, n, v32, nullptr, U + j, ldu, false, st);
        }
      } else if (lscr) {
        lin_apply(X, n, int(p), col, U + j, ldu, lscr, st);
      } else if (shift >= 20) {
        kapply_otf_l1q(xq.as<uint32_t>(), n, int(p), gamma, shift, col, U + j, ldu, mode == KQR_APPLY_EXACT, st);
      } else {
        kapply_otf(X, sqn, n, X, sqn, n, int(p), ks, col, U + j, ldu, 1.0, 0.0, st, mode == KQR_APPLY_EXACT);
      }
    }
    if (sqn) KQR_CHECK_HIP(hipFreeAsync(sqn, st));
    if (lscr) KQR_CHECK_HIP(hipFreeAsync(lscr, st));
    KQR_CHECK_HIP(hipFreeAsync(tmp, st));
  });
}

int kqr_kernel_apply_static(const void* K, int k_dtype, int64_t n, int64_t ldk, const double* v, int64_t incv,
                            double* u, int64_t incu, int mode, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(K && v && u, "K, v and u must be non-null");
    KQR_REQUIRE(n >= 1, "need n >= 1");
    KQR_REQUIRE(incv >= 1 && incu >= 1, "need incv >= 1 and incu >= 1");
    KQR_REQUIRE(mode == KQR_APPLY_FAST || mode == KQR_APPLY_EXACT, "mode must be KQR_APPLY_FAST or KQR_APPLY_EXACT");
    check_kmat(K, k_dtype, ldk, n);
    const size_t need = (size_t(n) * 8 + 255) / 256 * 256 + (size_t(n) * 4 + 255) / 256 * 256 + size_t(n) * 8;
    KQR_REQUIRE(need <= static_scratch_bytes(), "n = %lld needs %zu bytes of scratch, above the %zu of the static array",
                (long long)n, need, static_scratch_bytes());
    ensure_device();
    kapply_static(KMat{K, k_dtype, ldk}, n, v, incv, u, incu, mode == KQR_APPLY_EXACT,
                  static_cast<hipStream_t>(stream));
  });
}

int64_t kqr_packed_bytes(int64_t n, int k_dtype) {
  if (n < 1 || (k_dtype != KQR_FP32 && k_dtype != KQR_BF16)) return -1;
  return int64_t(packed_bytes(n, k_dtype));
}

int kqr_kernel_build_packed(const float* X, int64_t n, int64_t p, int kernel, double gamma, int k_dtype, void* K,
                            void* stream) {
  return guarded([&] {
    KQR_REQUIRE(X && K, "pointers must be non-null");
    KQR_REQUIRE(n >= 1 && p >= 1 && p <= 64, "need n >= 1 and 1 <= p <= 64");
    KQR_REQUIRE(k_dtype == KQR_FP32 || k_dtype == KQR_BF16, "k_dtype must be KQR_FP32 or KQR_BF16");
    check_kernel(kernel, gamma, false);
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    float* sqn = nullptr;
    KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&sqn), size_t(n) * sizeof(float), st));
    row_sqnorms(X, n, int(p), sqn, st);
    kbuild_packed(X, sqn, n, int(p), KernelSpec{kernel, gamma}, k_dtype, K, st);
    KQR_CHECK_HIP(hipFreeAsync(sqn, st));
  });
}

int kqr_kernel_apply_packed(const void* K, int k_dtype, int64_t n, const double* v, double* u, int mode,
                            void* stream) {
  return guarded([&] {
    KQR_REQUIRE(K && v && u, "pointers must be non-null");
    KQR_REQUIRE(n >= 1, "need n >= 1");
    KQR_REQUIRE(k_dtype == KQR_FP32 || k_dtype == KQR_BF16, "k_dtype must be KQR_FP32 or KQR_BF16");
    KQR_REQUIRE(mode == KQR_APPLY_FAST || mode == KQR_APPLY_EXACT, "mode must be KQR_APPLY_FAST or KQR_APPLY_EXACT");
    KQR_REQUIRE((reinterpret_cast<uintptr_t>(v) & 15) == 0, "v must be 16-byte aligned");
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    const KMat km{K, k_dtype, packed_tiles_per_side(n), 1};
    if (mode == KQR_APPLY_EXACT) {
      kapply_packed(km, n, nullptr, v, u, 1, true, st);
    } else {
      float* v32 = nullptr;
      KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&v32), size_t(n) * sizeof(float), st));
      to_f32(v, n, 1, 1, v32, 1, st);
      kapply_packed(km, n, v32, nullptr, u, 1, false, st);
      KQR_CHECK_HIP(hipFreeAsync(v32, st));
    }
  });
}

int kqr_autotune_packed(const void* K, int k_dtype, int64_t n, int mode, int reps, char* report, int64_t cap,
                        void* stream) {
  return guarded([&] {
    KQR_REQUIRE(K != nullptr, "K must be non-null");
    KQR_REQUIRE(n >= 1 && reps >= 1, "need n >= 1 and reps >= 1");
    KQR_REQUIRE(k_dtype == KQR_FP32 || k_dtype == KQR_BF16, "k_dtype must be KQR_FP32 or KQR_BF16");
    KQR_REQUIRE(mode == KQR_APPLY_FAST || mode == KQR_APPLY_EXACT, "mode must be KQR_APPLY_FAST or KQR_APPLY_EXACT");
    ensure_device();
    autotune_packed(KMat{K, k_dtype, packed_tiles_per_side(n), 1}, n, mode == KQR_APPLY_EXACT, reps, report, cap,
                    static_cast<hipStream_t>(stream));
  });
}

int kqr_set_packed_shape(int k_dtype, int mode, int map, int strip) {
  return guarded([&] {
    KQR_REQUIRE(k_dtype == KQR_FP32 || k_dtype == KQR_BF16, "k_dtype must be KQR_FP32 or KQR_BF16");
    KQR_REQUIRE(mode == KQR_APPLY_FAST || mode == KQR_APPLY_EXACT, "mode must be KQR_APPLY_FAST or KQR_APPLY_EXACT");
    const PackedShape s{map, strip};
    KQR_REQUIRE(packed_shape_supported(s), "need map 0 to 3 with 1 <= strip <= 32, or map 4 or 5 with strip 2 or 4");
    set_packed_shape(k_dtype, mode == KQR_APPLY_EXACT, s);
    tune_record(TuneEntry{"packed", k_dtype, mode == KQR_APPLY_EXACT ? 1 : 0, 0, 1, map, strip, 0, 0, 0.0});
  });
}

int kqr_set_otf_symmetric_limit(int64_t bytes) {
  return guarded([&] {
    KQR_REQUIRE(bytes >= 0, "bytes must be >= 0");
    set_otf_sym_budget(bytes);
  });
}

int kqr_set_otf_shape(int strip, int64_t wgs) {
  return guarded([&] {
    KQR_REQUIRE(strip >= 0 && strip <= kPkMaxStrip, "need 0 <= strip <= 32");
    KQR_REQUIRE(wgs == 0 || (wgs >= 256 && wgs <= (int64_t(1) << 20)), "need wgs = 0 or 256 <= wgs <= 2^20");
    set_otf_shape(strip, wgs);
    for (int64_t nc : {int64_t(1), int64_t(64) * kPkT, int64_t(256) * kPkT, int64_t(1024) * kPkT})
      tune_record(TuneEntry{"otf", 0, 0, nc, 1, strip, 0, 0, wgs, 0.0});
  });
}

int kqr_autotune_otf(const float* X, int64_t n, int64_t p, int kernel, double gamma, int mode, int reps,
                     char* report, int64_t cap, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(X != nullptr, "X must be non-null");
    KQR_REQUIRE(n >= 1 && p >= 1 && p <= 64 && reps >= 1, "need n >= 1, 1 <= p <= 64, reps >= 1");
    KQR_REQUIRE(kernel == KQR_RBF || kernel == KQR_LAPLACIAN, "kernel must be KQR_RBF or KQR_LAPLACIAN");
    KQR_REQUIRE(std::isfinite(gamma) && gamma > 0.0, "gamma must be positive and finite");
    KQR_REQUIRE(mode == KQR_APPLY_FAST || mode == KQR_APPLY_EXACT, "mode must be KQR_APPLY_FAST or KQR_APPLY_EXACT");
    ensure_device();
    autotune_otf(X, n, int(p), KernelSpec{kernel, gamma}, mode == KQR_APPLY_EXACT, reps, report, cap,
                 static_cast<hipStream_t>(stream));
  });
}

int kqr_tune_save(const char* path, int* count) {
  return guarded([&] {
    KQR_REQUIRE(path != nullptr && count != nullptr, "path and count must be non-null");
    ensure_device();
    *count = tune_save(path);
  });
}

int kqr_tune_load(const char* path, int* count) {
  return guarded([&] {
    KQR_REQUIRE(path != nullptr && count != nullptr, "path and count must be non-null");
    *count = tune_load(path);  // checks the file, then the device
  });
}

int kqr_predict(const float* Xtrain, int64_t n, int64_t p, const double* alpha, double beta, double lambda,
                int kernel, double gamma, const float* Xnew, int64_t m, double* f, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(Xtrain && alpha && Xnew && f, "pointers must be non-null");
    KQR_REQUIRE(n >= 1 && m >= 1 && p >= 1 && p <= 64, "need n, m >= 1 and 1 <= p <= 64");
    KQR_REQUIRE(std::isfinite(lambda) && lambda > 0.0, "lambda must be positive");
    KQR_REQUIRE(std::isfinite(beta), "beta must be finite");
    check_kernel(kernel, gamma);
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (kernel == KQR_LINEAR) {  // f = beta + Xnew (Xtrain^T alpha) / lambda
      double* scr = nullptr;
      KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&scr), lin_scratch_doubles(int(p)) * sizeof(double), st));
      lin_predict(Xtrain, n, int(p), alpha, Xnew, m, 1.0 / lambda, beta, f, scr, st);
      KQR_CHECK_HIP(hipFreeAsync(scr, st));
      return;
    }
    float* sq = nullptr;
    KQR_CHECK_HIP(hipMallocAsync(reinterpret_cast<void**>(&sq), size_t(n + m) * sizeof(float), st));
    row_sqnorms(Xtrain, n, int(p), sq, st);
    row_sqnorms(Xnew, m, int(p), sq + n, st);
    kapply_otf(Xnew, sq + n, m, Xtrain, sq, n, int(p), KernelSpec{kernel, gamma}, alpha, f, 1, 1.0 / lambda, beta, st,
               true);
    KQR_CHECK_HIP(hipFreeAsync(sq, st));
  });
}

int kqr_rpcholesky(const float* X, int64_t n, int64_t p, int kernel, double gamma, const void* K, int k_dtype,
                   int64_t ldk, int64_t rank, const double* uniforms, float* F, int64_t ldf, int64_t* pivots,
                   int64_t* rank_out, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(uniforms && F && pivots && rank_out, "pointers must be non-null");
    KQR_REQUIRE(n >= 1 && rank >= 1 && rank <= 1024, "need n >= 1 and 1 <= rank <= 1024");
    KQR_REQUIRE(ldf >= std::min(rank, n) && ldf % 4 == 0, "ldf must be >= rank and a multiple of 4");
    for (int64_t i = 0; i < std::min(rank, n); ++i)
      KQR_REQUIRE(uniforms[i] >= 0.0 && uniforms[i] < 1.0, "uniforms must lie in [0, 1)");
    if (!K) {
      KQR_REQUIRE(X != nullptr, "X must be non-null when K is NULL");
      KQR_REQUIRE(p >= 1 && p <= 64, "need 1 <= p <= 64");
      check_kernel(kernel, gamma, false);
    }
    check_kmat(K, k_dtype, ldk, n);
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    DevBuf sqn(size_t(n) * sizeof(float));
    if (X) row_sqnorms(X, n, int(p), sqn.as<float>(), st);
    KQR_CHECK_HIP(hipMemsetAsync(F, 0, size_t(n) * ldf * sizeof(float), st));
    Exec ex(st);
    std::vector<int64_t> piv = run_sync(rpcholesky(KMat{K, k_dtype, ldk}, X, sqn.as<float>(), n, int(p),
                                                   KernelSpec{kernel, gamma}, rank, uniforms, F, ldf, ex));
    for (size_t i = 0; i < piv.size(); ++i) pivots[i] = piv[i];
    *rank_out = int64_t(piv.size());
  });
}

int kqr_adaptive_rank(const float* F0, int64_t n, int64_t r0, int64_t ldf, double xi, int64_t* rank,
                      double* lambda1, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(F0 && rank, "F0 and rank must be non-null");
    KQR_REQUIRE(n >= 1 && r0 >= 1 && r0 <= 1023, "need n >= 1 and 1 <= r0 <= 1023");
    KQR_REQUIRE(ldf >= r0 && ldf % 4 == 0, "ldf must be >= r0 and a multiple of 4");
    KQR_REQUIRE(xi > 0.0 && xi < 1.0, "need 0 < xi < 1");
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    double l1 = 0.0;
    Exec ex(st);
    *rank = r0 <= 1 ? r0 : run_sync(adaptive_rank(F0, n, r0, ldf, xi, ex, &l1));
    if (lambda1) *lambda1 = l1;
  });
}

int kqr_autotune_apply(const void* K, int k_dtype, int64_t n, int64_t ldk, int mode, int reps, char* report,
                       int64_t cap, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(K != nullptr, "K must be non-null");
    KQR_REQUIRE(n >= 1 && reps >= 1, "need n >= 1 and reps >= 1");
    KQR_REQUIRE(mode == KQR_APPLY_FAST || mode == KQR_APPLY_EXACT || mode == KQR_APPLY_KV, "invalid mode");
    check_kmat(K, k_dtype, ldk, n);
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    const KMat km{K, k_dtype, ldk};
    if (mode == KQR_APPLY_KV) {
      autotune_kv(km, n, reps, report, cap, st);
      return;
    }
    DevBuf v64(size_t(n) * sizeof(double)), v32(size_t(n) * sizeof(float)), u(size_t(n) * sizeof(double));
    fill(n, 1.0 / double(n), v64.as<double>(), st);
    to_f32(v64.as<double>(), n, 1, 1, v32.as<float>(), 1, st);
    hipEvent_t e0, e1;
    KQR_CHECK_HIP(hipEventCreate(&e0));
    KQR_CHECK_HIP(hipEventCreate(&e1));
    std::string rep = "{\"n\": " + std::to_string(n) + ", \"k_dtype\": " + std::to_string(k_dtype) +
                      ", \"mode\": " + std::to_string(mode) + ", \"shapes\": [";
    ApplyShape best;
    double best_us = 1e300;
    bool first = true;
    const int rows_c[] = {2, 4, 8}, unroll_c[] = {1, 2, 4}, segs_c[] = {1, 2, 4, 8, 16};
    try {
      for (int rw : rows_c)
        for (int un : unroll_c)
          for (int sg : segs_c) {
            ApplyShape s;
            s.rows = rw;
            s.unroll = un;
            s.segs = sg;
            const bool ex = mode == KQR_APPLY_EXACT;
            kapply_dense(km, n, n, v32.as<float>(), v64.as<double>(), u.as<double>(), 1, ex, st, &s);  // warm-up
            KQR_CHECK_HIP(hipEventRecord(e0, st));
            for (int k = 0; k < reps; ++k)
              kapply_dense(km, n, n, v32.as<float>(), v64.as<double>(), u.as<double>(), 1, ex, st, &s);
            KQR_CHECK_HIP(hipEventRecord(e1, st));
            KQR_CHECK_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            KQR_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
            const double us = 1e3 * ms / reps;
            char buf[128];
            snprintf(buf, sizeof(buf), "%s{\"rows\": %d, \"unroll\": %d, \"segs\": %d, \"us\": %.2f}", first ? "" : ", ",
                     rw, un, sg, us);
            first = false;
            rep += buf;
            if (us < best_us) { best_us = us; best = s; }
          }
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_apply_shape(k_dtype, mode == KQR_APPLY_EXACT, n, best);
    tune_record(TuneEntry{"apply", k_dtype, mode == KQR_APPLY_EXACT ? 1 : 0, n, 1, best.rows, best.unroll, best.segs, 0,
                          best_us});
    char buf[160];
    snprintf(buf, sizeof(buf), "], \"best\": {\"rows\": %d, \"unroll\": %d, \"segs\": %d, \"us\": %.2f}}", best.rows,
             best.unroll, best.segs, best_us);
    rep += buf;
    if (report && cap > 0) {
      const size_t nb = std::min<size_t>(size_t(cap) - 1, rep.size());
      memcpy(report, rep.data(), nb);
      report[nb] = '\0';
    }
  });
}

int kqr_set_apply_shape(int k_dtype, int mode, int64_t n, int rows, int unroll, int segs) {
  return guarded([&] {
    KQR_REQUIRE(k_dtype == KQR_FP32 || k_dtype == KQR_BF16, "invalid k_dtype");
    KQR_REQUIRE(mode == KQR_APPLY_FAST || mode == KQR_APPLY_EXACT, "invalid mode");
    ApplyShape s;
    s.rows = rows;
    s.unroll = unroll;
    s.segs = segs;
    KQR_REQUIRE(apply_shape_supported(s), "unsupported shape (rows in {2,4,8}, unroll in {1,2,4}, 1 <= segs <= 64)");
    set_apply_shape(k_dtype, mode == KQR_APPLY_EXACT, n, s);
    tune_record(TuneEntry{"apply", k_dtype, mode == KQR_APPLY_EXACT ? 1 : 0, n, 1, rows, unroll, segs, 0, 0.0});
  });
}

int kqr_set_kv_shape(int k_dtype, int64_t n, int nld, int prefetch, int segs) {
  return guarded([&] {
    KQR_REQUIRE(k_dtype == KQR_FP32 || k_dtype == KQR_BF16, "invalid k_dtype");
    KQR_REQUIRE(prefetch == 0 || prefetch == 1, "prefetch must be 0 or 1");
    KvShape s;
    s.nld = nld;
    s.prefetch = prefetch;
    s.segs = segs;
    KQR_REQUIRE(kv_shape_supported(s), "unsupported K V shape (nld in {0,4,8}, 1 <= segs <= 8)");
    set_kv_shape(k_dtype, n, s);
    tune_record(TuneEntry{"kv", k_dtype, 0, n, 16, nld, prefetch, segs, 0, 0.0});
  });
}

int kqr_woodbury_apply(const float* F, int64_t n, int64_t r, int64_t ldf, double c, const double* Ldiag,
                       const double* w, double* out, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(Ldiag && w && out, "pointers must be non-null");
    KQR_REQUIRE(n >= 1 && r >= 0 && r <= 1023, "need n >= 1 and 0 <= r <= 1023");
    KQR_REQUIRE(r == 0 || (F && ldf >= r && ldf % 4 == 0), "F must be non-null with ldf >= r, ldf a multiple of 4");
    KQR_REQUIRE(std::isfinite(c) && c > 0.0, "c must be positive");
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace ws(st);
    Exec ex(st);
    Woodbury P(F, n, r, ldf);
    if (!run_sync(P.build(Ldiag, c, ex))) fail(KQR_ENUMERIC, "Woodbury core is not positive definite");
    P.apply(w, out, nullptr, nullptr, ws, st);
    KQR_CHECK_HIP(hipStreamSynchronize(st));
  });
}

int kqr_pcg_solve(const float* X, int64_t n, int64_t p, int kernel, double gamma, const void* K, int k_dtype,
                  int64_t ldk, const float* F, int64_t r, int64_t ldf, double c, const double* Ldiag, const double* b,
                  double tol, int maxit, double* x, int* iters, double* resnorm, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(Ldiag && b && x && iters && resnorm, "pointers must be non-null");
    KQR_REQUIRE(n >= 1 && r >= 0 && r <= 1023 && maxit >= 0, "need n >= 1, 0 <= r <= 1023, maxit >= 0");
    KQR_REQUIRE(r == 0 || (F && ldf >= r && ldf % 4 == 0), "F must be non-null with ldf >= r, ldf a multiple of 4");
    KQR_REQUIRE(std::isfinite(c) && c >= 0.0 && tol >= 0.0, "need c >= 0 and tol >= 0");
    KQR_REQUIRE(X != nullptr && p >= 1 && p <= 64, "X must be non-null with 1 <= p <= 64");
    check_kernel(kernel, gamma);
    check_kmat(K, k_dtype, ldk, n);
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    Operator op(X, n, int(p), KernelSpec{kernel, gamma}, KMat{K, k_dtype, ldk}, st);
    Workspace ws(st);
    Exec ex(st);
    Pcg pcg(op, ws, n, ex);
    std::unique_ptr<Woodbury> P;
    if (r > 0) {
      P.reset(new Woodbury(F, n, r, ldf));
      if (!run_sync(P->build(Ldiag, c, ex))) fail(KQR_ENUMERIC, "Woodbury core is not positive definite");
    }
    PcgStats s = run_sync(
        pcg.solve(c, Ldiag, P.get(), b, x, nullptr, false, tol, maxit, K != nullptr && k_dtype == KQR_FP32));
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    *iters = s.iters;
    *resnorm = s.resnorm;
  });
}

int kqr_ssn_gradient(int64_t n, double tau, double lambda, double beta, double sigma, double tau1, double tau2,
                     double eps_floor, const double* alpha, const double* Kalpha, const double* y, const double* z,
                     double* grad, uint8_t* S, double* Ldiag, double* rhs, double* gnorm, double* eps_t,
                     void* stream) {
  return guarded([&] {
    KQR_REQUIRE(alpha && Kalpha && y && z && grad && S && Ldiag && rhs && gnorm && eps_t, "pointers must be non-null");
    KQR_REQUIRE(n >= 1 && tau > 0.0 && tau < 1.0, "need n >= 1 and 0 < tau < 1");
    KQR_REQUIRE(lambda > 0.0 && sigma > 0.0 && tau1 > 0.0 && tau2 > 0.0 && eps_floor >= 0.0,
                "need positive lambda, sigma, tau1, tau2");
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace ws(st);
    DevBuf red(8 * sizeof(double));
    HostPinned h(8 * sizeof(double));
    vec_dots(n, alpha, nullptr, ws, red.as<double>(), st);
    KQR_CHECK_HIP(hipMemcpyAsync(h.ptr, red.ptr, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    const double sa = h.as<double>()[0];
    ssn_grad(n, alpha, Kalpha, y, z, beta, sigma, sa, tau, lambda, grad, S, ws, red.as<double>(), st);
    KQR_CHECK_HIP(hipMemcpyAsync(h.ptr, red.ptr, sizeof(double), hipMemcpyDeviceToHost, st));
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    const double gn = std::sqrt(h.as<double>()[0]);
    const double et = std::max(tau1 * std::min(tau2, gn), eps_floor);
    ssn_system(n, S, grad, lambda, sigma, et, Ldiag, rhs, st);
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    *gnorm = gn;
    *eps_t = et;
  });
}

int kqr_kkt_residuals(int64_t n, double tau, double lambda, double beta, double sigma, double step, int update,
                      const double* alpha, const double* Kalpha, const double* y, double* z, double* v, double* out,
                      void* stream) {
  return guarded([&] {
    KQR_REQUIRE(alpha && Kalpha && y && z && v && out, "pointers must be non-null");
    KQR_REQUIRE(n >= 1 && tau > 0.0 && tau < 1.0, "need n >= 1 and 0 < tau < 1");
    KQR_REQUIRE(std::isfinite(lambda) && lambda > 0.0 && std::isfinite(beta), "need lambda > 0 and finite beta");
    KQR_REQUIRE(update == 0 || update == 1, "update must be 0 or 1");
    KQR_REQUIRE(update == 0 || (std::isfinite(sigma) && sigma > 0.0 && std::isfinite(step)),
                "the multiplier step needs sigma > 0 and a finite step");
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace ws(st);
    DevBuf red(16 * sizeof(double));
    HostPinned h(16 * sizeof(double));
    vec_dots(n, y, nullptr, ws, red.as<double>(), st);  // [sum, -, ||y||^2]
    KQR_CHECK_HIP(hipMemcpyAsync(h.ptr, red.ptr, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    const double ynorm = std::sqrt(std::max(h.as<double>()[2], 0.0));
    multiplier_kkt(n, alpha, Kalpha, y, z, v, beta, update ? sigma : 1.0, update ? step : 0.0, tau, lambda,
                   update != 0, ws, red.as<double>(), st);
    KQR_CHECK_HIP(hipMemcpyAsync(h.ptr, red.ptr, kKktSums * sizeof(double), hipMemcpyDeviceToHost, st));
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    const Kkt k = kkt_from_sums(h.as<double>(), ynorm, lambda);
    const double vals[7] = {k.eta_p, k.eta_d, k.eta_c, k.eta_kkt, k.eta_gap, k.obj_p, k.obj_d};
    memcpy(out, vals, sizeof(vals));
  });
}

int kqr_fit(const float* X, const double* y, int64_t n, int64_t p, double tau, double lambda, int kernel, double gamma,
            const kqr_options* opt, double* alpha, double* beta, kqr_info* info, void* stream) {
  int converged = 0;
  int st_code = guarded([&] {
    KQR_REQUIRE(X && y && alpha && beta, "X, y, alpha and beta must be non-null");
    KQR_REQUIRE(n >= 2 && p >= 1 && p <= 64, "need n >= 2 and 1 <= p <= 64");
    KQR_REQUIRE(tau > 0.0 && tau < 1.0, "need 0 < tau < 1");
    KQR_REQUIRE(std::isfinite(lambda) && lambda > 0.0, "lambda must be positive and finite");
    check_kernel(kernel, gamma);
    kqr_options o;
    kqr_default_options(&o);
    if (opt) o = *opt;
    validate_options(o);
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    const KernelSpec ks{kernel, gamma};
    Exec ex(st);
    Prepared pr = run_sync(prepare_fit(X, n, int(p), ks, o, ex));
    Operator op(X, n, int(p), ks, pr.kmat(), st);
    pr.attach(op);
    op.enable_profile(o.profile != 0);
    FitOutcome out = run_sync(run_fit(op, pr, y, n, tau, lambda, o, alpha, ex, o.z_out, o.v_out));
    *beta = out.beta;
    converged = out.converged;
    if (info) *info = out.info;
  });
  if (st_code == KQR_OK && !converged) return KQR_NOT_CONVERGED;
  return st_code;
}

int kqr_fit_multi_tau(const float* X, const double* y, int64_t n, int64_t p, const double* taus, int ntau,
                      double lambda, int kernel, double gamma, const kqr_options* opt, double* alpha, double* beta,
                      kqr_info* info, int* status, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(X && y && taus && alpha && beta && status, "pointers must be non-null");
    KQR_REQUIRE(n >= 2 && p >= 1 && p <= 64, "need n >= 2 and 1 <= p <= 64");
    KQR_REQUIRE(ntau >= 1 && ntau <= 16, "need 1 <= ntau <= 16");
    for (int t = 0; t < ntau; ++t) KQR_REQUIRE(taus[t] > 0.0 && taus[t] < 1.0, "need 0 < tau < 1 for every level");
    KQR_REQUIRE(std::isfinite(lambda) && lambda > 0.0, "lambda must be positive and finite");
    check_kernel(kernel, gamma);
    kqr_options o;
    kqr_default_options(&o);
    if (opt) o = *opt;
    validate_options(o);
    ensure_device();
    fit_multi_tau(X, y, n, int(p), KernelSpec{kernel, gamma}, taus, ntau, lambda, o, alpha, beta, info, status,
                  static_cast<hipStream_t>(stream));
  });
}

int kqr_fit_path(const float* X, const double* y, int64_t n, int64_t p, double tau, const double* lambdas,
                 int nlam, int kernel, double gamma, const kqr_options* opt, double* alpha, double* beta,
                 kqr_info* info, int* status, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(X && y && lambdas && alpha && beta && status, "pointers must be non-null");
    KQR_REQUIRE(n >= 2 && p >= 1 && p <= 64, "need n >= 2 and 1 <= p <= 64");
    KQR_REQUIRE(nlam >= 1 && nlam <= 4096, "need 1 <= nlam <= 4096");
    KQR_REQUIRE(tau > 0.0 && tau < 1.0, "need 0 < tau < 1");
    for (int t = 0; t < nlam; ++t)
      KQR_REQUIRE(std::isfinite(lambdas[t]) && lambdas[t] > 0.0, "every lambda must be positive and finite");
    check_kernel(kernel, gamma);
    kqr_options o;
    kqr_default_options(&o);
    if (opt) o = *opt;
    validate_options(o);
    ensure_device();
    fit_path(X, y, n, int(p), KernelSpec{kernel, gamma}, tau, lambdas, nlam, o, alpha, beta, info, status,
             static_cast<hipStream_t>(stream));
  });
}

int kqr_fit_batch(int nprob, const float* const* X, const double* const* y, const int64_t* n, int64_t p,
                  const double* tau, const double* lambda, int kernel, const double* gamma, const kqr_options* opt,
                  double* const* alpha, double* beta, kqr_info* info, int* status, void* stream) {
  return guarded([&] {
    KQR_REQUIRE(X && y && n && tau && lambda && gamma && alpha && beta && status, "pointers must be non-null");
    KQR_REQUIRE(nprob >= 1 && nprob <= 256, "need 1 <= nprob <= 256");
    KQR_REQUIRE(p >= 1 && p <= 64, "need 1 <= p <= 64");
    KQR_REQUIRE(kernel == KQR_RBF || kernel == KQR_LAPLACIAN || kernel == KQR_LINEAR,
                "kernel must be KQR_RBF, KQR_LAPLACIAN or KQR_LINEAR");
    for (int i = 0; i < nprob; ++i) {
      KQR_REQUIRE(X[i] && y[i] && alpha[i], "per-problem pointers must be non-null");
      KQR_REQUIRE(n[i] >= 2, "need n_i >= 2");
      KQR_REQUIRE(tau[i] > 0.0 && tau[i] < 1.0, "need 0 < tau_i < 1");
      KQR_REQUIRE(std::isfinite(lambda[i]) && lambda[i] > 0.0, "lambda_i must be positive");
      KQR_REQUIRE(std::isfinite(gamma[i]) && gamma[i] > 0.0, "gamma_i must be positive");
    }
    kqr_options o;
    kqr_default_options(&o);
    if (opt) o = *opt;
    validate_options(o);
    ensure_device();
    fit_batch(nprob, X, y, n, int(p), KernelSpec{kernel, gamma[0]}, tau, lambda, gamma, o, alpha, beta, info, status,
              static_cast<hipStream_t>(stream));
  });
}

int kqr_fit_grad(const float* X, const double* y, int64_t n, int64_t p, double tau, double lambda, int kernel,
                 double gamma, const float* Xval, const double* yval, int64_t nval, const kqr_options* opt,
                 double* alpha, double* beta, double* val_loss, double* grad, int64_t* n_interior, int* polished,
                 kqr_info* info, void* stream) {
  int converged = 0;
  int st_code = guarded([&] {
    KQR_REQUIRE(X && y && Xval && yval && alpha && beta && val_loss && grad, "pointers must be non-null");
    KQR_REQUIRE(n >= 2 && p >= 1 && p <= 64, "need n >= 2 and 1 <= p <= 64");
    KQR_REQUIRE(nval >= 1, "need nval >= 1");
    KQR_REQUIRE(tau > 0.0 && tau < 1.0, "need 0 < tau < 1");
    KQR_REQUIRE(std::isfinite(lambda) && lambda > 0.0, "lambda must be positive and finite");
    check_kernel(kernel, gamma, false);
    kqr_options o;
    kqr_default_options(&o);
    if (opt) o = *opt;
    validate_options(o);
    ensure_device();
    hipStream_t st = static_cast<hipStream_t>(stream);
    const KernelSpec ks{kernel, gamma};
    DevBuf z(size_t(n) * sizeof(double));
    double b = 0.0;
    kqr_info inf{};
    {
      Exec ex(st);
      Prepared pr = run_sync(prepare_fit(X, n, int(p), ks, o, ex));
      Operator op(X, n, int(p), ks, pr.kmat(), st);
      pr.attach(op);
      op.enable_profile(o.profile != 0);
      FitOutcome out = run_sync(run_fit(op, pr, y, n, tau, lambda, o, alpha, ex, z.as<double>()));
      b = out.beta;
      converged = out.converged;
      inf = out.info;
    }  // K and F are released before the adjoint
    const double level = std::max(inf.eta_kkt, inf.eta_gap);
    GradOutcome g = adjoint_gradient(X, n, int(p), ks, tau, lambda, alpha, &b, z.as<double>(), y, Xval, nval, yval,
                                     std::max(level, 1e-16), st);
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    *beta = b;
    *val_loss = g.J;
    grad[0] = g.dgam;
    grad[1] = g.dlam;
    if (n_interior) *n_interior = g.n_interior;
    if (polished) *polished = g.polished ? 1 : 0;
    inf.n_interior = g.n_interior;
    if (info) *info = inf;
  });
  if (st_code == KQR_OK && !converged) return KQR_NOT_CONVERGED;
  return st_code;
}

}  // extern "C"
