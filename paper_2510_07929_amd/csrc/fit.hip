// Fit drivers.  One problem: materialise K, RPCholesky (+ the Section 3 rank
// rule), Phase I, Phase II, final residuals.  Batches: the same driver per
// problem as a coroutine; a few host threads (one scheduler and one stream
// each) drive all of them and meet for the batched K-apply launches.
#include "fit.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>

namespace kqr {

double wall_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// SplitMix64 (Steele, Lea, Flood 2014) on seed + i, top 53 bits -> [0, 1).
std::vector<double> default_uniforms(uint64_t seed, int64_t count) {
  std::vector<double> u(size_t(std::max<int64_t>(count, 0)));
  for (int64_t i = 0; i < count; ++i) {
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * uint64_t(i + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    u[size_t(i)] = double(z >> 11) * (1.0 / 9007199254740992.0);
  }
  return u;
}

#define KQR_OPT_REQUIRE(cond, msg) \
  do {                             \
    if (!(cond)) fail(KQR_EINVAL, msg); \
  } while (0)

void validate_options(const kqr_options& o) {
  KQR_OPT_REQUIRE(o.tol > 0.0 && o.admm_tol > 0.0 && o.admm_sigma > 0.0, "tolerances and sigma must be positive");
  KQR_OPT_REQUIRE(o.admm_step > 0.0 && o.admm_step < 1.6180339887498949, "admm_step must lie in (0, (1+sqrt 5)/2)");
  KQR_OPT_REQUIRE(o.admm_max_iter >= 0 && o.alm_max_iter >= 0 && o.pcg_max_iter >= 1, "iteration caps must be >= 0");
  KQR_OPT_REQUIRE(o.etabar > 0.0 && o.etabar < 1.0 && o.iota > 0.0 && o.iota <= 1.0,
                  "need etabar in (0,1), iota in (0,1]");
  KQR_OPT_REQUIRE(o.armijo > 0.0 && o.armijo < 0.5 && o.ls_shrink > 0.0 && o.ls_shrink < 1.0,
                  "need armijo in (0,1/2), ls_shrink in (0,1)");
  KQR_OPT_REQUIRE(o.tau1 > 0.0 && o.tau1 < 1.0 && o.tau2 > 0.0 && o.tau2 < 1.0, "need tau1, tau2 in (0,1)");
  KQR_OPT_REQUIRE(o.k_dtype == KQR_FP32 || o.k_dtype == KQR_BF16, "k_dtype must be KQR_FP32 or KQR_BF16");
  KQR_OPT_REQUIRE(o.kmode >= KQR_KMODE_AUTO && o.kmode <= KQR_KMODE_ON_THE_FLY, "invalid kmode");
  KQR_OPT_REQUIRE(o.exact_k == 0 || o.exact_k == 1, "exact_k must be 0 or 1");
  KQR_OPT_REQUIRE(o.ssn_adapt >= 0.0 && o.ssn_adapt <= 10.0, "need 0 <= ssn_adapt <= 10");
  KQR_OPT_REQUIRE(o.rank <= 1023, "rank must be <= 1023");
  KQR_OPT_REQUIRE(o.xi > 0.0 && o.xi < 1.0, "need 0 < xi < 1");
  KQR_OPT_REQUIRE(o.sigma_factor >= 1.0 && o.sigma_max >= o.admm_sigma,
                  "need sigma_factor >= 1, sigma_max >= admm_sigma");
  KQR_OPT_REQUIRE(o.ssn_max_iter >= 1 && o.ls_max >= 1 && o.ssn_rel > 0.0, "need ssn_max_iter, ls_max >= 1");
  KQR_OPT_REQUIRE(o.trace_cap >= 0 && (o.trace || o.trace_cap == 0), "trace_cap needs a trace buffer");
  KQR_OPT_REQUIRE(o.k_layout == 0 || o.k_layout == 1, "k_layout must be 0 (full) or 1 (packed)");
  KQR_OPT_REQUIRE(!o.warm_alpha || (o.warm_v && o.warm_z), "a warm start needs warm_alpha, warm_v and warm_z");
  KQR_OPT_REQUIRE(std::isfinite(o.warm_beta) && std::isfinite(o.warm_sigma) && o.warm_sigma >= 0.0,
                  "warm_beta must be finite and warm_sigma >= 0");
}

Co<Prepared> prepare_fit(const float* X, int64_t n, int p, KernelSpec ks, kqr_options o, Exec& ex) {
  const hipStream_t st = ex.st;
  Prepared pr;
  if (ks.kind == KQR_LINEAR) {
    // K = X X^T is applied in factored form and X is its exact factor: the
    // preconditioner (3.2) takes F = X (rank p), or none when rank < 0
    const double t1 = wall_seconds();
    if (o.rank >= 0) {
      pr.rank = p;
      pr.ldf = std::max<int64_t>(4, (p + 3) / 4 * 4);
      pr.F.alloc(size_t(n) * pr.ldf * sizeof(float));
      lin_factor(X, n, p, pr.F.as<float>(), pr.ldf, st);
    }
    co_await fence(ex);
    pr.t_precond = wall_seconds() - t1;
    co_return pr;
  }
  const double t0 = wall_seconds();
  pr.dtype = o.k_dtype;
  pr.layout = o.k_layout;
  const int esz = o.k_dtype == KQR_BF16 ? 2 : 4;
  pr.ldk = pr.layout == 1 ? packed_tiles_per_side(n) : (n + 63) / 64 * 64;
  const size_t kbytes = pr.layout == 1 ? packed_bytes(n, o.k_dtype) : size_t(n) * size_t(pr.ldk) * esz;
  bool materialize = o.kmode == KQR_KMODE_MATERIALIZE;
  if (o.kmode == KQR_KMODE_AUTO) {
    size_t freeb = 0, totalb = 0;
    KQR_CHECK_HIP(hipMemGetInfo(&freeb, &totalb));
    materialize = kbytes < freeb / 10 * 8;
  }
  DevBuf sqn(size_t(n) * sizeof(float));
  row_sqnorms(X, n, p, sqn.as<float>(), st);
  if (materialize && pr.layout == 1) {
    pr.K.alloc(kbytes);
    kbuild_packed(X, sqn.as<float>(), n, p, ks, o.k_dtype, pr.K.ptr, st);
    if (o.k_dtype == KQR_BF16 && o.exact_k == 1) {
      pr.K32.alloc(packed_bytes(n, KQR_FP32));
      kbuild_packed(X, sqn.as<float>(), n, p, ks, KQR_FP32, pr.K32.ptr, st);
    }
  } else if (materialize) {
    pr.K.alloc(kbytes);
    kbuild(X, sqn.as<float>(), n, p, ks, o.k_dtype, pr.K.ptr, pr.ldk, st);
    if (o.k_dtype == KQR_BF16 && o.exact_k == 1) {
      pr.K32.alloc(size_t(n) * size_t(pr.ldk) * 4);
      kbuild(X, sqn.as<float>(), n, p, ks, KQR_FP32, pr.K32.ptr, pr.ldk, st);
    }
  }
  co_await fence(ex);
  pr.t_kbuild = wall_seconds() - t0;
  const double t1 = wall_seconds();
  int64_t rank = 0;
  if (o.rank > 0) rank = std::min<int64_t>(o.rank, n);
  else if (o.rank == 0) rank = std::min<int64_t>(int64_t(std::ceil(std::sqrt(double(n)))), std::min<int64_t>(n, 1023));
  pr.ldf = std::max<int64_t>(4, (rank + 3) / 4 * 4);
  if (rank > 0) {
    pr.F.alloc(size_t(n) * pr.ldf * sizeof(float));
    KQR_CHECK_HIP(hipMemsetAsync(pr.F.ptr, 0, size_t(n) * pr.ldf * sizeof(float), st));
    std::vector<double> u;
    const double* uni = o.pivot_uniforms;
    if (!uni) {
      u = default_uniforms(o.seed, rank);
      uni = u.data();
    }
    std::vector<int64_t> piv = co_await rpcholesky(pr.kmat(), X, sqn.as<float>(), n, p, ks, rank, uni,
                                                   pr.F.as<float>(), pr.ldf, ex);
    pr.rank = int64_t(piv.size());
    // Section 3 rule: keep the first r columns (the first r steps of
    // RPCholesky are RPCholesky(K, r) on the same draws)
    if (o.rank == 0 && pr.rank > 1)
      pr.rank = co_await adaptive_rank(pr.F.as<float>(), n, pr.rank, pr.ldf, o.xi, ex, nullptr);
  }
  co_await fence(ex);
  pr.t_precond = wall_seconds() - t1;
  co_return pr;
}

Co<FitOutcome> run_fit(Operator& op, const Prepared& pr, const double* y, int64_t n, double tau, double lam,
                       kqr_options o, double* alpha_out, Exec& ex, double* z_out, double* v_out) {
  const hipStream_t st = ex.st;
  FitOutcome out;
  kqr_info& inf = out.info;
  memset(&inf, 0, sizeof(inf));
  const double t0 = wall_seconds();
  inf.rank_used = int(pr.rank);
  inf.t_kbuild = pr.t_kbuild;
  inf.t_precond = pr.t_precond;
  Solver solver(op, ex, y, n, tau, lam, o, pr.F.as<float>(), pr.rank, pr.ldf);
  co_await solver.init();
  if (o.warm_alpha) co_await solver.warm_start(inf);  // Phase II from the given iterate
  else co_await solver.phase1(inf);
  co_await solver.phase2(inf);
  co_await solver.finish(inf);
  KQR_CHECK_HIP(hipMemcpyAsync(alpha_out, solver.alpha(), size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (z_out)
    KQR_CHECK_HIP(hipMemcpyAsync(z_out, solver.z(), size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (v_out)
    KQR_CHECK_HIP(hipMemcpyAsync(v_out, solver.v(), size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, st));
  co_await fence(ex);
  out.beta = solver.beta();
  out.converged = solver.converged();
  inf.kapply_calls = op.calls();
  op.profile_totals(inf.kapply_fast_calls, inf.t_kapply_fast, inf.kapply_exact_calls, inf.t_kapply_exact);
  inf.t_total = pr.t_kbuild + pr.t_precond + (wall_seconds() - t0);
  co_return out;
}

// ================================================================= batch launchers
// Shared K: gather the requests into V (n x 16 FP32), one K V launch, scatter.
// With an FP32 K, requests for the exact operator (up to kKvMaxExact per
// launch) are served by the same pass over K in FP64.
// Whether the batches also run their PCG iterations' vector and
// preconditioner work in batched launches (kqr_test_batch_steps).
std::atomic<bool> g_batch_steps{true};

class KvLauncher : public BatchLauncher {
 public:
  KvLauncher(KMat km, int64_t n)
      : km_(km), n_(n), npad_(std::max<int64_t>(km.ld, n)), V_(size_t(npad_) * 16 * sizeof(float)),
        U_(size_t(n) * 16 * sizeof(double)), part_(kv_scratch_doubles(n) * sizeof(double)) {}
  bool exact_ok() const override { return km_.dtype == KQR_FP32 && km_.layout == 0; }
  // No batched PCG steps here: in the lock-step rounds of a shared K, the
  // fits' own step kernels run side by side on their streams, and eleven
  // batched launches in a row on the launch stream made a lambda path slower
  // (1.02-1.10 s against 1.01-1.03 s for 50 values at n = 20,000).
  void launch(const std::vector<int>& slots, const std::vector<ApplyReq>& reqs, hipStream_t st) override {
    (void)slots;
    if (reqs.size() > size_t(kKvMaxCols)) fail(KQR_EHIP, "internal: %zu requests for one K V launch", reqs.size());
    SrcTable16 src{}, xsrc{};
    DstTable16 dst{}, xdst{};
    int m = 0;
    std::vector<const ApplyReq*> ex;
    for (const ApplyReq& r : reqs) {
      if (r.exact) {
        ex.push_back(&r);
      } else {
        src.p[m] = r.v;
        dst.p[m] = r.out;
        ++m;
      }
    }
    if (m > 0) kv_gather(src, m, n_, npad_, V_.as<float>(), st);
    size_t e = 0;
    if (ex.empty()) {
      kapply_kv(km_, n_, V_.as<float>(), m, U_.as<double>(), 16, part_.as<double>(), st);
    } else {
      // the fast columns with the first exact ones, then any further exact ones
      bool first = true;
      while (e < ex.size()) {
        const int mx = int(std::min<size_t>(kKvMaxExact, ex.size() - e));
        for (int j = 0; j < mx; ++j) {
          xsrc.p[j] = ex[e + size_t(j)]->v;
          xdst.p[j] = ex[e + size_t(j)]->out;
        }
        kapply_kv_mixed(km_, n_, V_.as<float>(), first ? m : 0, U_.as<double>(), 16, xsrc, mx, xdst,
                        part_.as<double>(), st);
        first = false;
        e += size_t(mx);
      }
    }
    if (m > 0) kv_scatter(U_.as<double>(), m, n_, dst, st);
  }

 private:
  KMat km_;
  int64_t n_, npad_;
  DevBuf V_, U_, part_;
};

// Different K_i: one launch over (problem, row block) pairs, dealt to the
// workgroups from a queue (problems_launch), then the batched PCG steps.
class ProblemLauncher : public BatchLauncher {
 public:
  ProblemLauncher(std::vector<KMat> km, std::vector<int64_t> n) : km_(std::move(km)), n_(std::move(n)),
                                                                   q_(km_.size()), steps_(km_.size()) {}
  bool steps_ok() const override { return g_batch_steps.load(); }
  void launch(const std::vector<int>& slots, const std::vector<ApplyReq>& reqs, hipStream_t st) override {
    // largest problems first: their items (the longest rows) are taken
    // first, so the launch does not end on a tail of long items
    std::vector<size_t> order(slots.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return n_[size_t(slots[a])] > n_[size_t(slots[b])]; });
    std::vector<ProblemTask> tasks;
    tasks.reserve(order.size());
    for (size_t k : order) {
      const int s = slots[k];
      ProblemTask t;
      t.K = km_[size_t(s)].K;
      t.ld = km_[size_t(s)].ld;
      t.n = n_[size_t(s)];
      t.dtype = km_[size_t(s)].dtype;
      t.v = reqs[k].v;
      t.u = reqs[k].out;
      tasks.push_back(t);
    }
    q_.launch(tasks, st);
  }
  // the rest of the PCG iterations that came with their K-applies
  void launch_steps(const std::vector<ApplyReq>& reqs, hipStream_t st) override {
    std::vector<PcgStepDesc> steps;
    for (const ApplyReq& r : reqs)
      if (r.step) steps.push_back(*r.step);
    steps_.launch(steps, st);
  }

 private:
  std::vector<KMat> km_;
  std::vector<int64_t> n_;
  ProblemQueue q_;
  PcgStepBatch steps_;
};

// ================================================================= drivers
namespace {
// Host threads of a batch (one scheduler and one stream each): launches
// from one thread are issued one after another, and with every fit's small
// kernels in between the batched launches the host issue rate is what
// limits a batch of small problems, so several threads issue them.  At most
// 16 (and the host's core count); KQR_BATCH_THREADS (1..16) or
// kqr_set_batch_threads overrides.
std::atomic<int> g_batch_threads{-1};  // -1: not read yet; 0: default

int batch_threads(int fits) {
  int limit = g_batch_threads.load();
  if (limit < 0) {
    const char* e = std::getenv("KQR_BATCH_THREADS");
    const int v = e ? std::atoi(e) : 0;
    int expected = -1;
    g_batch_threads.compare_exchange_strong(expected, v >= 1 && v <= 16 ? v : 0);
    limit = g_batch_threads.load();
  }
  if (limit == 0) limit = std::max(1, std::min(16, int(std::thread::hardware_concurrency())));
  return std::max(1, std::min(fits, limit));
}

struct StreamSet {
  std::vector<hipStream_t> s;
  explicit StreamSet(int k) : s(size_t(k), nullptr) {
    for (auto& x : s) KQR_CHECK_HIP(hipStreamCreate(&x));
  }
  ~StreamSet() {
    for (auto& x : s)
      if (x) {
        (void)hipStreamSynchronize(x);
        (void)hipStreamDestroy(x);
      }
  }
  StreamSet(const StreamSet&) = delete;
  StreamSet& operator=(const StreamSet&) = delete;
};

int status_of(const std::exception_ptr& e, std::string& msg) {
  try {
    std::rethrow_exception(e);
  } catch (const Error& er) {
    msg = er.what();
    return er.status;
  } catch (const std::exception& er) {
    msg = er.what();
    return KQR_EHIP;
  } catch (...) {
    msg = "unknown failure";
    return KQR_EHIP;
  }
}

// Result of one fit of a batch: its outcome or the exception that ended it.
struct Slotted {
  FitOutcome out;
  std::exception_ptr err;
};

// Runs one fit inside a batch; failures stay with that fit.
Co<Unit> guarded_fit(Operator& op, const Prepared& pr, const double* y, int64_t n, double tau, double lam,
                     kqr_options o, double* alpha, Exec& ex, Slotted& res) {
  try {
    res.out = co_await run_fit(op, pr, y, n, tau, lam, o, alpha, ex);
  } catch (...) {
    res.err = std::current_exception();
  }
  co_return Unit{};
}

// Runs body(g) on threads g = 0 .. T-1 and waits for them.  Buffers released
// on those threads are freed here afterwards (a free waits for the whole
// device); the first exception a thread raised is rethrown.
template <typename Body>
void on_threads(int T, std::vector<void*>& deferred, Body body) {
  std::mutex mu;
  std::exception_ptr first;
  std::vector<std::thread> th;
  for (int g = 0; g < T; ++g) {
    th.emplace_back([&, g] {
      DeferFrees defer;
      try {
        body(g);
      } catch (...) {
        std::lock_guard<std::mutex> lk(mu);
        if (!first) first = std::current_exception();
      }
      std::lock_guard<std::mutex> lk(mu);
      defer.hand_to(deferred);
    });
  }
  for (auto& t : th) t.join();
  if (first) std::rethrow_exception(first);
}

// Writes beta, info and status of every fit; returns the first failure.
void collect(std::vector<Slotted>& res, Rendezvous* rv, double* beta, kqr_info* info, int* status,
             hipStream_t st) {
  const double tb = rv ? rv->device_seconds() : 0.0;
  const int64_t nb = rv ? rv->launches() : 0;
  std::string first_msg;
  int first_err = KQR_OK;
  for (size_t t = 0; t < res.size(); ++t) {
    int stt = KQR_OK;
    if (res[t].err) {
      std::string msg;
      stt = status_of(res[t].err, msg);
      if (first_err == KQR_OK) { first_err = stt; first_msg = msg; }
    } else {
      stt = res[t].out.converged ? KQR_OK : KQR_NOT_CONVERGED;
      beta[t] = res[t].out.beta;
      if (rv) {  // fast applies were the shared batched launches (of every fit)
        res[t].out.info.kapply_fast_calls = nb;
        res[t].out.info.t_kapply_fast = tb;
      }
      if (info) info[t] = res[t].out.info;
    }
    status[t] = stt;
  }
  KQR_CHECK_HIP(hipStreamSynchronize(st));
  if (first_err != KQR_OK) fail(first_err, "%s", first_msg.c_str());
}

void free_all(std::vector<void*>& ptrs) {
  for (void* p : ptrs) (void)hipFree(p);
  ptrs.clear();
}
}  // namespace

void set_batch_threads(int t) { g_batch_threads.store(t); }
void set_batch_steps(bool on) { g_batch_steps.store(on); }

void fit_levels(const float* X, const double* y, int64_t n, int p, KernelSpec ks, const double* taus,
                const double* lams, int nlev, const kqr_options& o_in, double* alpha, double* beta, kqr_info* info,
                int* status, hipStream_t st) {
  kqr_options o = o_in;
  o.trace = nullptr;  // one trace buffer cannot serve several concurrent fits
  o.trace_cap = 0;
  if (o.k_layout != 0) fail(KQR_EINVAL, "joint fits stream K in the full layout (k_layout = 0)");
  if (o.warm_alpha) fail(KQR_EINVAL, "joint fits take no warm start");
  Prepared pr;
  {
    Exec ex0(st);
    pr = run_sync(prepare_fit(X, n, p, ks, o, ex0));
  }
  const int nw = std::min(nlev, kKvMaxCols);  // fits running at once (columns of one K V launch)
  const int T = batch_threads(nw);
  const bool batched = pr.K.ptr != nullptr && nw > 1;
  std::unique_ptr<KvLauncher> launcher;
  std::unique_ptr<Rendezvous> rv;
  if (batched) {
    launcher.reset(new KvLauncher(pr.kmat(), n));
    rv.reset(new Rendezvous(launcher.get(), T, o.profile != 0));
  }
  StreamSet streams(T);
  std::vector<Slotted> res(static_cast<size_t>(nlev));
  std::atomic<int> next{0};
  std::vector<void*> deferred;
  on_threads(T, deferred, [&](int g) {
    // this thread's workers: w = g, g + T, ...; a worker takes the next
    // level when it finishes one and stays in the lock-step rounds until the
    // queue of levels is empty
    std::vector<int> ws;
    for (int w = g; w < nw; w += T) ws.push_back(w);
    Scheduler sched(rv.get(), ws);
    std::vector<std::unique_ptr<Exec>> exs;
    for (size_t k = 0; k < ws.size(); ++k) exs.emplace_back(new Exec(streams.s[size_t(g)], &sched, int(k)));
    auto worker = [&](Exec& ex) -> Co<Unit> {
      for (int t = next++; t < nlev; t = next++) {
        Operator op(X, n, p, ks, pr.kmat(), ex.st);
        pr.attach(op);
        op.enable_profile(o.profile != 0);
        op.attach_batching(batched);
        co_await guarded_fit(op, pr, y, n, taus[t], lams[t], o, alpha + int64_t(t) * n, ex, res[size_t(t)]);
      }
      co_return Unit{};
    };
    std::vector<Co<Unit>> tasks;
    for (auto& e : exs) tasks.push_back(worker(*e));
    sched.run(tasks);
    for (auto& t : tasks) t.result();  // the workers themselves do not fail
  });
  free_all(deferred);
  collect(res, rv.get(), beta, info, status, st);
}

void fit_multi_tau(const float* X, const double* y, int64_t n, int p, KernelSpec ks, const double* taus, int ntau,
                   double lam, const kqr_options& o, double* alpha, double* beta, kqr_info* info, int* status,
                   hipStream_t st) {
  const std::vector<double> lams(static_cast<size_t>(ntau), lam);
  fit_levels(X, y, n, p, ks, taus, lams.data(), ntau, o, alpha, beta, info, status, st);
}

void fit_path(const float* X, const double* y, int64_t n, int p, KernelSpec ks, double tau, const double* lams,
              int nlam, const kqr_options& o, double* alpha, double* beta, kqr_info* info, int* status,
              hipStream_t st) {
  const std::vector<double> taus(static_cast<size_t>(nlam), tau);
  fit_levels(X, y, n, p, ks, taus.data(), lams, nlam, o, alpha, beta, info, status, st);
}

void fit_batch(int nprob, const float* const* X, const double* const* y, const int64_t* n, int p, KernelSpec ks,
               const double* tau, const double* lam, const double* gamma, const kqr_options& o_in,
               double* const* alpha, double* beta, kqr_info* info, int* status, hipStream_t st) {
  kqr_options o = o_in;
  o.trace = nullptr;  // one trace buffer cannot serve several concurrent fits
  o.trace_cap = 0;
  if (o.k_layout != 0) fail(KQR_EINVAL, "batched problems stream K in the full layout (k_layout = 0)");
  if (o.warm_alpha) fail(KQR_EINVAL, "batched fits take no warm start");
  const int T = batch_threads(nprob);
  StreamSet streams(T);
  KQR_CHECK_HIP(hipStreamSynchronize(st));  // the caller's inputs are ready before other streams read them
  // problems dealt to the threads largest first, each to the thread with the
  // least work so far (n^2 per problem)
  std::vector<std::vector<int>> mine(static_cast<size_t>(T));
  {
    std::vector<int> order(static_cast<size_t>(nprob));
    for (int i = 0; i < nprob; ++i) order[size_t(i)] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
    std::vector<double> load(static_cast<size_t>(T), 0.0);
    for (int i : order) {
      const size_t g = size_t(std::min_element(load.begin(), load.end()) - load.begin());
      mine[g].push_back(i);
      load[g] += double(n[i]) * double(n[i]);
    }
  }
  std::vector<void*> deferred;
  // 1. every problem's K and preconditioner
  std::vector<Prepared> prs(static_cast<size_t>(nprob));
  on_threads(T, deferred, [&](int g) {
    const std::vector<int>& ids = mine[size_t(g)];
    Scheduler sched(nullptr, ids);
    std::vector<std::unique_ptr<Exec>> exs;
    std::vector<Co<Prepared>> tasks;
    for (size_t k = 0; k < ids.size(); ++k) {
      const int i = ids[k];
      exs.emplace_back(new Exec(streams.s[size_t(g)], &sched, int(k)));
      tasks.push_back(prepare_fit(X[i], n[i], p, KernelSpec{ks.kind, gamma[i]}, o, *exs.back()));
    }
    sched.run(tasks);
    for (size_t k = 0; k < ids.size(); ++k) prs[size_t(ids[k])] = tasks[k].result();
  });
  free_all(deferred);
  std::vector<KMat> kms;
  std::vector<int64_t> ns;
  bool all_mat = true;
  for (int i = 0; i < nprob; ++i) {
    kms.push_back(prs[size_t(i)].kmat());
    ns.push_back(n[i]);
    all_mat = all_mat && kms.back().K != nullptr;
  }
  // 2. the fits, their fast K-applies in one launch per round
  const bool batched = all_mat && nprob > 1;
  std::unique_ptr<ProblemLauncher> launcher;
  std::unique_ptr<Rendezvous> rv;
  if (batched) {
    launcher.reset(new ProblemLauncher(kms, ns));
    // open rounds when the launches run whole PCG iterations (no read-back per iteration)
    rv.reset(new Rendezvous(launcher.get(), T, o.profile != 0, launcher->steps_ok()));
  }
  std::vector<Slotted> res(static_cast<size_t>(nprob));
  std::vector<std::unique_ptr<Operator>> ops(static_cast<size_t>(nprob));
  on_threads(T, deferred, [&](int g) {
    const std::vector<int>& ids = mine[size_t(g)];
    Scheduler sched(rv.get(), ids);
    std::vector<std::unique_ptr<Exec>> exs;
    std::vector<Co<Unit>> tasks;
    for (size_t k = 0; k < ids.size(); ++k) {
      const int i = ids[k];
      exs.emplace_back(new Exec(streams.s[size_t(g)], &sched, int(k)));
      ops[size_t(i)].reset(new Operator(X[i], n[i], p, KernelSpec{ks.kind, gamma[i]}, kms[size_t(i)], exs.back()->st));
      prs[size_t(i)].attach(*ops[size_t(i)]);
      ops[size_t(i)]->enable_profile(o.profile != 0);
      ops[size_t(i)]->attach_batching(batched);
      tasks.push_back(guarded_fit(*ops[size_t(i)], prs[size_t(i)], y[i], n[i], tau[i], lam[i], o, alpha[i],
                                  *exs.back(), res[size_t(i)]));
    }
    sched.run(tasks);
    for (auto& t : tasks) t.result();
  });
  free_all(deferred);
  collect(res, rv.get(), beta, info, status, st);
}

}  // namespace kqr
