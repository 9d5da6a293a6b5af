// Fit drivers.  One problem: materialise K, RPCholesky (+ the Section 3 rank
// rule), Phase I, Phase II, final residuals.  Batches: one host thread and
// one stream per problem, each running the same driver, with their fast
// K-applies coalesced by a batcher into single launches.
#include "fit.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
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
}

Prepared prepare_fit(const float* X, int64_t n, int p, KernelSpec ks, const kqr_options& o, hipStream_t st) {
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
    KQR_CHECK_HIP(hipStreamSynchronize(st));
    pr.t_precond = wall_seconds() - t1;
    return pr;
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
  KQR_CHECK_HIP(hipStreamSynchronize(st));
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
    std::vector<int64_t> piv = rpcholesky(pr.kmat(), X, sqn.as<float>(), n, p, ks, rank, uni, pr.F.as<float>(),
                                          pr.ldf, st);
    pr.rank = int64_t(piv.size());
    // Section 3 rule: keep the first r columns (the first r steps of
    // RPCholesky are RPCholesky(K, r) on the same draws)
    if (o.rank == 0 && pr.rank > 1) pr.rank = adaptive_rank(pr.F.as<float>(), n, pr.rank, pr.ldf, o.xi, st, nullptr);
  }
  KQR_CHECK_HIP(hipStreamSynchronize(st));
  pr.t_precond = wall_seconds() - t1;
  return pr;
}

FitOutcome run_fit(Operator& op, const Prepared& pr, const double* y, int64_t n, double tau, double lam,
                   const kqr_options& o, double* alpha_out, hipStream_t st, double* z_out, double* v_out) {
  FitOutcome out;
  kqr_info& inf = out.info;
  memset(&inf, 0, sizeof(inf));
  const double t0 = wall_seconds();
  inf.rank_used = int(pr.rank);
  inf.t_kbuild = pr.t_kbuild;
  inf.t_precond = pr.t_precond;
  Solver solver(op, y, n, tau, lam, o, pr.F.as<float>(), pr.rank, pr.ldf, st);
  solver.phase1(inf);
  solver.phase2(inf);
  solver.finish(inf);
  KQR_CHECK_HIP(hipMemcpyAsync(alpha_out, solver.alpha(), size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (z_out)
    KQR_CHECK_HIP(hipMemcpyAsync(z_out, solver.z(), size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (v_out)
    KQR_CHECK_HIP(hipMemcpyAsync(v_out, solver.v(), size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, st));
  KQR_CHECK_HIP(hipStreamSynchronize(st));
  out.beta = solver.beta();
  out.converged = solver.converged();
  inf.kapply_calls = op.calls();
  op.profile_totals(inf.kapply_fast_calls, inf.t_kapply_fast, inf.kapply_exact_calls, inf.t_kapply_exact);
  inf.t_total = pr.t_kbuild + pr.t_precond + (wall_seconds() - t0);
  return out;
}

// ================================================================= batchers
// Rendezvous: a batch goes out when every solver still running has a request
// pending.  Requests are read after the requesting stream's event; every
// requester's stream waits for the batch's completion event.
class RendezvousBatcher : public ApplyBatcher {
 public:
  RendezvousBatcher(int slots, bool profile) : active_(slots), req_(size_t(slots)), ready_(size_t(slots)),
                                                profile_(profile) {
    KQR_CHECK_HIP(hipStreamCreate(&bst_));
    KQR_CHECK_HIP(hipEventCreateWithFlags(&done_, hipEventDisableTiming));
    for (auto& e : ready_) KQR_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  ~RendezvousBatcher() override {
    (void)hipStreamSynchronize(bst_);
    for (auto& s : spans_) {
      (void)hipEventDestroy(s.first);
      (void)hipEventDestroy(s.second);
    }
    for (auto& e : ready_) (void)hipEventDestroy(e);
    (void)hipEventDestroy(done_);
    (void)hipStreamDestroy(bst_);
  }
  void submit(int slot, const double* v, double* out, hipStream_t st, bool exact) override {
    std::unique_lock<std::mutex> lk(mu_);
    KQR_CHECK_HIP(hipEventRecord(ready_[size_t(slot)], st));
    req_[size_t(slot)] = Req{v, out, true, exact};
    ++pending_;
    const uint64_t my_gen = gen_;
    if (pending_ == active_) {
      fire();
    } else {
      cv_.wait(lk, [&] { return gen_ != my_gen || failed_; });
    }
    if (failed_) fail(KQR_EHIP, "batched K-apply failed");
    KQR_CHECK_HIP(hipStreamWaitEvent(st, done_, 0));
  }
  void leave(int slot) override {
    std::unique_lock<std::mutex> lk(mu_);
    (void)slot;
    --active_;
    if (pending_ > 0 && pending_ == active_) {
      try {
        fire();
      } catch (...) {
        failed_ = true;
        cv_.notify_all();
      }
    }
  }
  int64_t launches() const { return launches_; }
  // summed device time of the batched launches (seconds)
  double device_seconds() {
    double t = 0.0;
    for (auto& s : spans_) {
      (void)hipEventSynchronize(s.second);
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, s.first, s.second) == hipSuccess) t += 1e-3 * ms;
    }
    return t;
  }

 protected:
  struct Req {
    const double* v;
    double* out;
    bool live;
    bool exact;
  };
  virtual void launch(const std::vector<int>& slots, hipStream_t st) = 0;
  std::vector<Req> req_;

 private:
  void fire() {
    std::vector<int> slots;
    for (size_t s = 0; s < req_.size(); ++s)
      if (req_[s].live) {
        slots.push_back(int(s));
        KQR_CHECK_HIP(hipStreamWaitEvent(bst_, ready_[s], 0));
      }
    hipEvent_t a = nullptr, b = nullptr;
    if (profile_) {
      KQR_CHECK_HIP(hipEventCreate(&a));
      KQR_CHECK_HIP(hipEventCreate(&b));
      KQR_CHECK_HIP(hipEventRecord(a, bst_));
    }
    try {
      launch(slots, bst_);
    } catch (...) {
      failed_ = true;
      cv_.notify_all();
      throw;
    }
    if (profile_) {
      KQR_CHECK_HIP(hipEventRecord(b, bst_));
      spans_.emplace_back(a, b);
    }
    KQR_CHECK_HIP(hipEventRecord(done_, bst_));
    for (int s : slots) req_[size_t(s)].live = false;
    pending_ = 0;
    ++launches_;
    ++gen_;
    cv_.notify_all();
  }
  std::mutex mu_;
  std::condition_variable cv_;
  int active_;
  int pending_ = 0;
  uint64_t gen_ = 0;
  bool failed_ = false;
  std::vector<hipEvent_t> ready_;
  hipEvent_t done_ = nullptr;
  hipStream_t bst_ = nullptr;
  bool profile_;
  int64_t launches_ = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> spans_;
};

// Shared K: gather the requests into V (n x 16 FP32), one K V launch, scatter.
// With an FP32 K, requests for the exact operator (up to kKvMaxExact per
// launch) are served by the same pass over K in FP64.
class KvBatcher : public RendezvousBatcher {
 public:
  KvBatcher(int slots, KMat km, int64_t n, bool profile)
      : RendezvousBatcher(slots, profile), km_(km), n_(n), npad_(std::max<int64_t>(km.ld, n)),
        V_(size_t(npad_) * 16 * sizeof(float)), U_(size_t(n) * 16 * sizeof(double)),
        part_(kv_scratch_doubles(n) * sizeof(double)) {}
  bool exact_ok() const override { return km_.dtype == KQR_FP32 && km_.layout == 0; }

 protected:
  void launch(const std::vector<int>& slots, hipStream_t st) override {
    SrcTable16 src{}, xsrc{};
    DstTable16 dst{}, xdst{};
    int m = 0;
    std::vector<int> ex;
    for (int s : slots) {
      const Req& r = req_[size_t(s)];
      if (r.exact) {
        ex.push_back(s);
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
          xsrc.p[j] = req_[size_t(ex[e + size_t(j)])].v;
          xdst.p[j] = req_[size_t(ex[e + size_t(j)])].out;
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

// Different K_i: one launch over (problem, row block) pairs.
class ProblemBatcher : public RendezvousBatcher {
 public:
  ProblemBatcher(int slots, std::vector<KMat> km, std::vector<int64_t> n, bool profile)
      : RendezvousBatcher(slots, profile), km_(std::move(km)), n_(std::move(n)),
        tasks_(size_t(km_.size()) * sizeof(ProblemTask)), first_(size_t(km_.size() + 1) * sizeof(int)) {}

 protected:
  void launch(const std::vector<int>& slots, hipStream_t st) override {
    std::vector<ProblemTask> tasks;
    std::vector<int> first;
    int total = 0;
    // largest problems first: their workgroups (the longest rows) start
    // early, so the launch does not end on a tail of long workgroups
    std::vector<int> order(slots);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n_[size_t(a)] > n_[size_t(b)]; });
    for (int s : order) {
      const Req& r = req_[size_t(s)];
      ProblemTask t;
      t.K = km_[size_t(s)].K;
      t.ld = km_[size_t(s)].ld;
      t.n = n_[size_t(s)];
      t.dtype = km_[size_t(s)].dtype;
      t.v = r.v;
      t.u = r.out;
      tasks.push_back(t);
      first.push_back(total);
      total += problem_blocks(t.n);
    }
    first.push_back(total);
    KQR_CHECK_HIP(hipMemcpyAsync(tasks_.ptr, tasks.data(), tasks.size() * sizeof(ProblemTask), hipMemcpyHostToDevice, st));
    KQR_CHECK_HIP(hipMemcpyAsync(first_.ptr, first.data(), first.size() * sizeof(int), hipMemcpyHostToDevice, st));
    KQR_CHECK_HIP(hipStreamSynchronize(st));  // host vectors die at return
    kapply_problems(tasks_.as<ProblemTask>(), int(tasks.size()), first_.as<int>(), total, st);
  }

 private:
  std::vector<KMat> km_;
  std::vector<int64_t> n_;
  DevBuf tasks_, first_;
};

// ================================================================= drivers
namespace {
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
}  // namespace

void fit_levels(const float* X, const double* y, int64_t n, int p, KernelSpec ks, const double* taus,
                const double* lams, int nlev, const kqr_options& o_in, double* alpha, double* beta, kqr_info* info,
                int* status, hipStream_t st) {
  kqr_options o = o_in;
  o.trace = nullptr;  // one trace buffer cannot serve several concurrent fits
  o.trace_cap = 0;
  if (o.k_layout != 0) fail(KQR_EINVAL, "joint fits stream K in the full layout (k_layout = 0)");
  Prepared pr = prepare_fit(X, n, p, ks, o, st);
  const int nw = std::min(nlev, kKvMaxCols);
  const bool batched = pr.K.ptr != nullptr && nw > 1;
  std::unique_ptr<KvBatcher> batcher;
  if (batched) batcher.reset(new KvBatcher(nw, pr.kmat(), n, o.profile != 0));
  StreamSet streams(nw);
  std::vector<std::exception_ptr> errs(static_cast<size_t>(nlev));
  std::vector<FitOutcome> outs(static_cast<size_t>(nlev));
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int w = 0; w < nw; ++w) {
    th.emplace_back([&, w] {
      hipStream_t s = streams.s[size_t(w)];
      // a worker stays in the rendezvous until the queue of levels is empty
      for (int t = next.fetch_add(1); t < nlev; t = next.fetch_add(1)) {
        try {
          Operator op(X, n, p, ks, pr.kmat(), s);
          pr.attach(op);
          op.enable_profile(o.profile != 0);
          if (batcher) op.attach_batcher(batcher.get(), w);
          outs[size_t(t)] = run_fit(op, pr, y, n, taus[t], lams[t], o, alpha + int64_t(t) * n, s);
        } catch (...) {
          errs[size_t(t)] = std::current_exception();
        }
      }
      if (batcher) batcher->leave(w);
    });
  }
  for (auto& x : th) x.join();
  const double tkv = batcher ? batcher->device_seconds() : 0.0;
  const int64_t nkv = batcher ? batcher->launches() : 0;
  std::string first_msg;
  int first_err = KQR_OK;
  for (int t = 0; t < nlev; ++t) {
    int stt = KQR_OK;
    if (errs[size_t(t)]) {
      std::string msg;
      stt = status_of(errs[size_t(t)], msg);
      if (first_err == KQR_OK) { first_err = stt; first_msg = msg; }
    } else {
      stt = outs[size_t(t)].converged ? KQR_OK : KQR_NOT_CONVERGED;
      beta[t] = outs[size_t(t)].beta;
      if (batcher) {  // fast applies were the shared K V launches (of every level)
        outs[size_t(t)].info.kapply_fast_calls = nkv;
        outs[size_t(t)].info.t_kapply_fast = tkv;
      }
      if (info) info[t] = outs[size_t(t)].info;
    }
    status[t] = stt;
  }
  KQR_CHECK_HIP(hipStreamSynchronize(st));
  if (first_err != KQR_OK) fail(first_err, "%s", first_msg.c_str());
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
  std::vector<Prepared> prs;
  prs.reserve(size_t(nprob));
  std::vector<KMat> kms;
  std::vector<int64_t> ns;
  for (int i = 0; i < nprob; ++i) {
    const KernelSpec ksi{ks.kind, gamma[i]};
    prs.push_back(prepare_fit(X[i], n[i], p, ksi, o, st));
    kms.push_back(prs.back().kmat());
    ns.push_back(n[i]);
  }
  bool all_mat = true;
  for (auto& k : kms) all_mat = all_mat && k.K != nullptr;
  std::unique_ptr<ProblemBatcher> batcher;
  if (all_mat && nprob > 1) batcher.reset(new ProblemBatcher(nprob, kms, ns, o.profile != 0));
  StreamSet streams(nprob);
  std::vector<std::exception_ptr> errs(static_cast<size_t>(nprob));
  std::vector<FitOutcome> outs(static_cast<size_t>(nprob));
  std::vector<std::thread> th;
  for (int i = 0; i < nprob; ++i) {
    th.emplace_back([&, i] {
      hipStream_t s = streams.s[size_t(i)];
      try {
        Operator op(X[i], n[i], p, KernelSpec{ks.kind, gamma[i]}, kms[size_t(i)], s);
        prs[size_t(i)].attach(op);
        op.enable_profile(o.profile != 0);
        if (batcher) op.attach_batcher(batcher.get(), i);
        outs[size_t(i)] = run_fit(op, prs[size_t(i)], y[i], n[i], tau[i], lam[i], o, alpha[i], s);
      } catch (...) {
        errs[size_t(i)] = std::current_exception();
      }
      if (batcher) batcher->leave(i);
    });
  }
  for (auto& x : th) x.join();
  const double tb = batcher ? batcher->device_seconds() : 0.0;
  const int64_t nb = batcher ? batcher->launches() : 0;
  std::string first_msg;
  int first_err = KQR_OK;
  for (int i = 0; i < nprob; ++i) {
    int stt = KQR_OK;
    if (errs[size_t(i)]) {
      std::string msg;
      stt = status_of(errs[size_t(i)], msg);
      if (first_err == KQR_OK) { first_err = stt; first_msg = msg; }
    } else {
      stt = outs[size_t(i)].converged ? KQR_OK : KQR_NOT_CONVERGED;
      beta[i] = outs[size_t(i)].beta;
      if (batcher) {
        outs[size_t(i)].info.kapply_fast_calls = nb;
        outs[size_t(i)].info.t_kapply_fast = tb;
      }
      if (info) info[i] = outs[size_t(i)].info;
    }
    status[i] = stt;
  }
  KQR_CHECK_HIP(hipStreamSynchronize(st));
  if (first_err != KQR_OK) fail(first_err, "%s", first_msg.c_str());
}

}  // namespace kqr
