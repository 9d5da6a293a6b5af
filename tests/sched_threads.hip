// Host-only test program for the batch schedulers (csrc/coro.h, csrc/sched.hip)
// under ThreadSanitizer.  Built without the HIP runtime: the stream, event and
// copy calls the schedulers make are defined here on a "device" thread that
// runs every enqueued operation in order (one queue for all streams, a valid
// order for in-order streams), after a short random delay.  A fake launcher
// serves the batched K-apply requests (out = 2 v) and, for requests that carry
// a PCG step, writes the step's status pair and completion tag the way the
// step kernels do.  Several host threads, each with a scheduler over its share
// of the fits, meet at one rendezvous, in lock-step and in open rounds; a
// launcher that fails part-way checks that every thread stops.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <functional>
#include <mutex>
#include <random>
#include <stdexcept>
#include <thread>
#include <vector>

#include "coro.h"
#include "pstep.h"

// ----------------------------------------------------------------- fake device
namespace {

struct Device {
  std::mutex mu;
  std::condition_variable cv, idle;
  std::deque<std::function<void()>> q;
  bool busy = false, stop = false;
  std::mt19937 rng;
  std::thread th;
  explicit Device(unsigned seed) : rng(seed), th([this] { loop(); }) {}
  ~Device() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    th.join();
  }
  void loop() {
    for (;;) {
      std::function<void()> f;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !q.empty(); });
        if (q.empty()) return;
        f = std::move(q.front());
        q.pop_front();
        busy = true;
      }
      std::this_thread::sleep_for(std::chrono::microseconds(rng() % 40));
      f();
      {
        std::lock_guard<std::mutex> lk(mu);
        busy = false;
      }
      idle.notify_all();
    }
  }
  void push(std::function<void()> f) {
    {
      std::lock_guard<std::mutex> lk(mu);
      q.push_back(std::move(f));
    }
    cv.notify_one();
  }
  void drain() {
    std::unique_lock<std::mutex> lk(mu);
    idle.wait(lk, [&] { return q.empty() && !busy; });
  }
};

Device* g_dev = nullptr;

}  // namespace

// the opaque runtime types, as this program models them
struct ihipStream_t {
  int id;
};
struct ihipEvent_t {
  std::atomic<uint64_t> recorded{0}, completed{0};
};

extern "C" {
hipError_t hipStreamCreate(hipStream_t* s) {
  static std::atomic<int> next{1};
  *s = new ihipStream_t{next++};
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  g_dev->drain();
  delete s;
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t;
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  g_dev->drain();  // no queued record still refers to it
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  const uint64_t gen = e->recorded.fetch_add(1) + 1;
  g_dev->push([e, gen] {
    uint64_t c = e->completed.load();
    while (c < gen && !e->completed.compare_exchange_weak(c, gen, std::memory_order_release)) {
    }
  });
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  return e->completed.load(std::memory_order_acquire) >= e->recorded.load() ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  while (hipEventQuery(e) != hipSuccess) std::this_thread::yield();
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }  // one queue: in order
hipError_t hipStreamSynchronize(hipStream_t s) {
  hipEvent_t e;
  hipEventCreate(&e);
  hipEventRecord(e, s);
  hipEventSynchronize(e);
  hipEventDestroy(e);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
  g_dev->push([dst, src, bytes] { memcpy(dst, src, bytes); });
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "stub"; }
}

namespace kqr {
[[noreturn]] void fail(int status, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw std::runtime_error(std::string(buf) + " (status " + std::to_string(status) + ")");
}
HostPinned::HostPinned(size_t b) { ptr = calloc(1, b); }
HostPinned::~HostPinned() { free(ptr); }
}  // namespace kqr

// ----------------------------------------------------------------- the batch
namespace {

using namespace kqr;
constexpr int kN = 64;  // vector length of every fit

struct FakeLauncher : BatchLauncher {
  bool steps = false;
  int fail_at = -1;  // throw on this launch (0-based), -1: never
  std::atomic<int> launches{0};
  void launch(const std::vector<int>&, const std::vector<ApplyReq>& reqs, hipStream_t) override {
    if (launches.fetch_add(1) == fail_at) throw std::runtime_error("injected launch failure");
    std::vector<ApplyReq> r = reqs;
    g_dev->push([r] {
      for (const ApplyReq& q : r)
        for (int i = 0; i < kN; ++i) q.out[i] = 2.0 * q.v[i];
    });
  }
  void launch_steps(const std::vector<ApplyReq>& reqs, hipStream_t) override {
    std::vector<PcgStepDesc*> d;
    for (const ApplyReq& q : reqs)
      if (q.step) d.push_back(const_cast<PcgStepDesc*>(q.step));
    if (d.empty()) return;
    // the status values are read on the host after the tag: copy them now
    std::vector<std::pair<double*, double>> w;
    for (PcgStepDesc* s : d) w.emplace_back(s->status, s->c);
    g_dev->push([w] {
      for (const auto& e : w) {
        e.first[0] = e.second;
        e.first[1] = -e.second;
        const double one = 1.0;
        uint64_t bits;
        memcpy(&bits, &one, sizeof bits);
        __atomic_store_n(reinterpret_cast<uint64_t*>(e.first + 2), bits, __ATOMIC_RELEASE);
      }
    });
  }
  bool steps_ok() const override { return steps; }
};

struct FitData {
  double* v;    // "device" vectors of the fit
  double* out;
  std::vector<double> host;
  PcgStepDesc step;
  FitData() : v(new double[kN]), out(new double[kN]), host(kN) {}
  ~FitData() {
    delete[] v;
    delete[] out;
  }
};

std::atomic<long> g_checked{0}, g_bad{0};

Co<Unit> fit(Exec& ex, FitData& d, int id, int iters, bool use_steps) {
  for (int it = 0; it < iters; ++it) {
    const bool fresh = it == 0 || (it + id) % 3 != 0;  // some requests reuse the last v
    if (fresh) {  // "a kernel on the fit's stream" writes v
      double* v = d.v;
      const double base = 1000.0 * id + it;
      g_dev->push([v, base] {
        for (int i = 0; i < kN; ++i) v[i] = base + i;
      });
    }
    ApplyReq r{d.v, d.out, false, nullptr, ex.sched->complete_on_resume() && !fresh};
    if (use_steps && (it + id) % 2 == 0) {
      d.step.status = ex.hbuf.as<double>();
      d.step.c = 7.0 * id + it;
      d.step.status[2] = 0.0;  // the tag the launch sets
      r.step = &d.step;
    }
    co_await ApplyAwait{&ex, r};
    if (r.step) {  // open rounds resume a step's fit after its tag: the status pair is there
      if (d.step.status[0] != d.step.c || d.step.status[1] != -d.step.c) g_bad.fetch_add(1);
    }
    // v and out on the host (read-backs after the launch), out checked against 2 v
    co_await read_back(ex, d.v, sizeof(double) * kN, d.host.data());
    const std::vector<double> vh(d.host);
    co_await read_back(ex, d.out, sizeof(double) * kN, d.host.data());
    for (int i = 0; i < kN; ++i)
      if (d.host[size_t(i)] != 2.0 * vh[size_t(i)]) g_bad.fetch_add(1);
    g_checked.fetch_add(1);
  }
  co_return Unit{};
}

// threads x per_thread fits, each `iters` K-apply requests; returns the
// number of threads that ended with an exception
int run_batch(int threads, int per_thread, int iters, bool open, bool steps, bool profile, int fail_at) {
  FakeLauncher L;
  L.steps = steps;
  L.fail_at = fail_at;
  Rendezvous rv(&L, threads, profile, open);
  std::atomic<int> failed{0};
  std::vector<std::thread> ths;
  for (int t = 0; t < threads; ++t) {
    ths.emplace_back([&, t] {
      hipStream_t st;
      hipStreamCreate(&st);
      std::vector<int> ids;
      for (int k = 0; k < per_thread; ++k) ids.push_back(t * per_thread + k);
      Scheduler sch(&rv, ids);
      std::vector<std::unique_ptr<Exec>> ex;
      std::vector<std::unique_ptr<FitData>> data;
      std::vector<Co<Unit>> tasks;
      for (int k = 0; k < per_thread; ++k) {
        ex.push_back(std::make_unique<Exec>(st, &sch, k));
        data.push_back(std::make_unique<FitData>());
        tasks.push_back(fit(*ex.back(), *data.back(), ids[size_t(k)], iters + (ids[size_t(k)] % 3), steps));
      }
      try {
        sch.run(tasks);
        for (auto& c : tasks) c.result();
      } catch (const std::exception&) {
        failed.fetch_add(1);
      }
      tasks.clear();
      hipStreamSynchronize(st);
      hipStreamDestroy(st);
    });
  }
  for (auto& th : ths) th.join();
  g_dev->drain();
  return failed.load();
}

}  // namespace

int main(int argc, char** argv) {
  Device dev(argc > 1 ? unsigned(atoi(argv[1])) : 12345u);  // seed of the device's delays
  g_dev = &dev;
  struct Case {
    const char* name;
    int threads, per_thread, iters;
    bool open, steps, profile;
    int fail_at;
  } cases[] = {
      {"lock-step rounds", 4, 5, 12, false, false, true, -1},
      {"open rounds", 4, 5, 12, true, false, false, -1},
      {"open rounds with PCG steps", 4, 6, 12, true, true, false, -1},
      {"one thread, open rounds with PCG steps", 1, 8, 10, true, true, false, -1},
  };
  for (const Case& c : cases) {
    g_checked = 0;
    g_bad = 0;
    const int f = run_batch(c.threads, c.per_thread, c.iters, c.open, c.steps, c.profile, c.fail_at);
    printf("%s: %ld applies checked, %ld wrong, %d threads failed\n", c.name, g_checked.load(), g_bad.load(), f);
    if (f != 0 || g_bad.load() != 0 || g_checked.load() == 0) return 1;
  }
  // a launch that throws part-way: every thread stops with an error, none hangs
  for (bool open : {false, true}) {
    const int f = run_batch(4, 4, 20, open, open, false, 5);
    printf("failing launch (%s): %d of 4 threads ended with the error\n", open ? "open" : "lock-step", f);
    if (f == 0) return 1;
  }
  printf("schedulers ok\n");
  return 0;
}
