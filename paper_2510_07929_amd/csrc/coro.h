// Host-side sequencing of fits as coroutines.
//
// A fit is host code that enqueues kernels on a stream and, a few times per
// iteration, has to read back a handful of scalars (residual norms, the KKT
// sums) before it can decide what to enqueue next.  Written as a coroutine,
// each read-back is a suspension point: a lone fit (Exec without a scheduler)
// reads synchronously and never suspends, while a batch of fits runs on ONE
// host thread: the scheduler resumes every fit until it suspends on a read or
// on a batched K-apply request, waits for the reads, and issues one launch
// for all pending K-apply requests.  A batch may be split over a few host
// threads (one scheduler and one stream each) that meet for the batched
// launches; the fits themselves never block a thread.
#pragma once

#include <atomic>
#include <condition_variable>
#include <coroutine>
#include <cstring>
#include <exception>
#include <mutex>
#include <utility>

#include "kqr_internal.h"

namespace kqr {

// Lazily started coroutine returning T, awaited by its caller (symmetric
// transfer in both directions, so a chain of awaits costs no stack).
template <typename T>
class Co {
 public:
  struct promise_type {
    T value{};
    std::exception_ptr err;
    std::coroutine_handle<> cont;
    Co get_return_object() { return Co(std::coroutine_handle<promise_type>::from_promise(*this)); }
    std::suspend_always initial_suspend() noexcept { return {}; }
    struct Final {
      bool await_ready() noexcept { return false; }
      std::coroutine_handle<> await_suspend(std::coroutine_handle<promise_type> h) noexcept {
        auto c = h.promise().cont;
        return c ? c : std::noop_coroutine();
      }
      void await_resume() noexcept {}
    };
    Final final_suspend() noexcept { return {}; }
    template <typename U>
    void return_value(U&& v) { value = std::forward<U>(v); }
    void unhandled_exception() { err = std::current_exception(); }
  };
  using handle = std::coroutine_handle<promise_type>;
  Co() = default;
  explicit Co(handle h) : h_(h) {}
  Co(Co&& o) noexcept : h_(std::exchange(o.h_, {})) {}
  Co& operator=(Co&& o) noexcept {
    if (this != &o) { reset(); h_ = std::exchange(o.h_, {}); }
    return *this;
  }
  Co(const Co&) = delete;
  Co& operator=(const Co&) = delete;
  ~Co() { reset(); }
  bool await_ready() const noexcept { return false; }
  std::coroutine_handle<> await_suspend(std::coroutine_handle<> parent) noexcept {
    h_.promise().cont = parent;
    return h_;
  }
  T await_resume() {
    if (h_.promise().err) std::rethrow_exception(h_.promise().err);
    return std::move(h_.promise().value);
  }
  // top-level use (schedulers)
  handle get() const { return h_; }
  bool done() const { return !h_ || h_.done(); }
  T result() { return await_resume(); }

 private:
  void reset() {
    if (h_) h_.destroy();
    h_ = {};
  }
  handle h_;
};

// Value type for coroutines that return nothing useful.
struct Unit {};

class Scheduler;

constexpr size_t kReadBackBytes = 16384;  // largest read-back (1024 RPCholesky pivots, 8 bytes each) and then some

// Execution context of one fit: its stream, a pinned buffer for read-backs
// and, in a batch, its scheduler and slot.  Reads are sequential within a
// fit (each is awaited before the next is issued), so one buffer serves all.
struct Exec {
  hipStream_t st = nullptr;
  Scheduler* sched = nullptr;  // nullptr: reads complete synchronously, K-applies launch directly
  int slot = -1;
  HostPinned hbuf{kReadBackBytes};
  hipEvent_t ev = nullptr;
  explicit Exec(hipStream_t s, Scheduler* sc = nullptr, int sl = -1);
  ~Exec();
  Exec(const Exec&) = delete;
  Exec& operator=(const Exec&) = delete;
};

struct PcgStepDesc;

// Batched K-apply request of one fit: out = K v (fast: FP32 products; exact:
// the exact operator), served by a BatchLauncher.  With step (a launcher
// whose steps_ok() holds), the launch also runs the rest of that fit's PCG
// iteration after the K-apply (pstep.h); the descriptor lives in the
// suspended fit until the launch has been enqueued.
struct ApplyReq {
  const double* v = nullptr;
  double* out = nullptr;
  bool exact = false;
  const PcgStepDesc* step = nullptr;
  // the fit has enqueued nothing since the batched launch that last served it
  // (its inputs come from that launch): the next launch need not wait for its stream
  bool clean = false;
};

// One launch for the K-apply requests of several fits (a shared K: K V; or
// each fit's own K: one launch over (problem, row block) pairs).
class BatchLauncher {
 public:
  virtual ~BatchLauncher() = default;
  // slots[i] asks for reqs[i]; launched on st.
  virtual void launch(const std::vector<int>& slots, const std::vector<ApplyReq>& reqs, hipStream_t st) = 0;
  // The rest of the PCG iterations of the requests that carry a step (after
  // launch, on the same stream; launchers whose steps_ok() holds).
  virtual void launch_steps(const std::vector<ApplyReq>& /*reqs*/, hipStream_t /*st*/) {}
  virtual bool exact_ok() const { return false; }
  virtual bool steps_ok() const { return false; }  // serves ApplyReq::step
};

// Meeting point of the host threads that drive a batch (one Scheduler per
// thread): a batched launch goes out when every thread that still has live
// fits has handed over the K-apply requests of all its fits.  Each thread's
// streams wait for the launch; the launch waits for the work already
// enqueued on every requester stream.
//
// Open mode (a launcher that runs whole PCG iterations, steps_ok()): a round
// goes out as soon as every fit of the last round has come back and handed in
// its next request (or parked on a read-back, or finished), carrying whatever
// requests are pending; fits busy between read-backs (Newton systems, line
// searches, KKT checks) join a later round instead of holding this one.  A
// served fit resumes once the host has seen its part of the round complete
// (for a PCG step, the completion tag it writes into the fit's pinned buffer;
// otherwise the round's event), so no stream waits on the launch on the device.
class Rendezvous {
 public:
  // One open-mode request: out.served is set when a launch carries it.
  struct Pending {
    int id;
    ApplyReq req;
    std::atomic<int>* served;
  };
  Rendezvous(BatchLauncher* launcher, int threads, bool profile, bool open = false);
  ~Rendezvous();
  Rendezvous(const Rendezvous&) = delete;
  Rendezvous& operator=(const Rendezvous&) = delete;
  // Blocks until the launch that carries these requests is enqueued.
  // ids: the problems' batch-wide indices (BatchLauncher slots).
  void arrive(const std::vector<hipStream_t>& streams, const std::vector<int>& ids, const std::vector<ApplyReq>& reqs);
  void leave();  // the calling thread has no live fit left
  // Open mode: `resumed` fits of the last round have come back; regs are the
  // requests they (or fits back from read-backs) made, streams those of them
  // whose stream work so far must precede the launch.
  void hand_in(const std::vector<hipStream_t>& streams, const std::vector<Pending>& regs, int resumed);
  void abort();  // a scheduler failed: the other threads stop
  hipEvent_t done_event() const { return done_; }  // completion of the last round (open mode)
  void check_failed();
  bool open() const { return open_; }
  bool exact_ok() const { return launcher_->exact_ok(); }
  bool steps_ok() const { return launcher_->steps_ok(); }
  int64_t launches() const { return launches_; }
  double device_seconds();  // summed time of the batched launches (profile on)

 private:
  void fire_locked();
  void launch_locked();
  hipEvent_t stream_event(hipStream_t s);
  BatchLauncher* launcher_;
  bool profile_;
  bool open_;
  int inflight_ = 0;  // open mode: fits of the last round not yet back
  std::vector<std::atomic<int>*> served_;
  std::mutex mu_;
  std::condition_variable cv_;
  int active_;
  int arrived_ = 0;
  uint64_t gen_ = 0;
  bool failed_ = false;
  std::vector<int> ids_;
  std::vector<ApplyReq> reqs_;
  std::vector<hipStream_t> streams_;
  std::vector<std::pair<hipStream_t, hipEvent_t>> stream_ev_;
  hipStream_t bst_ = nullptr;
  hipEvent_t done_ = nullptr;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> spans_;
  int64_t launches_ = 0;
};

// Drives a set of fit coroutines on the calling thread.  When no fit can run
// and none waits on a read, every live fit has a K-apply request pending:
// they go to the rendezvous together (lock-step over the fits that have not
// finished).
class Scheduler {
 public:
  // ids[i]: batch-wide index of local slot i (nullptr rendezvous: no batching)
  Scheduler(Rendezvous* rv, std::vector<int> ids);
  // Runs every task to completion (tasks[i] uses slot i); leaves the
  // rendezvous at the end.  Exceptions stay in the tasks (Co::result
  // rethrows them); a failed batched launch is thrown from here.
  template <typename T>
  void run(std::vector<Co<T>>& tasks) {
    std::vector<std::coroutine_handle<>> tops;
    for (auto& t : tasks) tops.push_back(t.get());
    run_handles(tops);
  }
  // parking (called by the awaitables)
  void park_read(int slot, std::coroutine_handle<> h, hipEvent_t ev);
  void park_apply(int slot, std::coroutine_handle<> h, hipStream_t st, ApplyReq r);
  bool exact_ok() const { return rv_ && rv_->exact_ok(); }
  bool steps_ok() const { return rv_ && rv_->steps_ok(); }
  // A fit resumed from a batched K-apply finds the launch complete (open
  // mode); otherwise only enqueued ahead of its stream's later work.
  bool complete_on_resume() const { return rv_ && rv_->open(); }

 private:
  enum State { kRun, kRead, kApply, kFlight, kDone };
  struct Slot {
    std::coroutine_handle<> h;
    State state = kRun;
    hipEvent_t ev = nullptr;
    hipStream_t st = nullptr;
    ApplyReq req;
  };
  void run_handles(const std::vector<std::coroutine_handle<>>& tops);
  void run_open(const std::vector<std::coroutine_handle<>>& tops);
  void hand_over();
  Rendezvous* rv_;
  std::vector<int> ids_;
  std::vector<Slot> slots_;
};

// co_await read_back(ex, dev, bytes, out): copies `bytes` from device memory
// into out (host).
struct ReadBack {
  Exec& ex;
  const void* dev;
  size_t bytes;
  void* out;
  bool await_ready() {
    if (bytes > kReadBackBytes) fail(KQR_EHIP, "internal: read-back of %zu bytes", bytes);
    KQR_CHECK_HIP(hipMemcpyAsync(ex.hbuf.ptr, dev, bytes, hipMemcpyDeviceToHost, ex.st));
    if (!ex.sched) {
      KQR_CHECK_HIP(hipStreamSynchronize(ex.st));
      return true;
    }
    KQR_CHECK_HIP(hipEventRecord(ex.ev, ex.st));
    return false;
  }
  void await_suspend(std::coroutine_handle<> h) { ex.sched->park_read(ex.slot, h, ex.ev); }
  void await_resume() { memcpy(out, ex.hbuf.ptr, bytes); }
};
inline ReadBack read_back(Exec& ex, const void* dev, size_t bytes, void* out) { return ReadBack{ex, dev, bytes, out}; }

// co_await fence(ex): resumes once everything enqueued on ex's stream has run.
struct Fence {
  Exec& ex;
  bool await_ready() {
    if (!ex.sched) {
      KQR_CHECK_HIP(hipStreamSynchronize(ex.st));
      return true;
    }
    KQR_CHECK_HIP(hipEventRecord(ex.ev, ex.st));
    return false;
  }
  void await_suspend(std::coroutine_handle<> h) { ex.sched->park_read(ex.slot, h, ex.ev); }
  void await_resume() const noexcept {}
};
inline Fence fence(Exec& ex) { return Fence{ex}; }

// co_await of a K-apply: suspends only when the request went to a batch.
struct ApplyAwait {
  Exec* ex = nullptr;  // non-null: request pending in ex->sched
  ApplyReq req;
  bool await_ready() const noexcept { return ex == nullptr; }
  void await_suspend(std::coroutine_handle<> h) const;
  void await_resume() const noexcept {}
};

// Runs a coroutine whose Exec has no scheduler (it never suspends).
template <typename T>
T run_sync(Co<T> c) {
  c.get().resume();
  if (!c.done()) fail(KQR_EHIP, "internal: a synchronous fit suspended");
  return c.result();
}

}  // namespace kqr
