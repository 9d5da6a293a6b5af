// The single-thread scheduler of batched fits (coro.h).
#include "coro.h"

#include <algorithm>

namespace kqr {

Exec::Exec(hipStream_t s, Scheduler* sc, int sl) : st(s), sched(sc), slot(sl) {
  KQR_CHECK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
}

Exec::~Exec() {
  if (ev) (void)hipEventDestroy(ev);
}

void ApplyAwait::await_suspend(std::coroutine_handle<> h) const { ex->sched->park_apply(ex->slot, h, ex->st, req); }

Scheduler::Scheduler(BatchLauncher* launcher, bool profile) : launcher_(launcher), profile_(profile) {
  if (launcher_) {
    KQR_CHECK_HIP(hipStreamCreate(&bst_));
    KQR_CHECK_HIP(hipEventCreateWithFlags(&done_, hipEventDisableTiming));
  }
}

Scheduler::~Scheduler() {
  if (bst_) (void)hipStreamSynchronize(bst_);
  for (auto& s : spans_) {
    (void)hipEventDestroy(s.first);
    (void)hipEventDestroy(s.second);
  }
  for (auto& e : stream_ev_) (void)hipEventDestroy(e);
  if (done_) (void)hipEventDestroy(done_);
  if (bst_) (void)hipStreamDestroy(bst_);
}

void Scheduler::park_read(int slot, std::coroutine_handle<> h, hipEvent_t ev) {
  Slot& s = slots_[size_t(slot)];
  s.h = h;
  s.ev = ev;
  s.state = kRead;
}

void Scheduler::park_apply(int slot, std::coroutine_handle<> h, hipStream_t st, ApplyReq r) {
  Slot& s = slots_[size_t(slot)];
  s.h = h;
  s.st = st;
  s.req = r;
  s.state = kApply;
}

double Scheduler::device_seconds() {
  double t = 0.0;
  for (auto& s : spans_) {
    KQR_CHECK_HIP(hipEventSynchronize(s.second));
    float ms = 0.f;
    KQR_CHECK_HIP(hipEventElapsedTime(&ms, s.first, s.second));
    t += 1e-3 * ms;
  }
  return t;
}

void Scheduler::fire() {
  std::vector<int> sl;
  std::vector<ApplyReq> rq;
  std::vector<hipStream_t> streams;  // distinct requester streams
  for (size_t i = 0; i < slots_.size(); ++i) {
    const Slot& s = slots_[i];
    if (s.state != kApply) continue;
    sl.push_back(int(i));
    rq.push_back(s.req);
    if (std::find(streams.begin(), streams.end(), s.st) == streams.end()) streams.push_back(s.st);
  }
  while (stream_ev_.size() < streams.size()) {
    hipEvent_t e = nullptr;
    KQR_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    stream_ev_.push_back(e);
  }
  // the batch reads every requester's vector: wait for the work enqueued on their streams
  for (size_t k = 0; k < streams.size(); ++k) {
    KQR_CHECK_HIP(hipEventRecord(stream_ev_[k], streams[k]));
    KQR_CHECK_HIP(hipStreamWaitEvent(bst_, stream_ev_[k], 0));
  }
  hipEvent_t a = nullptr, b = nullptr;
  if (profile_) {
    KQR_CHECK_HIP(hipEventCreate(&a));
    KQR_CHECK_HIP(hipEventCreate(&b));
    KQR_CHECK_HIP(hipEventRecord(a, bst_));
  }
  launcher_->launch(sl, rq, bst_);
  if (profile_) {
    KQR_CHECK_HIP(hipEventRecord(b, bst_));
    spans_.emplace_back(a, b);
  }
  KQR_CHECK_HIP(hipEventRecord(done_, bst_));
  for (hipStream_t st : streams) KQR_CHECK_HIP(hipStreamWaitEvent(st, done_, 0));
  for (int i : sl) slots_[size_t(i)].state = kRun;
  ++launches_;
}

void Scheduler::run_handles(const std::vector<std::coroutine_handle<>>& tops) {
  slots_.assign(tops.size(), Slot{});
  size_t live = 0;
  for (size_t i = 0; i < tops.size(); ++i) {
    slots_[i].h = tops[i];
    slots_[i].state = tops[i] && !tops[i].done() ? kRun : kDone;
    if (slots_[i].state == kRun) ++live;
  }
  while (live > 0) {
    // run every runnable fit up to its next read-back or K-apply request
    for (size_t i = 0; i < slots_.size(); ++i) {
      Slot& s = slots_[i];
      if (s.state != kRun) continue;
      s.state = kDone;  // a park below sets the waiting state
      s.h.resume();
      if (tops[i].done()) {
        s.state = kDone;
        --live;
      } else if (s.state == kDone) {
        fail(KQR_EHIP, "internal: a fit suspended outside a read-back or K-apply");
      }
    }
    if (live == 0) break;
    bool reading = false, progressed = false;
    for (auto& s : slots_) {
      if (s.state != kRead) continue;
      reading = true;
      const hipError_t e = hipEventQuery(s.ev);
      if (e == hipSuccess) {
        s.state = kRun;
        progressed = true;
      } else if (e != hipErrorNotReady) {
        KQR_CHECK_HIP(e);
      }
    }
    if (!reading) {
      // every live fit waits for a K-apply: one launch serves them all
      if (!launcher_) fail(KQR_EHIP, "internal: K-apply request without a batch launcher");
      fire();
      continue;
    }
    if (!progressed) {
      for (auto& s : slots_)
        if (s.state == kRead) {
          KQR_CHECK_HIP(hipEventSynchronize(s.ev));
          s.state = kRun;
          break;
        }
    }
  }
}

}  // namespace kqr
