// Schedulers of batched fits (coro.h): one per host thread, meeting at a
// rendezvous for the batched K-apply launches.
#include "coro.h"
#include "pstep.h"

#include <algorithm>
#include <memory>
#include <thread>

namespace kqr {

Exec::Exec(hipStream_t s, Scheduler* sc, int sl) : st(s), sched(sc), slot(sl) {
  KQR_CHECK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
}

Exec::~Exec() {
  if (ev) (void)hipEventDestroy(ev);
}

void ApplyAwait::await_suspend(std::coroutine_handle<> h) const { ex->sched->park_apply(ex->slot, h, ex->st, req); }

// ================================================================= rendezvous
Rendezvous::Rendezvous(BatchLauncher* launcher, int threads, bool profile, bool open)
    : launcher_(launcher), profile_(profile), open_(open), active_(threads) {
  KQR_CHECK_HIP(hipStreamCreate(&bst_));
  KQR_CHECK_HIP(hipEventCreateWithFlags(&done_, hipEventDisableTiming));
}

Rendezvous::~Rendezvous() {
  (void)hipStreamSynchronize(bst_);
  for (auto& s : spans_) {
    (void)hipEventDestroy(s.first);
    (void)hipEventDestroy(s.second);
  }
  for (auto& e : stream_ev_) (void)hipEventDestroy(e.second);
  (void)hipEventDestroy(done_);
  (void)hipStreamDestroy(bst_);
}

hipEvent_t Rendezvous::stream_event(hipStream_t s) {
  for (auto& e : stream_ev_)
    if (e.first == s) return e.second;
  hipEvent_t e = nullptr;
  KQR_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  stream_ev_.emplace_back(s, e);
  return e;
}

void Rendezvous::arrive(const std::vector<hipStream_t>& streams, const std::vector<int>& ids,
                        const std::vector<ApplyReq>& reqs) {
  std::unique_lock<std::mutex> lk(mu_);
  if (failed_) fail(KQR_EHIP, "batched K-apply failed");
  for (hipStream_t s : streams) {
    // this thread's work on s so far (its fits' vectors) precedes the launch
    KQR_CHECK_HIP(hipEventRecord(stream_event(s), s));
    streams_.push_back(s);
  }
  ids_.insert(ids_.end(), ids.begin(), ids.end());
  reqs_.insert(reqs_.end(), reqs.begin(), reqs.end());
  ++arrived_;
  const uint64_t my_gen = gen_;
  if (arrived_ == active_) {
    fire_locked();
  } else {
    cv_.wait(lk, [&] { return gen_ != my_gen || failed_; });
  }
  if (failed_) fail(KQR_EHIP, "batched K-apply failed");
  // done_ is recorded again only once every thread served by this launch has
  // arrived for the next one, which this thread has not yet
  for (hipStream_t s : streams) KQR_CHECK_HIP(hipStreamWaitEvent(s, done_, 0));
}

void Rendezvous::leave() {
  std::unique_lock<std::mutex> lk(mu_);
  if (open_) return;  // open rounds do not count threads
  --active_;
  if (arrived_ > 0 && arrived_ == active_ && !failed_) {
    try {
      fire_locked();
    } catch (...) {
      failed_ = true;
      cv_.notify_all();
    }
  }
}

// The launch of the pending requests on bst_ (after the requesters' work so
// far), ending with done_.
void Rendezvous::launch_locked() {
  for (hipStream_t s : streams_) KQR_CHECK_HIP(hipStreamWaitEvent(bst_, stream_event(s), 0));
  hipEvent_t a = nullptr, b = nullptr;
  if (profile_) {
    KQR_CHECK_HIP(hipEventCreate(&a));
    KQR_CHECK_HIP(hipEventCreate(&b));
    KQR_CHECK_HIP(hipEventRecord(a, bst_));
  }
  launcher_->launch(ids_, reqs_, bst_);
  if (profile_) {  // the K-apply alone
    KQR_CHECK_HIP(hipEventRecord(b, bst_));
    spans_.emplace_back(a, b);
  }
  launcher_->launch_steps(reqs_, bst_);
  KQR_CHECK_HIP(hipEventRecord(done_, bst_));
}

void Rendezvous::fire_locked() {
  try {
    launch_locked();
  } catch (...) {
    failed_ = true;
    cv_.notify_all();
    throw;
  }
  ids_.clear();
  reqs_.clear();
  streams_.clear();
  arrived_ = 0;
  ++launches_;
  ++gen_;
  cv_.notify_all();
}

void Rendezvous::hand_in(const std::vector<hipStream_t>& streams, const std::vector<Pending>& regs, int resumed) {
  std::unique_lock<std::mutex> lk(mu_);
  inflight_ -= resumed;
  if (failed_) fail(KQR_EHIP, "batched K-apply failed");
  for (hipStream_t s : streams) {
    // the requesters' work on s so far precedes the launch
    KQR_CHECK_HIP(hipEventRecord(stream_event(s), s));
    if (std::find(streams_.begin(), streams_.end(), s) == streams_.end()) streams_.push_back(s);
  }
  for (const Pending& p : regs) {
    ids_.push_back(p.id);
    reqs_.push_back(p.req);
    served_.push_back(p.served);
  }
  if (inflight_ > 0 || reqs_.empty()) return;
  try {
    launch_locked();
  } catch (...) {
    failed_ = true;
    throw;
  }
  for (std::atomic<int>* f : served_) f->store(1, std::memory_order_release);
  inflight_ = int(reqs_.size());
  ids_.clear();
  reqs_.clear();
  streams_.clear();
  served_.clear();
  ++launches_;
}

void Rendezvous::abort() {
  std::unique_lock<std::mutex> lk(mu_);
  failed_ = true;
}

void Rendezvous::check_failed() {
  std::unique_lock<std::mutex> lk(mu_);
  if (failed_) fail(KQR_EHIP, "batched K-apply failed");
}

double Rendezvous::device_seconds() {
  double t = 0.0;
  for (auto& s : spans_) {
    KQR_CHECK_HIP(hipEventSynchronize(s.second));
    float ms = 0.f;
    KQR_CHECK_HIP(hipEventElapsedTime(&ms, s.first, s.second));
    t += 1e-3 * ms;
  }
  return t;
}

// ================================================================= scheduler
Scheduler::Scheduler(Rendezvous* rv, std::vector<int> ids) : rv_(rv), ids_(std::move(ids)) {}

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

void Scheduler::hand_over() {
  std::vector<int> ids;
  std::vector<ApplyReq> reqs;
  std::vector<hipStream_t> streams;
  for (size_t i = 0; i < slots_.size(); ++i) {
    const Slot& s = slots_[i];
    if (s.state != kApply) continue;
    ids.push_back(ids_[i]);
    reqs.push_back(s.req);
    if (std::find(streams.begin(), streams.end(), s.st) == streams.end()) streams.push_back(s.st);
  }
  rv_->arrive(streams, ids, reqs);
  for (auto& s : slots_)
    if (s.state == kApply) s.state = kRun;
}

void Scheduler::run_handles(const std::vector<std::coroutine_handle<>>& tops) {
  if (ids_.size() != tops.size()) fail(KQR_EHIP, "internal: scheduler slots do not match its tasks");
  if (rv_ && rv_->open()) {
    run_open(tops);
    return;
  }
  struct Leave {  // the other threads must not wait for this one after it stops
    Rendezvous* rv;
    ~Leave() {
      if (rv) rv->leave();
    }
  } leave{rv_};
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
      // every live fit waits for a K-apply
      if (!rv_) fail(KQR_EHIP, "internal: K-apply request without a batch launcher");
      hand_over();
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

// Open mode: resume the fits back from a round first, each handing in its
// next request at once, then the fits whose read-backs completed; then poll
// this thread's read-backs, its requests' rounds and their completion until a
// fit can run again.
void Scheduler::run_open(const std::vector<std::coroutine_handle<>>& tops) {
  slots_.assign(tops.size(), Slot{});
  std::unique_ptr<std::atomic<int>[]> served(new std::atomic<int>[tops.size()]);
  std::vector<char> back(tops.size(), 0);  // resumed from a round (not from a read-back)
  size_t live = 0;
  for (size_t i = 0; i < tops.size(); ++i) {
    served[i].store(0);
    slots_[i].h = tops[i];
    slots_[i].state = tops[i] && !tops[i].done() ? kRun : kDone;
    if (slots_[i].state == kRun) ++live;
  }
  // a PCG step's completion tag in the fit's pinned buffer (pstep.h): 0.0
  // until the step's last kernel stores 1.0 there, after the status pair;
  // read as an acquire load of its bits, which orders the fit's later reads
  // of the pair after it
  auto tag = [](const Slot& s) -> const uint64_t* {
    return s.req.step && s.req.step->status ? reinterpret_cast<const uint64_t*>(s.req.step->status + 2) : nullptr;
  };
  try {
    while (live > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        for (size_t i = 0; i < slots_.size(); ++i) {
          Slot& s = slots_[i];
          if (s.state != kRun || (pass == 0) != (back[i] != 0)) continue;
          const int resumed = back[i] ? 1 : 0;
          back[i] = 0;
          s.state = kDone;  // a park below sets the waiting state
          s.h.resume();
          std::vector<Rendezvous::Pending> regs;
          std::vector<hipStream_t> streams;
          if (tops[i].done()) {
            s.state = kDone;
            --live;
          } else if (s.state == kDone) {
            fail(KQR_EHIP, "internal: a fit suspended outside a read-back or K-apply");
          } else if (s.state == kApply) {
            served[i].store(0);
            regs.push_back(Rendezvous::Pending{ids_[i], s.req, &served[i]});
            if (!s.req.clean) streams.push_back(s.st);
          }
          if (resumed || !regs.empty()) rv_->hand_in(streams, regs, resumed);
        }
      }
      if (live == 0) break;
      for (bool any = false; !any;) {
        for (size_t i = 0; i < slots_.size(); ++i) {
          Slot& s = slots_[i];
          if (s.state == kRead) {
            const hipError_t e = hipEventQuery(s.ev);
            if (e == hipSuccess) {
              s.state = kRun;
              any = true;
            } else if (e != hipErrorNotReady) {
              KQR_CHECK_HIP(e);
            }
          } else if (s.state == kApply && served[i].load(std::memory_order_acquire)) {
            s.state = kFlight;
          }
          if (s.state != kFlight) continue;
          const uint64_t* t = tag(s);
          bool complete;
          if (t) {
            complete = __atomic_load_n(t, __ATOMIC_ACQUIRE) != 0;
          } else {
            const hipError_t e = hipEventQuery(rv_->done_event());
            if (e != hipSuccess && e != hipErrorNotReady) KQR_CHECK_HIP(e);
            complete = e == hipSuccess;
          }
          if (complete) {
            std::atomic_thread_fence(std::memory_order_acquire);
            s.state = kRun;
            back[i] = 1;
            any = true;
          }
        }
        if (!any) {
          rv_->check_failed();
          std::this_thread::yield();
        }
      }
    }
  } catch (...) {
    rv_->abort();
    throw;
  }
}

}  // namespace kqr
