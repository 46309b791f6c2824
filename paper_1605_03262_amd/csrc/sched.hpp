// Scheduler core of the continuous-batching server (host C++, no HIP).
//
// Requests (a mechanism key, n states, a Newton mode and gamma, and an opaque
// payload owned by the executor) arrive from any thread.  A scheduler thread
// forms rounds in arrival order: the head request fixes the round's mode and
// gamma, and later requests with the same mode and gamma join while each
// mechanism's share fits the executor's per-round capacity and the round stays
// within max_round_states.  A round runs on a free executor slot (a stream
// with its own resident pools); several rounds are in flight at once.  A
// completion thread polls in-flight rounds, lets the executor deliver their
// results (without holding the lock), marks the requests done and records
// their latencies.  The device side is the Executor: HIP streams, pools,
// graphs and kernels in serve.hip, a fake one in the CPU tests.
//
// Lifetime rules that keep the two threads apart: a round enters `inflight`
// only after the executor accepted it, and only the completion thread removes
// it; shutdown first drains every pending request, then every round.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace pyjac {
namespace sched {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0;
  int mech = 0;            // executor's mechanism key
  int64_t n = 0;
  int mode = 0;
  double gamma = 0.0;
  void* payload = nullptr; // executor-owned (staging, caller arrays)
  Clock::time_point t_submit, t_done;
  bool done = false;
  int status = 0;          // 0 ok, else the executor's error code
};

struct Round {
  int slot = -1;
  int mode = 0;
  double gamma = 0.0;
  std::vector<std::shared_ptr<Request>> reqs;   // grouped by mechanism in arrival order
  bool failed = false;
};

class Executor {
 public:
  virtual ~Executor() = default;
  virtual int n_slots() const = 0;
  // states of mechanism `mech` one round may hold
  virtual int64_t capacity(int mech) const = 0;
  // enqueue the round on its slot; 0 when accepted, else an error code (the
  // round then completes at once with that status)
  virtual int launch(Round& r) = 0;
  // true once the round's device work has finished (any thread, no lock held)
  virtual bool poll(Round& r) = 0;
  // deliver the round's results to the callers (no lock held)
  virtual void finish(Round& r) = 0;
};

struct Stats {
  int64_t requests_done = 0, states_done = 0, rounds_done = 0;
  std::vector<double> latencies;
};

class Scheduler {
 public:
  Scheduler(Executor* ex, int64_t max_round_states) : ex_(ex), max_round_(max_round_states) {
    busy_.assign(ex_->n_slots(), 0);
    sched_ = std::thread([this] { schedule_loop(); });
    reap_ = std::thread([this] { reap_loop(); });
  }
  ~Scheduler() { shutdown(); }

  // Queues a request; returns its id, or 0 after shutdown began.
  uint64_t submit(std::shared_ptr<Request> r) {
    {
      std::lock_guard<std::mutex> g(mu_);
      if (stop_) return 0;
      r->id = next_id_++;
      r->t_submit = Clock::now();
      pending_.push_back(r);
      all_[r->id] = r;
    }
    cv_sched_.notify_all();
    return r->id;
  }

  // Waits for a request (timeout_s < 0: no limit).  Returns 1 done (then the
  // request is forgotten and *out holds it), 0 on timeout, -1 unknown id.
  int wait(uint64_t id, double timeout_s, std::shared_ptr<Request>* out) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = all_.find(id);
    if (it == all_.end()) return -1;
    auto r = it->second;
    auto pred = [&] { return r->done; };
    if (timeout_s < 0) cv_done_.wait(lk, pred);
    else if (!cv_done_.wait_until(lk, deadline(timeout_s), pred)) return 0;
    all_.erase(id);
    if (out) *out = r;
    return 1;
  }

  Stats stats() {
    std::lock_guard<std::mutex> g(mu_);
    return stats_;
  }

  // Finishes every submitted request, then stops both threads.
  void shutdown() {
    {
      std::lock_guard<std::mutex> g(mu_);
      if (stopped_) return;
      stop_ = true;
    }
    cv_sched_.notify_all();
    cv_done_.notify_all();
    if (sched_.joinable()) sched_.join();
    if (reap_.joinable()) reap_.join();
    std::lock_guard<std::mutex> g(mu_);
    stopped_ = true;
  }

 private:
  // Timed waits use the system clock: its pthread_cond_timedwait is the form
  // that thread checkers follow (a steady-clock wait maps to a newer call some
  // do not intercept).
  static std::chrono::system_clock::time_point deadline(double seconds) {
    return std::chrono::system_clock::now() +
           std::chrono::duration_cast<std::chrono::system_clock::duration>(std::chrono::duration<double>(seconds));
  }

  // Forms the next round from the pending queue (lock held).  Requests larger
  // than a round still run alone.
  std::unique_ptr<Round> form_round(int slot) {
    auto R = std::make_unique<Round>();
    const auto& head = pending_.front();
    R->slot = slot;
    R->mode = head->mode;
    R->gamma = head->gamma;
    std::map<int, int64_t> used;
    int64_t total = 0;
    std::vector<size_t> pick;
    for (size_t q = 0; q < pending_.size(); ++q) {
      const auto& r = pending_[q];
      if (r->mode != R->mode || r->gamma != R->gamma) continue;
      const int64_t cap = ex_->capacity(r->mech);
      if (!pick.empty() && (used[r->mech] + r->n > cap || total + r->n > max_round_)) continue;
      used[r->mech] += r->n;
      total += r->n;
      pick.push_back(q);
      if (total >= max_round_) break;
    }
    // group by mechanism, arrival order within a mechanism
    std::vector<std::shared_ptr<Request>> chosen;
    for (size_t q : pick) chosen.push_back(pending_[q]);
    std::stable_sort(chosen.begin(), chosen.end(),
                     [](const std::shared_ptr<Request>& a, const std::shared_ptr<Request>& b) { return a->mech < b->mech; });
    R->reqs = std::move(chosen);
    for (auto it = pick.rbegin(); it != pick.rend(); ++it) pending_.erase(pending_.begin() + *it);
    return R;
  }

  void schedule_loop() {
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      // wake for a pending request once a slot is free, or to exit once a
      // stop was requested and nothing is pending (pending requests keep the
      // loop alive after a stop; it still waits, releasing the lock)
      cv_sched_.wait(lk, [&] {
        if (pending_.empty()) return stop_;
        return std::find(busy_.begin(), busy_.end(), 0) != busy_.end();
      });
      if (pending_.empty()) break;
      const int slot = (int)(std::find(busy_.begin(), busy_.end(), 0) - busy_.begin());
      auto R = form_round(slot);
      busy_[slot] = 1;
      Round* raw = R.get();
      lk.unlock();
      const int rc = ex_->launch(*raw);
      lk.lock();
      if (rc != 0) {
        raw->failed = true;
        for (auto& r : raw->reqs) r->status = rc;
      }
      inflight_.push_back(std::move(R));       // visible to the completion thread only now
      cv_done_.notify_all();
    }
    cv_done_.notify_all();
  }

  void reap_loop() {
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      if (inflight_.empty()) {
        if (stop_ && pending_.empty() && sched_exited()) break;
        cv_done_.wait_until(lk, deadline(0.002));
        continue;
      }
      // only this thread removes rounds, so the pointers stay valid while the
      // scheduler appends new ones
      std::vector<Round*> snap;
      for (auto& r : inflight_) snap.push_back(r.get());
      lk.unlock();
      std::vector<Round*> fin;
      for (Round* r : snap)
        if (r->failed || ex_->poll(*r)) fin.push_back(r);
      for (Round* r : fin)
        if (!r->failed) ex_->finish(*r);
      lk.lock();
      const auto now = Clock::now();
      for (Round* R : fin) {
        for (auto& r : R->reqs) {
          r->t_done = now;
          r->done = true;
          stats_.latencies.push_back(std::chrono::duration<double>(r->t_done - r->t_submit).count());
          stats_.requests_done += 1;
          stats_.states_done += r->n;
        }
        stats_.rounds_done += 1;
        busy_[R->slot] = 0;
        for (auto it = inflight_.begin(); it != inflight_.end(); ++it)
          if (it->get() == R) { inflight_.erase(it); break; }
      }
      if (!fin.empty()) {
        cv_sched_.notify_all();
        cv_done_.notify_all();
      } else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        lk.lock();
      }
    }
  }

  // the scheduler thread has left its loop once a stop is set and nothing is
  // pending or being launched (every slot free or its round registered)
  bool sched_exited() const {
    for (int b : busy_)
      if (b) return false;
    return true;
  }

  Executor* ex_;
  int64_t max_round_;
  std::mutex mu_;
  std::condition_variable cv_sched_, cv_done_;
  std::deque<std::shared_ptr<Request>> pending_;
  std::map<uint64_t, std::shared_ptr<Request>> all_;
  std::deque<std::unique_ptr<Round>> inflight_;
  std::vector<int> busy_;
  Stats stats_;
  uint64_t next_id_ = 1;
  bool stop_ = false, stopped_ = false;
  std::thread sched_, reap_;
};

}  // namespace sched
}  // namespace pyjac
