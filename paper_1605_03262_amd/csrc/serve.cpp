// Continuous-batching server for Jacobian + Newton requests (host C++ side of
// libpyjac_mi355x).
//
// Requests (a mechanism, n states, step sizes and right-hand sides in host
// memory) arrive at any time.  A scheduler thread admits them in arrival order
// as device memory frees up: every request's device footprint is reserved from
// a fixed arena whose size is the server's HBM budget, so a request that does
// not fit waits (backpressure) and one larger than the budget is rejected at
// submission.  Admitted requests of the same mechanism are packed side by side
// into one batch (states are independent, so a state's result is the same in
// any batch), copied in, evaluated with pyjac_eval_jacobian and
// pyjac_newton_factor_solve on one of several streams, and copied out; a
// completion thread releases the batch's memory when its stream reaches the
// end and records each request's latency (completion - submission).
// Batches on different streams run concurrently on the device, and new
// requests are admitted while earlier batches are still running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pyjac.h"

namespace pyjac {
pyjac_status fail(pyjac_status code, const std::string& msg);
int mech_device(const pyjac_mech* m);
int mech_species(const pyjac_mech* m);
}  // namespace pyjac

namespace {

using Clock = std::chrono::steady_clock;

// First-fit sub-allocator over one device allocation or one pinned host
// allocation (256-byte granules).
class Arena {
 public:
  bool init(size_t bytes, bool pinned_host = false) {
    size_ = (bytes + 255) & ~size_t(255);
    host_ = pinned_host;
    const hipError_t e = host_ ? hipHostMalloc(&base_, size_, hipHostMallocDefault) : hipMalloc(&base_, size_);
    if (e != hipSuccess) {
      base_ = nullptr;
      return false;
    }
    free_[0] = size_;
    return true;
  }
  ~Arena() {
    if (base_) (host_ ? hipHostFree(base_) : hipFree(base_));
  }
  // returns offset or SIZE_MAX
  size_t take(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_ += bytes;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void give(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
    }
  }
  char* ptr(size_t off) const { return static_cast<char*>(base_) + off; }
  size_t size() const { return size_; }
  size_t used() const { return used_; }

 private:
  void* base_ = nullptr;
  bool host_ = false;
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t id = 0;
  const pyjac_mech* mech = nullptr;
  int64_t n = 0;
  int N = 0;
  const double *phi = nullptr, *p = nullptr, *h = nullptr, *rhs = nullptr;
  double gamma = 0;
  int mode = 1;
  double* x = nullptr;
  int32_t* info = nullptr;
  size_t bytes = 0;
  // pinned staging slot: phi [N][n], p [n], h [n], rhs [N][n] in, x [N][n],
  // info [n] out; the caller's arrays are only touched by submit (inputs)
  // and by the completion thread (outputs)
  size_t pin_off = 0, pin_bytes = 0;
  char* pin = nullptr;
  Clock::time_point t_submit, t_done;
  bool done = false;
  pyjac_status status = PYJAC_OK;
};

struct Batch {
  std::vector<std::shared_ptr<Request>> reqs;
  const pyjac_mech* mech = nullptr;
  int64_t n = 0;
  int N = 0;
  size_t off = 0, bytes = 0;
  int stream = 0;
  hipEvent_t done_ev = nullptr;
  bool launched = false;   // set under the lock once done_ev has been recorded
};

struct PinLayout {
  size_t phi, p, h, rhs, x, info, total;
};
PinLayout pin_layout(int N, int64_t n) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  PinLayout L;
  size_t o = 0;
  L.phi = o; o += al((size_t)N * n * 8);
  L.p = o; o += al((size_t)n * 8);
  L.h = o; o += al((size_t)n * 8);
  L.rhs = o; o += al((size_t)N * n * 8);
  L.x = o; o += al((size_t)N * n * 8);
  L.info = o; o += al((size_t)n * 4);
  L.total = o;
  return L;
}

size_t request_bytes(int N, int64_t n, int mode) {
  (void)mode;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  size_t b = 0;
  b += al((size_t)N * n * 8);               // phi
  b += al((size_t)n * 8) * 2;               // p, h
  b += al((size_t)N * n * 8) * 2;           // rhs, x
  b += al((size_t)n * 4);                   // info
  b += al((size_t)N * N * n * 8);           // jac
  return b;
}

}  // namespace

struct pyjac_server {
  int device = 0;
  int n_streams = 2;
  int64_t max_batch = 4096;
  int max_refine = 4;
  double rtol = 1e-14;
  Arena arena;                 // device memory of admitted batches
  Arena pinned;                // host staging of submitted requests
  std::vector<hipStream_t> streams;
  std::vector<int> stream_busy;

  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_pin;
  std::deque<std::shared_ptr<Request>> pending;
  std::map<uint64_t, std::shared_ptr<Request>> all;
  std::deque<std::unique_ptr<Batch>> inflight;
  std::vector<double> latencies;
  uint64_t next_id = 1;
  int64_t states_done = 0, batches_done = 0, requests_done = 0;
  bool stop = false;
  std::string error;
  std::thread sched, reaper;
};

namespace {

size_t batch_bytes(const pyjac_mech* m, int N, int64_t n, int mode) {
  return request_bytes(N, n, mode) + ((pyjac_newton_workspace_bytes(m, n, mode) + 255) & ~size_t(255));
}

// Launch one batch on its stream (called with the lock released).
pyjac_status launch_batch(pyjac_server* S, Batch& B) {
  hipStream_t st = S->streams[B.stream];
  const int N = B.N;
  const int64_t n = B.n;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* base = S->arena.ptr(B.off);
  size_t o = 0;
  double* phi = reinterpret_cast<double*>(base + o); o += al((size_t)N * n * 8);
  double* p = reinterpret_cast<double*>(base + o); o += al((size_t)n * 8);
  double* h = reinterpret_cast<double*>(base + o); o += al((size_t)n * 8);
  double* rhs = reinterpret_cast<double*>(base + o); o += al((size_t)N * n * 8);
  double* x = reinterpret_cast<double*>(base + o); o += al((size_t)N * n * 8);
  int32_t* info = reinterpret_cast<int32_t*>(base + o); o += al((size_t)n * 4);
  double* jac = reinterpret_cast<double*>(base + o); o += al((size_t)N * N * n * 8);
  void* ws = base + o;
  const int mode = B.reqs.front()->mode;
  const double gamma = B.reqs.front()->gamma;
  const size_t wsb = pyjac_newton_workspace_bytes(B.mech, n, mode);
  int64_t col = 0;
  for (auto& r : B.reqs) {
    const size_t w = (size_t)r->n * 8;
    const PinLayout P = pin_layout(N, r->n);
    if (hipMemcpy2DAsync(phi + col, n * 8, r->pin + P.phi, w, w, N, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(p + col, r->pin + P.p, w, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h + col, r->pin + P.h, w, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpy2DAsync(rhs + col, n * 8, r->pin + P.rhs, w, w, N, hipMemcpyHostToDevice, st) != hipSuccess)
      return pyjac::fail(PYJAC_E_DEVICE, "request copy-in failed");
    col += r->n;
  }
  pyjac_status rc = pyjac_eval_jacobian(B.mech, n, n, phi, p, jac, st);
  if (rc == PYJAC_OK)
    rc = pyjac_newton_factor_solve(B.mech, n, n, jac, h, gamma, rhs, x, mode, S->max_refine, S->rtol, info, ws,
                                   wsb, st);
  if (rc != PYJAC_OK) return rc;
  col = 0;
  for (auto& r : B.reqs) {
    const size_t w = (size_t)r->n * 8;
    const PinLayout P = pin_layout(N, r->n);
    if (hipMemcpy2DAsync(r->pin + P.x, w, x + col, n * 8, w, N, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(r->pin + P.info, info + col, (size_t)r->n * 4, hipMemcpyDeviceToHost, st) != hipSuccess)
      return pyjac::fail(PYJAC_E_DEVICE, "request copy-out failed");
    col += r->n;
  }
  if (hipEventRecord(B.done_ev, st) != hipSuccess) return pyjac::fail(PYJAC_E_DEVICE, "event record failed");
  return PYJAC_OK;
}

void scheduler_loop(pyjac_server* S) {
  hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    // Wake for a pending request once a stream is free, or to exit once a
    // stop has been requested and nothing is pending.  Pending requests keep
    // the loop alive after a stop; it then still waits (releasing the lock)
    // until the completion thread frees a stream.
    S->cv_sched.wait(lk, [&] {
      if (S->pending.empty()) return S->stop;
      for (int b : S->stream_busy) if (!b) return true;
      return false;
    });
    if (S->pending.empty()) break;
    int sidx = -1;
    for (int i = 0; i < S->n_streams; ++i) if (!S->stream_busy[i]) { sidx = i; break; }
    // Form a batch: the head request's mechanism and mode, then later requests
    // with the same mechanism/mode, in arrival order, while the packed batch
    // stays within max_batch states and fits the free arena.
    auto head = S->pending.front();
    auto B = std::make_unique<Batch>();
    B->mech = head->mech;
    B->N = head->N;
    int64_t n = 0;
    std::vector<size_t> pick;
    for (size_t q = 0; q < S->pending.size(); ++q) {
      auto& r = S->pending[q];
      if (r->mech != head->mech || r->mode != head->mode || r->gamma != head->gamma) continue;
      if (n > 0 && n + r->n > S->max_batch) break;
      n += r->n;
      pick.push_back(q);
    }
    size_t need = batch_bytes(B->mech, B->N, n, head->mode);
    size_t off = S->arena.take(need);
    while (off == SIZE_MAX && pick.size() > 1) {   // shrink to what fits
      n -= S->pending[pick.back()]->n;
      pick.pop_back();
      need = batch_bytes(B->mech, B->N, n, head->mode);
      off = S->arena.take(need);
    }
    if (off == SIZE_MAX) {                          // head waits for memory (backpressure)
      S->cv_sched.wait_for(lk, std::chrono::milliseconds(2));
      continue;
    }
    for (auto it = pick.rbegin(); it != pick.rend(); ++it) {
      B->reqs.insert(B->reqs.begin(), S->pending[*it]);
      S->pending.erase(S->pending.begin() + *it);
    }
    B->n = n;
    B->off = off;
    B->bytes = need;
    B->stream = sidx;
    S->stream_busy[sidx] = 1;
    hipEventCreateWithFlags(&B->done_ev, hipEventDisableTiming);
    Batch* raw = B.get();
    S->inflight.push_back(std::move(B));
    lk.unlock();
    pyjac_status rc = launch_batch(S, *raw);
    if (rc != PYJAC_OK) {
      hipStreamSynchronize(S->streams[raw->stream]);
      hipEventRecord(raw->done_ev, S->streams[raw->stream]);
    }
    lk.lock();
    if (rc != PYJAC_OK) {
      S->error = pyjac_last_error();
      for (auto& r : raw->reqs) r->status = rc;
    }
    // Only now may the completion thread look at the batch: an event that was
    // never recorded reads as complete.
    raw->launched = true;
    S->cv_done.notify_all();
  }
}

void reaper_loop(pyjac_server* S) {
  hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    if (S->inflight.empty()) {
      if (S->stop && S->pending.empty()) break;
      S->cv_done.wait_for(lk, std::chrono::milliseconds(5));
      continue;
    }
    // Snapshot the launched batches under the lock and query their events
    // without it.  Only this thread erases from `inflight`, so the pointers
    // stay valid while the scheduler appends new batches.
    std::vector<Batch*> snap;
    for (auto& b : S->inflight)
      if (b->launched) snap.push_back(b.get());
    std::vector<hipError_t> st(snap.size());
    lk.unlock();
    for (size_t q = 0; q < snap.size(); ++q) st[q] = hipEventQuery(snap[q]->done_ev);
    lk.lock();
    // results of the finished batches go from the pinned slots to the
    // callers' arrays without the lock (the requests are not done yet, so
    // nobody else touches those slots)
    lk.unlock();
    for (size_t q = 0; q < snap.size(); ++q) {
      if (st[q] != hipSuccess) continue;
      for (auto& r : snap[q]->reqs) {
        const PinLayout P = pin_layout(r->N, r->n);
        std::memcpy(r->x, r->pin + P.x, (size_t)r->N * r->n * 8);
        std::memcpy(r->info, r->pin + P.info, (size_t)r->n * 4);
      }
    }
    lk.lock();
    bool any = false;
    for (size_t q = 0; q < snap.size(); ++q) {
      if (st[q] == hipErrorNotReady) continue;
      Batch* B = snap[q];
      const hipError_t qs = st[q];
      const auto now = Clock::now();
      for (auto& r : B->reqs) {
        S->pinned.give(r->pin_off, r->pin_bytes);
        r->pin = nullptr;
        r->t_done = now;
        r->done = true;
        if (qs != hipSuccess && r->status == PYJAC_OK) r->status = PYJAC_E_DEVICE;
        S->latencies.push_back(std::chrono::duration<double>(r->t_done - r->t_submit).count());
        S->requests_done += 1;
      }
      S->states_done += B->n;
      S->batches_done += 1;
      S->arena.give(B->off, B->bytes);
      S->stream_busy[B->stream] = 0;
      hipEventDestroy(B->done_ev);
      for (auto it = S->inflight.begin(); it != S->inflight.end(); ++it)
        if (it->get() == B) { S->inflight.erase(it); break; }
      any = true;
    }
    if (any) {
      S->cv_sched.notify_all();
      S->cv_done.notify_all();
      S->cv_pin.notify_all();
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      lk.lock();
    }
  }
}

}  // namespace

extern "C" {

pyjac_status pyjac_serve_create(int32_t device, size_t hbm_budget_bytes, int64_t max_batch_states,
                                int32_t n_streams, int32_t max_refine, double rtol, pyjac_server** out) {
  if (!out) return pyjac::fail(PYJAC_E_INVALID, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes < (1u << 20) || max_batch_states < 1 || n_streams < 1 || n_streams > 16 || max_refine < 1 ||
      !(rtol > 0))
    return pyjac::fail(PYJAC_E_INVALID, "bad server parameters");
  auto S = std::make_unique<pyjac_server>();
  S->device = device;
  S->n_streams = n_streams;
  S->max_batch = max_batch_states;
  S->max_refine = max_refine;
  S->rtol = rtol;
  int prev = 0;
  hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) return pyjac::fail(PYJAC_E_DEVICE, "no such device");
  if (!S->arena.init(hbm_budget_bytes)) {
    hipSetDevice(prev);
    return pyjac::fail(PYJAC_E_NOMEM, "cannot reserve the HBM budget");
  }
  const size_t pin_bytes = std::max<size_t>(64u << 20, std::min<size_t>(hbm_budget_bytes / 4, size_t(2) << 30));
  if (!S->pinned.init(pin_bytes, true)) {
    hipSetDevice(prev);
    return pyjac::fail(PYJAC_E_NOMEM, "cannot allocate pinned host staging memory");
  }
  for (int i = 0; i < n_streams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      hipSetDevice(prev);
      return pyjac::fail(PYJAC_E_DEVICE, "stream creation failed");
    }
    S->streams.push_back(st);
  }
  S->stream_busy.assign(n_streams, 0);
  hipSetDevice(prev);
  pyjac_server* raw = S.release();
  raw->sched = std::thread(scheduler_loop, raw);
  raw->reaper = std::thread(reaper_loop, raw);
  *out = raw;
  return PYJAC_OK;
}

pyjac_status pyjac_serve_submit(pyjac_server* S, const pyjac_mech* mech, int64_t n_states, const double* phi,
                                const double* p, const double* h, const double* rhs, double gamma, int32_t mode,
                                double* x, int32_t* info, uint64_t* request_id) {
  if (!S || !mech || !request_id) return pyjac::fail(PYJAC_E_INVALID, "NULL argument");
  if (n_states < 1) return pyjac::fail(PYJAC_E_INVALID, "n_states must be >= 1");
  if (!phi || !p || !h || !rhs || !x || !info) return pyjac::fail(PYJAC_E_INVALID, "NULL array");
  if (mode != 0 && mode != 1) return pyjac::fail(PYJAC_E_INVALID, "mode must be 0 or 1");
  if (pyjac::mech_device(mech) != S->device) return pyjac::fail(PYJAC_E_INVALID, "mechanism on another device");
  auto r = std::make_shared<Request>();
  r->mech = mech;
  r->n = n_states;
  r->N = pyjac::mech_species(mech);
  r->phi = phi; r->p = p; r->h = h; r->rhs = rhs;
  r->gamma = gamma;
  r->mode = mode;
  r->x = x;
  r->info = info;
  r->bytes = batch_bytes(mech, r->N, n_states, mode);
  if (r->bytes > S->arena.size()) return pyjac::fail(PYJAC_E_NOMEM, "request larger than the server's HBM budget");
  if (n_states > S->max_batch) return pyjac::fail(PYJAC_E_INVALID, "request larger than max_batch_states");
  const PinLayout P = pin_layout(r->N, n_states);
  r->pin_bytes = P.total;
  if (P.total > S->pinned.size()) return pyjac::fail(PYJAC_E_NOMEM, "request larger than the pinned staging memory");
  const auto t0 = Clock::now();
  std::unique_lock<std::mutex> lk(S->mu);
  // backpressure on the submitting thread while the staging memory is full
  size_t off = SIZE_MAX;
  while (!S->stop && (off = S->pinned.take(P.total)) == SIZE_MAX) S->cv_pin.wait(lk);
  if (S->stop) {
    if (off != SIZE_MAX) S->pinned.give(off, P.total);
    return pyjac::fail(PYJAC_E_INVALID, "server is shutting down");
  }
  r->pin_off = off;
  r->pin = S->pinned.ptr(off);
  lk.unlock();
  const size_t w = (size_t)n_states * 8;
  std::memcpy(r->pin + P.phi, phi, (size_t)r->N * w);
  std::memcpy(r->pin + P.p, p, w);
  std::memcpy(r->pin + P.h, h, w);
  std::memcpy(r->pin + P.rhs, rhs, (size_t)r->N * w);
  lk.lock();
  r->id = S->next_id++;
  r->t_submit = t0;
  S->pending.push_back(r);
  S->all[r->id] = r;
  *request_id = r->id;
  lk.unlock();
  S->cv_sched.notify_all();
  return PYJAC_OK;
}

// Waits until the request has completed (timeout_s < 0: no limit).  Returns
// PYJAC_OK with *latency_s set, the request's error, or PYJAC_E_INVALID for an
// unknown id / timeout.  A completed request is forgotten after this call.
pyjac_status pyjac_serve_wait(pyjac_server* S, uint64_t request_id, double timeout_s, double* latency_s) {
  if (!S) return pyjac::fail(PYJAC_E_INVALID, "NULL server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(request_id);
  if (it == S->all.end()) return pyjac::fail(PYJAC_E_INVALID, "unknown request id");
  auto r = it->second;
  auto pred = [&] { return r->done; };
  if (timeout_s < 0) S->cv_done.wait(lk, pred);
  else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
    return pyjac::fail(PYJAC_E_INVALID, "timed out");
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  S->all.erase(it);
  if (r->status != PYJAC_OK) return pyjac::fail(r->status, S->error);
  return PYJAC_OK;
}

// Totals since creation; p50/p99 latency over all completed requests.
pyjac_status pyjac_serve_stats(pyjac_server* S, int64_t* requests_done, int64_t* states_done, int64_t* batches_done,
                               double* p50_s, double* p99_s, size_t* hbm_in_use) {
  if (!S) return pyjac::fail(PYJAC_E_INVALID, "NULL server");
  std::lock_guard<std::mutex> g(S->mu);
  if (requests_done) *requests_done = S->requests_done;
  if (states_done) *states_done = S->states_done;
  if (batches_done) *batches_done = S->batches_done;
  std::vector<double> l = S->latencies;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) { return l.empty() ? 0.0 : l[std::min(l.size() - 1, (size_t)(q * (l.size() - 1) + 0.5))]; };
  if (p50_s) *p50_s = pct(0.50);
  if (p99_s) *p99_s = pct(0.99);
  if (hbm_in_use) *hbm_in_use = S->arena.used();
  return PYJAC_OK;
}

// Finishes every submitted request, then releases the streams and the arena.
pyjac_status pyjac_serve_destroy(pyjac_server* S) {
  if (!S) return PYJAC_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_sched.notify_all();
  S->cv_done.notify_all();
  S->cv_pin.notify_all();
  if (S->sched.joinable()) S->sched.join();
  if (S->reaper.joinable()) S->reaper.join();
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(S->device);
  for (auto st : S->streams) { hipStreamSynchronize(st); hipStreamDestroy(st); }
  hipSetDevice(prev);
  delete S;
  return PYJAC_OK;
}

}  // extern "C"
