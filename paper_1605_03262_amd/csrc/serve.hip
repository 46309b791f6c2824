// Continuous-batching server for Jacobian + Newton requests (host C++ side of
// libpyjac_mi355x), on the scheduler core of sched.hpp.
//
// Requests (a mechanism, n states, step sizes and right-hand sides in host
// memory) arrive at any time; submit() copies the inputs into pinned staging
// memory and queues them.  Rounds run on one of n_streams streams, each with
// resident slot pools per mechanism (device arrays for states, Jacobians and
// Newton workspace, sized at the mechanism's first request from the HBM
// budget): a round places its requests side by side in its stream's pools,
// copies the inputs in, evaluates every mechanism's Jacobian in one
// work-list launch per launch shape (pyjac_eval_jacobian_multi), solves each
// mechanism's Newton systems (pyjac_newton_factor_solve), and copies the
// results out.  The pool extent a round computes is its mechanism's state
// count rounded up to 256, so rounds repeat the same kernel sequence; the
// second round with a given sequence (mode, gamma, per-mechanism extents) on a
// stream captures it into a HIP graph and later ones replay it (the first runs
// eagerly, which also sets every kernel attribute outside the capture).
// Padding columns hold valid states from earlier rounds or the initial fill,
// and states are independent, so a request's result is the same in any round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pyjac.h"
#include "sched.hpp"

namespace pyjac {
pyjac_status fail(pyjac_status code, const std::string& msg);
int mech_device(const pyjac_mech* m);
int mech_species(const pyjac_mech* m);
}  // namespace pyjac

namespace {

constexpr int64_t kExtentQuantum = 256;   // a round's per-mechanism extent is a multiple of this

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// First-fit sub-allocator over one pinned host allocation (256-byte granules).
class PinnedArena {
 public:
  bool init(size_t bytes) {
    size_ = al256(bytes);
    if (hipHostMalloc(&base_, size_, hipHostMallocDefault) != hipSuccess) {
      base_ = nullptr;
      return false;
    }
    free_[0] = size_;
    return true;
  }
  ~PinnedArena() {
    if (base_) hipHostFree(base_);
  }
  size_t take(size_t bytes) {
    bytes = al256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void give(size_t off, size_t bytes) {
    bytes = al256(bytes);
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

 private:
  void* base_ = nullptr;
  size_t size_ = 0;
  std::map<size_t, size_t> free_;
};

// Staging layout of one request: phi [N][n], p [n], h [n], rhs [N][n] in,
// x [N][n], info [n] out.
struct PinLayout {
  size_t phi, p, h, rhs, x, info, total;
};
PinLayout pin_layout(int N, int64_t n) {
  PinLayout L;
  size_t o = 0;
  L.phi = o; o += al256((size_t)N * n * 8);
  L.p = o; o += al256((size_t)n * 8);
  L.h = o; o += al256((size_t)n * 8);
  L.rhs = o; o += al256((size_t)N * n * 8);
  L.x = o; o += al256((size_t)N * n * 8);
  L.info = o; o += al256((size_t)n * 4);
  L.total = o;
  return L;
}

struct Payload {
  int N = 0;
  double* x = nullptr;          // caller's output arrays
  int32_t* info = nullptr;
  size_t pin_off = 0, pin_bytes = 0;
  char* pin = nullptr;
  int64_t col = 0;              // first column in the round's pool (set at launch)
};

// Resident device arrays of one mechanism on one stream, capacity C states.
struct Pool {
  int64_t C = 0;
  void* mem = nullptr;
  size_t bytes = 0, wsb = 0;
  double *phi = nullptr, *p = nullptr, *h = nullptr, *rhs = nullptr, *x = nullptr, *jac = nullptr;
  int32_t* info = nullptr;
  void* ws = nullptr;
};

size_t pool_bytes(const pyjac_mech* m, int64_t C) {
  const int N = pyjac::mech_species(m);
  size_t b = 0;
  b += al256((size_t)N * C * 8) * 3;         // phi, rhs, x
  b += al256((size_t)C * 8) * 2;             // p, h
  b += al256((size_t)C * 4);                 // info
  b += al256((size_t)N * N * C * 8);         // jac
  b += al256(std::max(pyjac_newton_workspace_bytes(m, C, 0), pyjac_newton_workspace_bytes(m, C, 1)));
  return b;
}

struct GraphEntry {
  int seen = 0;
  bool no_graph = false;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct pyjac_server : public pyjac::sched::Executor {
  int device = 0;
  int n_streams_ = 1;
  int64_t max_batch = 4096;
  int max_refine = 4;
  double rtol = 1e-14;
  size_t budget = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  hipStream_t setup = nullptr;                         // pool fills, waited for at once
  PinnedArena pinned;
  std::mutex pin_mu;
  std::condition_variable cv_pin;
  bool closing = false;
  // mechanism registry and pools (pools[slot][key]); a slot's pools and graphs
  // are touched only by the round running on it
  mutable std::mutex reg_mu;
  std::vector<const pyjac_mech*> mechs;
  std::vector<int64_t> cap;                            // per key
  std::vector<std::map<int, Pool>> pools;
  std::vector<std::map<std::string, GraphEntry>> graphs;
  size_t pool_total = 0;
  std::atomic<int64_t> n_eager{0}, n_captured{0}, n_replayed{0}, n_jac_launches{0}, n_multi_mech{0};
  std::mutex err_mu;
  std::string error;
  std::unique_ptr<pyjac::sched::Scheduler> sch;

  // ---- Executor
  int n_slots() const override { return n_streams_; }
  int64_t capacity(int key) const override {
    std::lock_guard<std::mutex> g(reg_mu);
    return cap[key];
  }
  int launch(pyjac::sched::Round& R) override;
  bool poll(pyjac::sched::Round& R) override { return hipEventQuery(events[R.slot]) != hipErrorNotReady; }
  void finish(pyjac::sched::Round& R) override;

  void set_error(const std::string& s) {
    std::lock_guard<std::mutex> g(err_mu);
    error = s;
  }
  const pyjac_mech* mech_of(int key) const {
    std::lock_guard<std::mutex> g(reg_mu);
    return mechs[key];
  }
  int compute(pyjac::sched::Round& R, const std::vector<std::pair<int, int64_t>>& extents);
};

namespace {

// Fills a new pool with valid states (T 1500 K, equal mass fractions, 1 atm,
// h = 0 so that A = I, zero right-hand sides), so that padding columns never
// hold garbage.  One thread per element of the N x C state block.
__global__ void fill_pool_kernel(int N, int64_t C, double* __restrict__ phi, double* __restrict__ p,
                                 double* __restrict__ h, double* __restrict__ rhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)N * C) {
    phi[i] = i < C ? 1500.0 : 1.0 / N;
    rhs[i] = 0.0;
  }
  if (i < C) {
    p[i] = 101325.0;
    h[i] = 0.0;
  }
}

// The fill runs on the server's setup stream (not a round's stream, which may
// be capturing a graph on the scheduler thread, and not the null stream), and
// is waited for before the pool is registered.
pyjac_status init_pool(const pyjac_mech* m, Pool& P, hipStream_t setup) {
  const int N = pyjac::mech_species(m);
  const int64_t total = (int64_t)N * P.C;
  const int64_t blocks = (total + 255) / 256;
  fill_pool_kernel<<<dim3((unsigned)blocks), dim3(256), 0, setup>>>(N, P.C, P.phi, P.p, P.h, P.rhs);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(setup);
  if (e != hipSuccess)
    return pyjac::fail(PYJAC_E_DEVICE, std::string("pool initialization failed: ") + hipGetErrorName(e));
  return PYJAC_OK;
}

}  // namespace

int pyjac_server::compute(pyjac::sched::Round& R, const std::vector<std::pair<int, int64_t>>& extents) {
  hipStream_t st = streams[R.slot];
  auto& pl = pools[R.slot];
  // Jacobians: one work-list launch per launch shape over the round's mechanisms
  std::map<std::pair<int, int>, std::vector<pyjac_work_item>> groups;
  for (auto& [key, E] : extents) {
    const pyjac_mech* m = mech_of(key);
    const Pool& P = pl.at(key);
    int32_t ts = 0, nt = 0;
    pyjac_mech_get_variant(m, 1, &ts, &nt, nullptr);
    groups[{ts, nt}].push_back(pyjac_work_item{m, E, P.C, P.phi, P.p, P.jac});
  }
  for (auto& [shape, items] : groups) {
    pyjac_status rc = pyjac_eval_jacobian_multi((int32_t)items.size(), items.data(), st);
    if (rc == PYJAC_E_UNSUPPORTED) {      // different column-stream forms: one launch per mechanism
      for (auto& it : items) {
        rc = pyjac_eval_jacobian_multi(1, &it, st);
        if (rc != PYJAC_OK) break;
        n_jac_launches += 1;
      }
    } else if (rc == PYJAC_OK) {
      n_jac_launches += (int64_t)(items.size() + 7) / 8;
      if (items.size() > 1) n_multi_mech += 1;
    }
    if (rc != PYJAC_OK) return rc;
  }
  for (auto& [key, E] : extents) {
    const pyjac_mech* m = mech_of(key);
    const Pool& P = pl.at(key);
    pyjac_status rc = pyjac_newton_factor_solve(m, E, P.C, P.jac, P.h, R.gamma, P.rhs, P.x, R.mode, max_refine, rtol,
                                                P.info, P.ws, P.wsb, st);
    if (rc != PYJAC_OK) return rc;
  }
  return PYJAC_OK;
}

int pyjac_server::launch(pyjac::sched::Round& R) {
  hipSetDevice(device);
  hipStream_t st = streams[R.slot];
  auto& pl = pools[R.slot];
  // place the requests side by side per mechanism and copy their inputs in
  std::vector<std::pair<int, int64_t>> extents;
  for (size_t q = 0; q < R.reqs.size();) {
    const int key = R.reqs[q]->mech;
    const Pool& P = pl.at(key);
    int64_t col = 0;
    for (; q < R.reqs.size() && R.reqs[q]->mech == key; ++q) {
      auto* pay = static_cast<Payload*>(R.reqs[q]->payload);
      const int64_t n = R.reqs[q]->n;
      const int N = pay->N;
      const PinLayout L = pin_layout(N, n);
      const size_t w = (size_t)n * 8;
      pay->col = col;
      if (hipMemcpy2DAsync(P.phi + col, P.C * 8, pay->pin + L.phi, w, w, N, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync(P.p + col, pay->pin + L.p, w, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync(P.h + col, pay->pin + L.h, w, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpy2DAsync(P.rhs + col, P.C * 8, pay->pin + L.rhs, w, w, N, hipMemcpyHostToDevice, st) != hipSuccess) {
        set_error("request copy-in failed");
        return PYJAC_E_DEVICE;
      }
      col += n;
    }
    extents.push_back({key, std::min(P.C, (col + kExtentQuantum - 1) / kExtentQuantum * kExtentQuantum)});
  }
  // the round's kernel sequence: eager the first time, captured the second,
  // replayed afterwards
  std::string sig = std::to_string(R.mode) + "/";
  sig.append(reinterpret_cast<const char*>(&R.gamma), sizeof(double));
  for (auto& [key, E] : extents) sig += "/" + std::to_string(key) + ":" + std::to_string(E);
  GraphEntry& G = graphs[R.slot][sig];
  int rc = PYJAC_OK;
  if (G.exec) {
    if (hipGraphLaunch(G.exec, st) != hipSuccess) {
      set_error("graph launch failed");
      return PYJAC_E_DEVICE;
    }
    n_replayed += 1;
  } else if (G.seen == 0 || G.no_graph) {
    rc = compute(R, extents);
    G.seen += 1;
    n_eager += 1;
  } else {
    hipGraph_t graph = nullptr;
    bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      rc = compute(R, extents);
      const bool ended = hipStreamEndCapture(st, &graph) == hipSuccess;
      ok = ended && rc == PYJAC_OK && graph;
    }
    if (ok) ok = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) hipGraphDestroy(graph);
    if (ok) ok = hipGraphLaunch(G.exec, st) == hipSuccess;
    if (ok) {
      n_captured += 1;
    } else {
      // capture refused: run this and later rounds of the sequence eagerly
      if (G.exec) {
        hipGraphExecDestroy(G.exec);
        G.exec = nullptr;
      }
      G.no_graph = true;
      hipGetLastError();
      rc = compute(R, extents);
      n_eager += 1;
    }
  }
  if (rc != PYJAC_OK) {
    set_error(pyjac_last_error());
    return rc;
  }
  // results out
  for (auto& r : R.reqs) {
    auto* pay = static_cast<Payload*>(r->payload);
    const Pool& P = pl.at(r->mech);
    const PinLayout L = pin_layout(pay->N, r->n);
    const size_t w = (size_t)r->n * 8;
    if (hipMemcpy2DAsync(pay->pin + L.x, w, P.x + pay->col, P.C * 8, w, pay->N, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipMemcpyAsync(pay->pin + L.info, P.info + pay->col, (size_t)r->n * 4, hipMemcpyDeviceToHost, st) !=
            hipSuccess) {
      set_error("request copy-out failed");
      return PYJAC_E_DEVICE;
    }
  }
  if (hipEventRecord(events[R.slot], st) != hipSuccess) {
    set_error("event record failed");
    return PYJAC_E_DEVICE;
  }
  return PYJAC_OK;
}

void pyjac_server::finish(pyjac::sched::Round& R) {
  const bool dev_ok = hipEventQuery(events[R.slot]) == hipSuccess;
  for (auto& r : R.reqs) {
    auto* pay = static_cast<Payload*>(r->payload);
    const PinLayout L = pin_layout(pay->N, r->n);
    std::memcpy(pay->x, pay->pin + L.x, (size_t)pay->N * r->n * 8);
    std::memcpy(pay->info, pay->pin + L.info, (size_t)r->n * 4);
    if (!dev_ok) r->status = PYJAC_E_DEVICE;
  }
  std::lock_guard<std::mutex> g(pin_mu);
  for (auto& r : R.reqs) {
    auto* pay = static_cast<Payload*>(r->payload);
    pinned.give(pay->pin_off, pay->pin_bytes);
    pay->pin = nullptr;
  }
  cv_pin.notify_all();
}

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
  S->n_streams_ = n_streams;
  S->max_batch = max_batch_states;
  S->max_refine = max_refine;
  S->rtol = rtol;
  S->budget = hbm_budget_bytes;
  int prev = 0;
  hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) return pyjac::fail(PYJAC_E_DEVICE, "no such device");
  const size_t pin_bytes = std::max<size_t>(64u << 20, std::min<size_t>(hbm_budget_bytes / 4, size_t(2) << 30));
  if (!S->pinned.init(pin_bytes)) {
    hipSetDevice(prev);
    return pyjac::fail(PYJAC_E_NOMEM, "cannot allocate pinned host staging memory");
  }
  for (int i = 0; i < n_streams; ++i) {
    hipStream_t st;
    hipEvent_t ev;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      hipSetDevice(prev);
      return pyjac::fail(PYJAC_E_DEVICE, "stream creation failed");
    }
    S->streams.push_back(st);
    S->events.push_back(ev);
  }
  if (hipStreamCreateWithFlags(&S->setup, hipStreamNonBlocking) != hipSuccess) {
    hipSetDevice(prev);
    return pyjac::fail(PYJAC_E_DEVICE, "stream creation failed");
  }
  S->pools.resize(n_streams);
  S->graphs.resize(n_streams);
  hipSetDevice(prev);
  pyjac_server* raw = S.release();
  raw->sch = std::make_unique<pyjac::sched::Scheduler>(raw, INT64_MAX / 4);
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
  if (n_states > S->max_batch) return pyjac::fail(PYJAC_E_INVALID, "request larger than max_batch_states");
  const int N = pyjac::mech_species(mech);
  // the mechanism's pools: at its first request, one per stream, of capacity
  // min(max_batch_states, what 90 % of the remaining budget holds)
  int key = -1;
  {
    std::lock_guard<std::mutex> g(S->reg_mu);
    for (size_t k = 0; k < S->mechs.size(); ++k)
      if (S->mechs[k] == mech) key = (int)k;
    if (key < 0) {
      const size_t per = pool_bytes(mech, kExtentQuantum) / kExtentQuantum + 1;
      const size_t room = S->budget > S->pool_total ? (size_t)(0.9 * (double)(S->budget - S->pool_total)) : 0;
      const int64_t fit = (int64_t)(room / ((size_t)S->n_streams_ * per));
      int64_t C = std::min<int64_t>(S->max_batch, fit);
      if (C >= kExtentQuantum) C = C / kExtentQuantum * kExtentQuantum;
      if (C < n_states) return pyjac::fail(PYJAC_E_NOMEM, "request larger than the server's HBM budget holds");
      int prev = 0;
      hipGetDevice(&prev);
      hipSetDevice(S->device);
      std::vector<Pool> made;
      pyjac_status rc = PYJAC_OK;
      for (int sl = 0; sl < S->n_streams_ && rc == PYJAC_OK; ++sl) {
        Pool P;
        P.C = C;
        P.bytes = pool_bytes(mech, C);
        const hipError_t ea = hipMalloc(&P.mem, P.bytes);
        if (ea != hipSuccess) {
          P.mem = nullptr;
          rc = pyjac::fail(PYJAC_E_NOMEM, std::string("pool allocation failed: ") + hipGetErrorName(ea));
          break;
        }
        char* b = static_cast<char*>(P.mem);
        size_t o = 0;
        auto take = [&](size_t bytes) {
          char* q = b + o;
          o += al256(bytes);
          return q;
        };
        P.phi = reinterpret_cast<double*>(take((size_t)N * C * 8));
        P.rhs = reinterpret_cast<double*>(take((size_t)N * C * 8));
        P.x = reinterpret_cast<double*>(take((size_t)N * C * 8));
        P.p = reinterpret_cast<double*>(take((size_t)C * 8));
        P.h = reinterpret_cast<double*>(take((size_t)C * 8));
        P.info = reinterpret_cast<int32_t*>(take((size_t)C * 4));
        P.jac = reinterpret_cast<double*>(take((size_t)N * N * C * 8));
        P.wsb = std::max(pyjac_newton_workspace_bytes(mech, C, 0), pyjac_newton_workspace_bytes(mech, C, 1));
        P.ws = take(P.wsb);
        made.push_back(P);
        rc = init_pool(mech, made.back(), S->setup);
      }
      hipSetDevice(prev);
      if (rc != PYJAC_OK) {
        for (auto& P : made)
          if (P.mem) hipFree(P.mem);
        return rc;
      }
      key = (int)S->mechs.size();
      S->mechs.push_back(mech);
      S->cap.push_back(C);
      for (int sl = 0; sl < S->n_streams_; ++sl) {
        S->pools[sl][key] = made[sl];
        S->pool_total += made[sl].bytes;
      }
    } else if (n_states > S->cap[key]) {
      return pyjac::fail(PYJAC_E_NOMEM, "request larger than the mechanism's pool");
    }
  }
  const PinLayout L = pin_layout(N, n_states);
  if (L.total > S->pinned.size()) return pyjac::fail(PYJAC_E_NOMEM, "request larger than the pinned staging memory");
  auto pay = std::make_unique<Payload>();
  pay->N = N;
  pay->x = x;
  pay->info = info;
  pay->pin_bytes = L.total;
  {
    // backpressure on the submitting thread while the staging memory is full
    std::unique_lock<std::mutex> lk(S->pin_mu);
    size_t off = SIZE_MAX;
    while (!S->closing && (off = S->pinned.take(L.total)) == SIZE_MAX) S->cv_pin.wait(lk);
    if (S->closing) {
      if (off != SIZE_MAX) S->pinned.give(off, L.total);
      return pyjac::fail(PYJAC_E_INVALID, "server is shutting down");
    }
    pay->pin_off = off;
    pay->pin = S->pinned.ptr(off);
  }
  const size_t w = (size_t)n_states * 8;
  std::memcpy(pay->pin + L.phi, phi, (size_t)N * w);
  std::memcpy(pay->pin + L.p, p, w);
  std::memcpy(pay->pin + L.h, h, w);
  std::memcpy(pay->pin + L.rhs, rhs, (size_t)N * w);
  auto r = std::make_shared<pyjac::sched::Request>();
  r->mech = key;
  r->n = n_states;
  r->mode = mode;
  r->gamma = gamma;
  r->payload = pay.release();
  const uint64_t id = S->sch->submit(r);
  if (!id) {
    auto* q = static_cast<Payload*>(r->payload);
    {
      std::lock_guard<std::mutex> g(S->pin_mu);
      S->pinned.give(q->pin_off, q->pin_bytes);
    }
    delete q;
    return pyjac::fail(PYJAC_E_INVALID, "server is shutting down");
  }
  *request_id = id;
  return PYJAC_OK;
}

// Waits until the request has completed (timeout_s < 0: no limit).  Returns
// PYJAC_OK with *latency_s set, the request's error, or PYJAC_E_INVALID for an
// unknown id / timeout.  A completed request is forgotten after this call.
pyjac_status pyjac_serve_wait(pyjac_server* S, uint64_t request_id, double timeout_s, double* latency_s) {
  if (!S) return pyjac::fail(PYJAC_E_INVALID, "NULL server");
  std::shared_ptr<pyjac::sched::Request> r;
  const int rc = S->sch->wait(request_id, timeout_s, &r);
  if (rc < 0) return pyjac::fail(PYJAC_E_INVALID, "unknown request id");
  if (rc == 0) return pyjac::fail(PYJAC_E_INVALID, "timed out");
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  delete static_cast<Payload*>(r->payload);
  r->payload = nullptr;
  if (r->status != PYJAC_OK) {
    std::lock_guard<std::mutex> g(S->err_mu);
    return pyjac::fail(r->status, S->error);
  }
  return PYJAC_OK;
}

// Totals since creation; p50/p99 latency over all completed requests;
// hbm_in_use: bytes of the resident pools.
pyjac_status pyjac_serve_stats(pyjac_server* S, int64_t* requests_done, int64_t* states_done, int64_t* batches_done,
                               double* p50_s, double* p99_s, size_t* hbm_in_use) {
  if (!S) return pyjac::fail(PYJAC_E_INVALID, "NULL server");
  pyjac::sched::Stats st = S->sch->stats();
  if (requests_done) *requests_done = st.requests_done;
  if (states_done) *states_done = st.states_done;
  if (batches_done) *batches_done = st.rounds_done;
  std::vector<double>& l = st.latencies;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) { return l.empty() ? 0.0 : l[std::min(l.size() - 1, (size_t)(q * (l.size() - 1) + 0.5))]; };
  if (p50_s) *p50_s = pct(0.50);
  if (p99_s) *p99_s = pct(0.99);
  if (hbm_in_use) {
    std::lock_guard<std::mutex> g(S->reg_mu);
    *hbm_in_use = S->pool_total;
  }
  return PYJAC_OK;
}

pyjac_status pyjac_serve_graph_stats(pyjac_server* S, int64_t* eager_rounds, int64_t* captured_rounds,
                                     int64_t* replayed_rounds, int64_t* jacobian_launches,
                                     int64_t* multi_mechanism_launches) {
  if (!S) return pyjac::fail(PYJAC_E_INVALID, "NULL server");
  if (eager_rounds) *eager_rounds = S->n_eager;
  if (captured_rounds) *captured_rounds = S->n_captured;
  if (replayed_rounds) *replayed_rounds = S->n_replayed;
  if (jacobian_launches) *jacobian_launches = S->n_jac_launches;
  if (multi_mechanism_launches) *multi_mechanism_launches = S->n_multi_mech;
  return PYJAC_OK;
}

// Finishes every submitted request, then releases graphs, pools and streams.
pyjac_status pyjac_serve_destroy(pyjac_server* S) {
  if (!S) return PYJAC_OK;
  S->sch->shutdown();
  {
    std::lock_guard<std::mutex> g(S->pin_mu);
    S->closing = true;
  }
  S->cv_pin.notify_all();
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(S->device);
  for (auto st : S->streams) hipStreamSynchronize(st);
  for (auto& gm : S->graphs)
    for (auto& [sig, G] : gm)
      if (G.exec) hipGraphExecDestroy(G.exec);
  for (auto& pm : S->pools)
    for (auto& [key, P] : pm) hipFree(P.mem);
  for (auto ev : S->events) hipEventDestroy(ev);
  for (auto st : S->streams) hipStreamDestroy(st);
  if (S->setup) hipStreamDestroy(S->setup);
  hipSetDevice(prev);
  S->sch.reset();
  delete S;
  return PYJAC_OK;
}

}  // extern "C"
