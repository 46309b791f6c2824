// CPU test of the server's scheduler core with a fake executor: several
// submitting threads, random device latencies, rounds that fail to launch,
// NaN outputs, and shutdown with requests still pending.  Built with g++
// under ThreadSanitizer and AddressSanitizer by tests/test_sched_cpu.py.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_1605_03262_amd/csrc/sched.hpp"

using namespace pyjac::sched;

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c); \
      std::abort();                                                       \
    }                                                                     \
  } while (0)

struct Payload {
  std::vector<double> in;
  std::vector<double> out;
  bool poison = false;   // the round holding it fails to launch
  bool nan = false;      // the "device" produces NaN for it
};

class FakeExec : public Executor {
 public:
  FakeExec(int slots, int64_t cap) : slots_(slots), cap_(cap), inuse_(slots) {
    for (auto& u : inuse_) u = 0;
  }
  int n_slots() const override { return slots_; }
  int64_t capacity(int) const override { return cap_; }
  int launch(Round& r) override {
    CHECK(r.slot >= 0 && r.slot < slots_);
    CHECK(inuse_[r.slot].exchange(1) == 0);          // one round per slot at a time
    int64_t total = 0;
    for (auto& q : r.reqs) {
      CHECK(q->mode == r.mode && q->gamma == r.gamma);
      total += q->n;
      if (static_cast<Payload*>(q->payload)->poison) {
        inuse_[r.slot] = 0;
        return 7;
      }
    }
    for (size_t i = 1; i < r.reqs.size(); ++i) CHECK(r.reqs[i - 1]->mech <= r.reqs[i]->mech);
    std::lock_guard<std::mutex> g(mu_);
    const auto delay = std::chrono::microseconds(50 + rng_() % 400);
    due_[&r] = Clock::now() + delay;
    launched_ += 1;
    return 0;
  }
  bool poll(Round& r) override {
    std::lock_guard<std::mutex> g(mu_);
    return Clock::now() >= due_.at(&r);
  }
  void finish(Round& r) override {
    for (auto& q : r.reqs) {
      auto* p = static_cast<Payload*>(q->payload);
      p->out.resize(p->in.size());
      for (size_t i = 0; i < p->in.size(); ++i) p->out[i] = p->nan ? NAN : 2.0 * p->in[i] + (double)q->mech;
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      due_.erase(&r);
    }
    CHECK(inuse_[r.slot].exchange(0) == 1);
  }
  int launched() {
    std::lock_guard<std::mutex> g(mu_);
    return launched_;
  }

 private:
  int slots_;
  int64_t cap_;
  std::vector<std::atomic<int>> inuse_;
  std::mutex mu_;
  std::mt19937 rng_{12345};
  std::map<Round*, Clock::time_point> due_;
  int launched_ = 0;
};

static void scenario_mixed_traffic() {
  FakeExec ex(3, 600);
  Scheduler S(&ex, 900);
  const int threads = 4, per = 60;
  std::vector<std::vector<std::shared_ptr<Request>>> reqs(threads);
  std::vector<std::vector<std::unique_ptr<Payload>>> pays(threads);
  std::vector<std::thread> th;
  for (int t = 0; t < threads; ++t)
    th.emplace_back([&, t] {
      std::mt19937 g(100 + t);
      for (int i = 0; i < per; ++i) {
        auto p = std::make_unique<Payload>();
        const int n = 1 + g() % 500;
        for (int k = 0; k < n; ++k) p->in.push_back(t * 1e6 + i * 1e3 + k);
        p->poison = (i % 17 == 5);
        p->nan = (i % 13 == 3);
        auto r = std::make_shared<Request>();
        r->mech = (int)(g() % 4);
        r->n = n;
        r->mode = (int)(g() % 2);
        r->gamma = 0.4358665;
        r->payload = p.get();
        CHECK(S.submit(r) != 0);
        reqs[t].push_back(r);
        pays[t].push_back(std::move(p));
      }
    });
  for (auto& x : th) x.join();
  for (int t = 0; t < threads; ++t)
    for (int i = 0; i < per; ++i) {
      std::shared_ptr<Request> got;
      CHECK(S.wait(reqs[t][i]->id, -1.0, &got) == 1);
      const Payload& p = *pays[t][i];
      if (p.poison) {
        CHECK(got->status == 7);
        continue;
      }
      if (got->status != 0) continue;   // shared a round with a poisoned request
      CHECK(p.out.size() == p.in.size());
      for (size_t k = 0; k < p.in.size(); ++k)
        CHECK(p.nan ? std::isnan(p.out[k]) : p.out[k] == 2.0 * p.in[k] + got->mech);
    }
  const Stats st = S.stats();
  CHECK(st.requests_done == threads * per);
  CHECK((int64_t)st.latencies.size() == threads * per);
  std::printf("mixed traffic: %lld requests in %lld rounds\n", (long long)st.requests_done,
              (long long)st.rounds_done);
}

static void scenario_shutdown_with_pending() {
  FakeExec ex(1, 64);
  std::vector<std::unique_ptr<Payload>> pays;
  std::vector<std::shared_ptr<Request>> reqs;
  {
    Scheduler S(&ex, 64);
    for (int i = 0; i < 40; ++i) {
      auto p = std::make_unique<Payload>();
      p->in.assign(37, (double)i);
      auto r = std::make_shared<Request>();
      r->mech = i % 3;
      r->n = 37;
      r->payload = p.get();
      CHECK(S.submit(r) != 0);
      pays.push_back(std::move(p));
      reqs.push_back(r);
    }
    S.shutdown();                                   // returns only after every request ran
    auto late = std::make_shared<Request>();
    CHECK(S.submit(late) == 0);                     // refused after shutdown
  }
  for (size_t i = 0; i < reqs.size(); ++i) {
    CHECK(reqs[i]->done && reqs[i]->status == 0);
    CHECK(pays[i]->out.size() == 37 && pays[i]->out[0] == 2.0 * i + reqs[i]->mech);
  }
  std::printf("shutdown with pending: %d requests finished\n", (int)reqs.size());
}

static void scenario_timeout_and_unknown() {
  FakeExec ex(2, 1000);
  Scheduler S(&ex, 1000);
  std::shared_ptr<Request> got;
  CHECK(S.wait(424242, 0.01, &got) == -1);
  Payload p;
  p.in.assign(10, 1.0);
  auto r = std::make_shared<Request>();
  r->n = 10;
  r->payload = &p;
  const uint64_t id = S.submit(r);
  int rc = 0;
  while ((rc = S.wait(id, 0.0001, &got)) == 0) {}
  CHECK(rc == 1 && got->status == 0 && p.out[9] == 2.0);
  std::printf("timeouts: ok\n");
}

int main() {
  scenario_mixed_traffic();
  scenario_shutdown_with_pending();
  scenario_timeout_and_unknown();
  std::printf("OK\n");
  return 0;
}
