// CPU-only tests of the serving loop's admission policy (csrc/admission.h)
// against a mock device allocator.  Built and run by tests/test_admission_cpu.py
// with the address and undefined-behaviour sanitizers, and again with the
// thread sanitizer for the threaded part.  Exit status 0 = all checks passed.
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "admission.h"

using mlcc::Admission;
using mlcc::AdmitStatus;

static int failures = 0;
#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

// Device memory with a hard budget: an allocation past it is a failure of
// the policy under test (admission must have prevented it).
struct MockHBM {
  uint64_t budget, used = 0, peak = 0;
  explicit MockHBM(uint64_t b) : budget(b) {}
  void alloc(uint64_t n) {
    CHECK(used + n <= budget);
    used += n;
    if (used > peak) peak = used;
  }
  void free(uint64_t n) {
    CHECK(n <= used);
    used -= n;
  }
};

struct Req {
  int id;
  uint64_t hbm, host;
  bool done = false;
};

static void test_accounting() {
  Admission<Req> a(100, 50, 3);
  Req r1{1, 60, 20}, r2{2, 50, 20}, r3{3, 30, 5}, r4{4, 10, 1};
  CHECK(a.reserve(101, 0) == AdmitStatus::too_large_hbm);
  CHECK(a.reserve(10, 51) == AdmitStatus::too_large_host);
  CHECK(a.reserve(r1.hbm, r1.host) == AdmitStatus::ok);
  CHECK(a.host_held() == 20);
  CHECK(a.enqueue(&r1, r1.hbm, r1.host) == AdmitStatus::ok);
  CHECK(a.reserve(r2.hbm, r2.host) == AdmitStatus::ok && a.enqueue(&r2, r2.hbm, r2.host) == AdmitStatus::ok);
  // host bound: 40 held, 20 more would pass 50
  CHECK(a.reserve(10, 20) == AdmitStatus::busy);
  CHECK(a.reserve(r3.hbm, r3.host) == AdmitStatus::ok && a.enqueue(&r3, r3.hbm, r3.host) == AdmitStatus::ok);
  // queue of three is full
  CHECK(a.reserve(r4.hbm, r4.host) == AdmitStatus::busy);
  CHECK(a.queued() == 3 && a.host_queued() == 45);
  // FIFO with backfill: r1 (60) fits, then r2 (50) does not (40 left) but r3 (30) does
  uint64_t h = 0, x = 0;
  CHECK(a.admit(&h, &x) == &r1 && h == 60 && x == 20);
  CHECK(a.admit(&h, &x) == &r3 && h == 30);
  CHECK(a.admit() == nullptr);
  CHECK(a.hbm_in_use() == 90 && a.queued() == 1);
  a.drop_host(r1.host);
  a.drop_host(r3.host);
  CHECK(a.host_held() == 20);
  a.release(r1.hbm);
  CHECK(a.admit() == &r2 && a.hbm_in_use() == 80);
  // a reservation given back
  CHECK(a.reserve(5, 10) == AdmitStatus::ok);
  CHECK(a.host_held() == 30);
  a.cancel(10);
  CHECK(a.host_held() == 20);
  // stop returns what is queued and refuses further work
  CHECK(a.reserve(r4.hbm, r4.host) == AdmitStatus::ok && a.enqueue(&r4, r4.hbm, r4.host) == AdmitStatus::ok);
  auto left = a.stop();
  CHECK(left.size() == 1 && left[0].req == &r4);
  CHECK(a.reserve(1, 1) == AdmitStatus::stopped);
  CHECK(a.enqueue(&r4, 1, 1) == AdmitStatus::stopped);
}

// Event-driven simulation: lanes admit, hold device memory for a random
// duration, release.  Device use never passes the budget, host bytes never
// pass the host bound, every request that fits alone finishes.
static void test_simulation(unsigned seed) {
  std::mt19937_64 rng(seed);
  const uint64_t budget = 1000, host_budget = 400;
  Admission<Req> a(budget, host_budget, 16);
  MockHBM hbm(budget);
  std::vector<Req> reqs(300);
  for (int i = 0; i < (int)reqs.size(); ++i)
    reqs[i] = Req{i, 1 + rng() % budget, rng() % 120};
  struct Running { Req *r; int left; };
  std::vector<Running> running;
  const int lanes = 6;
  size_t next = 0, finished = 0, refused = 0;
  for (int step = 0; step < 200000 && finished + refused < reqs.size(); ++step) {
    // submit a few
    for (int s = 0; s < 2 && next < reqs.size(); ++s) {
      Req &r = reqs[next];
      const AdmitStatus st = a.reserve(r.hbm, r.host);
      if (st == AdmitStatus::busy) break;  // try again next step
      ++next;
      if (st != AdmitStatus::ok) { ++refused; continue; }
      CHECK(a.enqueue(&r, r.hbm, r.host) == AdmitStatus::ok);
    }
    CHECK(a.host_held() <= host_budget);
    // admit into free lanes
    while ((int)running.size() < lanes) {
      uint64_t h = 0, x = 0;
      Req *r = a.admit(&h, &x);
      if (!r) break;
      hbm.alloc(h);
      a.drop_host(x);  // inputs staged on the device
      running.push_back(Running{r, 1 + (int)(rng() % 5)});
    }
    CHECK(a.hbm_in_use() == hbm.used && hbm.used <= budget);
    // progress
    for (size_t i = 0; i < running.size();) {
      if (--running[i].left == 0) {
        hbm.free(running[i].r->hbm);
        a.release(running[i].r->hbm);
        running[i].r->done = true;
        ++finished;
        running[i] = running.back();
        running.pop_back();
      } else {
        ++i;
      }
    }
  }
  CHECK(finished + refused == reqs.size());
  CHECK(running.empty() && a.hbm_in_use() == 0 && a.host_held() == 0);
  for (auto &r : reqs) CHECK(r.done || r.host > host_budget);
}

// Threads as in the server: submitters and lanes around one mutex and a
// condition variable.
static void test_threads() {
  const uint64_t budget = 500, host_budget = 300;
  Admission<Req> a(budget, host_budget, 8);
  MockHBM hbm(budget);
  std::mutex mu;
  std::condition_variable cv;
  const int n_req = 400;
  std::vector<Req> reqs(n_req);
  std::mt19937_64 rng(7);
  for (int i = 0; i < n_req; ++i) reqs[i] = Req{i, 1 + rng() % budget, rng() % 100};
  std::atomic<int> submitted{0}, done{0};
  std::vector<std::thread> th;
  for (int s = 0; s < 3; ++s)
    th.emplace_back([&, s]() {
      for (int i = s; i < n_req; i += 3) {
        for (;;) {
          std::unique_lock<std::mutex> lk(mu);
          const AdmitStatus st = a.reserve(reqs[i].hbm, reqs[i].host);
          if (st == AdmitStatus::ok) {
            CHECK(a.enqueue(&reqs[i], reqs[i].hbm, reqs[i].host) == AdmitStatus::ok);
            ++submitted;
            break;
          }
          CHECK(st == AdmitStatus::busy);
          cv.wait(lk);
        }
        cv.notify_all();
      }
    });
  for (int l = 0; l < 4; ++l)
    th.emplace_back([&]() {
      for (;;) {
        Req *r = nullptr;
        {
          std::unique_lock<std::mutex> lk(mu);
          for (;;) {
            if (done.load() == n_req) return;
            r = a.admit();
            if (r) break;
            cv.wait(lk);
          }
          hbm.alloc(r->hbm);
          a.drop_host(r->host);
        }
        cv.notify_all();
        std::this_thread::yield();
        {
          std::lock_guard<std::mutex> lk(mu);
          CHECK(hbm.used <= budget && a.host_held() <= host_budget);
          hbm.free(r->hbm);
          a.release(r->hbm);
          r->done = true;
          ++done;
        }
        cv.notify_all();
      }
    });
  for (auto &t : th) t.join();
  CHECK(done.load() == n_req && submitted.load() == n_req);
  CHECK(a.hbm_in_use() == 0 && a.host_held() == 0 && hbm.used == 0);
}

int main(int argc, char **argv) {
  const bool threads_only = argc > 1 && std::string(argv[1]) == "threads";
  if (!threads_only) {
    test_accounting();
    for (unsigned seed = 0; seed < 20; ++seed) test_simulation(seed);
  }
  test_threads();
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("admission: all checks passed\n");
  return 0;
}
