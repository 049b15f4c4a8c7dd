// CPU checks of the serving core (serve_core.cpp) behind a fake executor: admission order
// and skip-ahead, jobs that can never fit, poll semantics, cancellation at shutdown,
// injected allocation failures with no leaked bytes, progress when memory is freed by a
// synchronous call without a notification, several pollers of one job, and a stress run
// with concurrent submitters, pollers and a synchronous caller holding cached workspace;
// a large job is not starved by small ones that keep arriving.
// Built by tests/test_serve_core.py with AddressSanitizer + UndefinedBehaviorSanitizer
// and, separately, with ThreadSanitizer; any failed check exits with status 1.
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "serve_core.hpp"

using namespace rpa;

static int g_failures = 0;
#define CHECK(cond)                                                              \
  do {                                                                           \
    if (!(cond)) {                                                               \
      fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond);         \
      ++g_failures;                                                              \
    }                                                                            \
  } while (0)

static void sleep_ms(int ms) { std::this_thread::sleep_for(std::chrono::milliseconds(ms)); }

struct FakeJob {
  int tag = 0;
  int64_t need = 0;
  int allocs = 1;       // pieces the run allocates, need / allocs bytes each
  int run_us = 0;
  std::vector<char> inputs = std::vector<char>(64);
};

// Executor stand-in: a ledger of its own, gates that hold chosen jobs inside run, and a
// simulated synchronous caller whose idle cached workspace release_cache may free.
class FakeBackend : public ServeBackend {
 public:
  MemLedger mem;
  FaultPlan faults;
  std::mutex m;
  std::condition_variable cv;
  std::set<int> gated;            // tags held inside run until opened
  std::vector<int> started;       // tags in the order their runs began
  bool sync_busy = false;         // a synchronous call is running: release_cache refuses
  int64_t sync_idle_cached = 0;   // idle cached bytes release_cache may free
  std::atomic<int> n_start{0}, n_stop{0}, n_begin{0}, n_end{0}, n_retired{0}, n_destroyed{0};
  std::atomic<int> violations{0};

  explicit FakeBackend(int64_t limit) { mem.set_limit(limit); }

  void open(int tag) {
    std::lock_guard<std::mutex> g(m);
    gated.erase(tag);
    cv.notify_all();
  }
  bool has_started(int tag) {
    std::lock_guard<std::mutex> g(m);
    for (int t : started)
      if (t == tag) return true;
    return false;
  }
  bool wait_started(int tag, int ms) {
    for (int i = 0; i < ms; ++i) {
      if (has_started(tag)) return true;
      sleep_ms(1);
    }
    return has_started(tag);
  }
  void check_invariants() {
    const MemLedger::Snapshot s = mem.snapshot();
    // jobs allocate only within their reservations, and nothing exceeds the limit
    if (s.in_use > s.limit || s.reserved < 0 || s.in_use - s.cached > s.reserved || s.cached < 0) ++violations;
  }

  int64_t limit() override { return mem.limit(); }
  bool try_reserve(int64_t need, int64_t *cached_out) override { return mem.try_reserve(need, cached_out); }
  void unreserve(int64_t need) override { mem.unreserve(need); }
  bool release_cache() override {
    std::lock_guard<std::mutex> g(m);
    if (sync_busy || sync_idle_cached == 0) return false;
    mem.refund(sync_idle_cached, true);
    sync_idle_cached = 0;
    return true;
  }
  void start() override { ++n_start; }
  void stop() override { ++n_stop; }
  void *worker_begin(int w) override {
    ++n_begin;
    return new int(w);
  }
  void worker_end(void *state) override {
    ++n_end;
    delete (int *)state;
  }
  int run(void *state, void *payload, std::string *err) override {
    (void)state;
    FakeJob *j = (FakeJob *)payload;
    {
      std::unique_lock<std::mutex> lk(m);
      started.push_back(j->tag);
      cv.wait(lk, [&] { return gated.count(j->tag) == 0; });
    }
    std::vector<int64_t> held;
    int rc = RPA_OK;
    for (int i = 0; i < j->allocs; ++i) {
      if (faults.alloc_fails()) {
        rc = RPA_E_NOMEM;
        *err = "injected allocation failure";
        break;
      }
      const int64_t part = j->need / j->allocs;
      if (!mem.charge(part, false)) {
        rc = RPA_E_NOMEM;
        *err = "allocation beyond the limit";
        break;
      }
      held.push_back(part);
      check_invariants();
    }
    if (j->run_us > 0) std::this_thread::sleep_for(std::chrono::microseconds(j->run_us));
    for (int64_t b : held) mem.refund(b, false);
    return rc;
  }
  void retire(void *payload) override {
    ++n_retired;
    std::vector<char>().swap(((FakeJob *)payload)->inputs);
  }
  void destroy(void *payload) override {
    ++n_destroyed;
    delete (FakeJob *)payload;
  }
};

static uint64_t submit(ServeQueue &q, int tag, int64_t need, int allocs = 1, int run_us = 0) {
  FakeJob *j = new FakeJob();
  j->tag = tag;
  j->need = need;
  j->allocs = allocs;
  j->run_us = run_us;
  uint64_t id = 0;
  const int rc = q.submit(j, need, &id);
  CHECK(rc == RPA_OK);
  if (rc != RPA_OK) delete j;
  return id;
}

static int poll_status(ServeQueue &q, uint64_t id, int timeout_ms, std::string *err = nullptr) {
  return q.poll(id, timeout_ms, [&](const ServeQueue::Record &r) {
    if (err) *err = *r.err;
    CHECK(r.t_submit <= r.t_done);
  });
}

static void check_ledger_zero(FakeBackend &be) {
  const MemLedger::Snapshot s = be.mem.snapshot();
  CHECK(s.in_use == 0);
  CHECK(s.cached == 0);
  CHECK(s.reserved == 0);
}

// ---- tests --------------------------------------------------------------------------

static void test_ledger() {
  MemLedger m;
  m.set_limit(100);
  CHECK(m.charge(30, true));              // a synchronous call's workspace
  CHECK(m.try_reserve(60));               // 100 - 30 cached - 0 reserved
  CHECK(!m.try_reserve(20));              // only 10 left
  CHECK(m.would_fit(10));                 // 30 in use + 60 outstanding + 10
  CHECK(!m.would_fit(11));
  CHECK(m.charge(40, false));             // the admitted job allocates within its 60
  int64_t held = 0;
  CHECK(!m.charge(11, true, &held));      // 70 in use + 20 outstanding + 11 > 100
  CHECK(held == 90);
  CHECK(m.charge(10, true));
  CHECK(m.sync_budget() == 100 - 60);     // the limit minus the reservation
  CHECK(!m.charge(-1, false));
  MemLedger::Snapshot s = m.snapshot();
  CHECK(s.in_use == 80 && s.cached == 40 && s.reserved == 60 && s.high_water == 80);
  m.refund(40, false);
  m.refund(40, true);
  m.unreserve(60);
  s = m.snapshot();
  CHECK(s.in_use == 0 && s.cached == 0 && s.reserved == 0 && s.high_water == 80);
  printf("ok ledger\n");
}

static void test_fault_plan() {
  FaultPlan f;
  CHECK(f.parse(nullptr) && !f.active() && !f.alloc_fails());
  CHECK(f.parse("") && !f.active());
  CHECK(f.parse("alloc:3") && f.active());
  std::vector<bool> got;
  for (int i = 0; i < 5; ++i) got.push_back(f.alloc_fails());
  CHECK(!got[0] && !got[1] && got[2] && !got[3] && !got[4]);
  CHECK(f.parse("alloc:5,2,5"));
  got.clear();
  for (int i = 0; i < 6; ++i) got.push_back(f.alloc_fails());
  CHECK(!got[0] && got[1] && !got[2] && !got[3] && got[4] && !got[5]);
  for (const char *bad : {"alloc:", "alloc:0", "alloc:-1", "alloc:3x", "free:1", "alloc:1,,2", "alloc:2,"}) {
    CHECK(!f.parse(bad));
    CHECK(!f.active());
  }
  printf("ok fault_plan\n");
}

static void test_admission_order() {
  FakeBackend be(100);
  {
    ServeQueue q(be, 2, 5);
    be.gated = {1, 3};
    const uint64_t a = submit(q, 1, 60), b = submit(q, 2, 60), c = submit(q, 3, 30);
    CHECK(be.wait_started(1, 2000));
    CHECK(be.wait_started(3, 2000));   // skips ahead of job 2, which does not fit beside job 1
    sleep_ms(30);
    CHECK(!be.has_started(2));
    CHECK(q.counts().queued == 1 && q.counts().running == 2);
    be.open(1);
    CHECK(be.wait_started(2, 2000));   // fits beside job 3 once job 1 has ended
    be.open(3);
    CHECK(poll_status(q, a, -1) == RPA_OK);
    CHECK(poll_status(q, b, -1) == RPA_OK);
    CHECK(poll_status(q, c, -1) == RPA_OK);
    {
      std::lock_guard<std::mutex> g(be.m);
      CHECK(be.started.size() == 3 && be.started[0] == 1 && be.started[1] == 3 && be.started[2] == 2);
    }
    // a job that can never fit is refused at submit and stays the caller's
    FakeJob *big = new FakeJob();
    uint64_t id = 0;
    CHECK(q.submit(big, 101, &id) == RPA_E_NOMEM);
    delete big;
    const ServeQueue::Counts n = q.counts();
    CHECK(n.submitted == 3 && n.done == 3 && n.running == 0 && n.queued == 0);
  }
  check_ledger_zero(be);
  CHECK(be.n_destroyed == 3 && be.n_retired == 3);
  CHECK(be.n_begin == 2 && be.n_end == 2 && be.n_start == 1 && be.n_stop == 1);
  printf("ok admission_order\n");
}

static void test_poll_semantics() {
  FakeBackend be(100);
  ServeQueue q(be, 1, 5);
  be.gated = {7};
  const uint64_t a = submit(q, 7, 10);
  CHECK(q.poll(a + 100, 0, nullptr) == RPA_E_UNKNOWN_JOB);
  CHECK(q.poll(a, 0, nullptr) == RPA_PENDING);
  const auto t0 = std::chrono::steady_clock::now();
  CHECK(q.poll(a, 30, nullptr) == RPA_PENDING);
  const double waited = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  CHECK(waited >= 0.025);
  be.open(7);
  CHECK(poll_status(q, a, -1) == RPA_OK);
  CHECK(q.poll(a, 0, nullptr) == RPA_E_UNKNOWN_JOB);   // consumed
  q.shutdown();
  check_ledger_zero(be);
  CHECK(be.n_destroyed == 1);
  printf("ok poll_semantics\n");
}

static void test_cancel_at_shutdown() {
  FakeBackend be(100);
  ServeQueue q(be, 1, 5);
  be.gated = {1};
  const uint64_t a = submit(q, 1, 50), b = submit(q, 2, 50);
  submit(q, 3, 50);   // never polled: destroyed by the shutdown
  CHECK(be.wait_started(1, 2000));
  int st_a = 1, st_b = 1;
  std::string err_b;
  std::thread pa([&] { st_a = poll_status(q, a, -1); });
  std::thread pb([&] { st_b = poll_status(q, b, -1, &err_b); });
  sleep_ms(20);
  bool shut = false;
  std::thread sd([&] {
    q.shutdown();
    shut = true;
  });
  pb.join();   // the queued job is cancelled while job 1 still runs
  CHECK(st_b == RPA_E_CANCELLED);
  CHECK(err_b.find("cancelled") != std::string::npos);
  sleep_ms(20);
  CHECK(!shut);   // shutdown waits for the running job
  be.open(1);
  sd.join();
  pa.join();
  CHECK(st_a == RPA_OK);
  FakeJob *late = new FakeJob();
  uint64_t id = 0;
  CHECK(q.submit(late, 10, &id) == RPA_E_CANCELLED);
  delete late;
  CHECK(q.poll(a, 0, nullptr) == RPA_E_UNKNOWN_JOB);
  check_ledger_zero(be);
  CHECK(be.n_destroyed == 3 && be.n_retired == 1);
  CHECK(be.n_begin == 1 && be.n_end == 1 && be.n_stop == 1);
  printf("ok cancel_at_shutdown\n");
}

static void test_alloc_failure() {
  FakeBackend be(1000);
  CHECK(be.faults.parse("alloc:3,10"));
  {
    ServeQueue q(be, 1, 5);
    std::vector<uint64_t> ids;
    for (int i = 0; i < 4; ++i) ids.push_back(submit(q, 10 + i, 400, 4));
    // one worker: job 0 allocates #1 #2, #3 fails; job 1 #4..#7; job 2 #8 #9, #10 fails; job 3 #11..#14
    std::vector<int> st;
    std::vector<std::string> errs(4);
    for (int i = 0; i < 4; ++i) st.push_back(poll_status(q, ids[i], -1, &errs[i]));
    CHECK(st[0] == RPA_E_NOMEM && st[1] == RPA_OK && st[2] == RPA_E_NOMEM && st[3] == RPA_OK);
    CHECK(errs[0].find("injected") != std::string::npos);
    check_ledger_zero(be);   // the failed runs gave back what they had taken
  }
  CHECK(be.n_destroyed == 4);
  CHECK(be.violations == 0);
  printf("ok alloc_failure\n");
}

static void test_progress_without_notify() {
  FakeBackend be(100);
  CHECK(be.mem.charge(80, true));   // a synchronous call's workspace
  be.sync_idle_cached = 80;
  be.sync_busy = true;              // ... and the call is still running
  ServeQueue q(be, 2, 5);
  const uint64_t a = submit(q, 1, 50);
  sleep_ms(50);
  CHECK(!be.has_started(1));        // 20 bytes free, and the cache may not be released
  {
    std::lock_guard<std::mutex> g(be.m);
    be.sync_busy = false;           // the call ends; nobody tells the queue
  }
  CHECK(be.wait_started(1, 2000));  // a worker looks again within the recheck interval
  CHECK(poll_status(q, a, -1) == RPA_OK);
  q.shutdown();
  check_ledger_zero(be);
  printf("ok progress_without_notify\n");
}

static void test_two_pollers() {
  FakeBackend be(100);
  ServeQueue q(be, 1, 5);
  be.gated = {5};
  const uint64_t a = submit(q, 5, 10);
  int s1 = 1, s2 = 1;
  std::thread p1([&] { s1 = q.poll(a, -1, nullptr); });
  std::thread p2([&] { s2 = q.poll(a, -1, nullptr); });
  sleep_ms(20);
  be.open(5);
  p1.join();
  p2.join();
  CHECK((s1 == RPA_OK && s2 == RPA_E_UNKNOWN_JOB) || (s2 == RPA_OK && s1 == RPA_E_UNKNOWN_JOB));
  q.shutdown();
  CHECK(be.n_destroyed == 1);
  printf("ok two_pollers\n");
}

static void test_destructor_destroys_unpolled() {
  FakeBackend be(100);
  {
    ServeQueue q(be, 3, 5);
    for (int i = 0; i < 6; ++i) submit(q, i, 30);
    sleep_ms(20);
  }
  CHECK(be.n_destroyed == 6);
  check_ledger_zero(be);
  printf("ok destructor_destroys_unpolled\n");
}

static void test_no_starvation() {
  // two workers, a large job behind a steady stream of small ones that always fit beside
  // each other: once the large job has waited hold_ms, no small job is admitted past it
  FakeBackend be(100);
  std::atomic<bool> done{false};
  {
    ServeQueue q(be, 2, 2, 50);
    be.gated = {1, 2};
    const uint64_t a = submit(q, 1, 30), b = submit(q, 2, 30);
    CHECK(be.wait_started(1, 2000) && be.wait_started(2, 2000));
    const uint64_t big = submit(q, 1000, 80);
    std::vector<uint64_t> small;
    std::thread feeder([&] {
      for (int i = 0; i < 400 && !done; ++i) {
        small.push_back(submit(q, 2000 + i, 30, 1, 3000));
        sleep_ms(1);
      }
    });
    sleep_ms(5);
    be.open(1);
    be.open(2);
    CHECK(be.wait_started(1000, 3000));   // admitted while small jobs keep arriving
    done = true;
    feeder.join();
    CHECK(poll_status(q, a, -1) == RPA_OK && poll_status(q, b, -1) == RPA_OK);
    CHECK(poll_status(q, big, -1) == RPA_OK);
    for (uint64_t id : small) CHECK(poll_status(q, id, -1) == RPA_OK);
  }
  check_ledger_zero(be);
  printf("ok no_starvation\n");
}

static void test_stress() {
  const int64_t limit = 1000;
  FakeBackend be(limit);
  const int nsub = 4, per = 100;
  std::atomic<bool> done{false};
  std::atomic<int> ok{0}, bad{0};
  {
    ServeQueue q(be, 8, 2);
    std::mutex ids_mu;
    std::vector<uint64_t> ids;
    std::vector<std::thread> th;
    for (int s = 0; s < nsub; ++s)
      th.emplace_back([&, s] {
        std::mt19937 rng(1234 + s);
        for (int i = 0; i < per; ++i) {
          const uint64_t id = submit(q, s * per + i, 1 + rng() % 600, 1 + rng() % 3, rng() % 2000);
          std::lock_guard<std::mutex> g(ids_mu);
          ids.push_back(id);
        }
      });
    // a synchronous caller growing and dropping cached workspace beside the jobs
    std::thread sync([&] {
      std::mt19937 rng(99);
      while (!done) {
        const int64_t want = rng() % 300;
        {
          std::lock_guard<std::mutex> g(be.m);
          be.sync_busy = true;
        }
        const bool got = be.mem.charge(want, true);
        be.check_invariants();
        sleep_ms(1);
        {
          std::lock_guard<std::mutex> g(be.m);
          be.sync_busy = false;
          // sometimes the workspace stays cached (idle) for release_cache to take
          if (got && be.sync_idle_cached == 0 && rng() % 2) be.sync_idle_cached = want;
          else if (got) be.mem.refund(want, true);
        }
      }
    });
    std::thread monitor([&] {
      while (!done) {
        be.check_invariants();
        std::this_thread::yield();
      }
    });
    for (auto &t : th) t.join();
    std::vector<std::thread> pollers;
    for (int p = 0; p < 2; ++p)
      pollers.emplace_back([&, p] {
        for (size_t i = p; i < ids.size(); i += 2) {
          const int st = q.poll(ids[i], -1, nullptr);
          if (st == RPA_OK) ++ok;
          else ++bad;
        }
      });
    for (auto &t : pollers) t.join();
    done = true;
    sync.join();
    monitor.join();
    {
      std::lock_guard<std::mutex> g(be.m);
      if (be.sync_idle_cached) be.mem.refund(be.sync_idle_cached, true);
      be.sync_idle_cached = 0;
    }
    const ServeQueue::Counts n = q.counts();
    CHECK(n.submitted == nsub * per && n.done == nsub * per && n.queued == 0 && n.running == 0);
  }
  CHECK(ok == nsub * per && bad == 0);
  CHECK(be.violations == 0);
  CHECK(be.n_destroyed == nsub * per);
  check_ledger_zero(be);
  printf("ok stress\n");
}

int main() {
  test_ledger();
  test_fault_plan();
  test_admission_order();
  test_poll_semantics();
  test_cancel_at_shutdown();
  test_alloc_failure();
  test_progress_without_notify();
  test_two_pollers();
  test_destructor_destroys_unpolled();
  test_no_starvation();
  test_stress();
  if (g_failures) {
    fprintf(stderr, "%d check(s) failed\n", g_failures);
    return 1;
  }
  printf("all ok\n");
  return 0;
}
