// Host-only core of the serving loop and of the device-memory accounting (see
// serve_core.hpp).  No HIP header is included here.
#include "serve_core.hpp"

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>

namespace rpa {

namespace {
// Timed waits on a condition variable, with and without a predicate.  Steady-clock waits
// go through pthread_cond_clockwait, which GCC 11's ThreadSanitizer does not intercept
// (it then takes the waiting thread for the mutex's holder); its build defines
// RPA_WAIT_ON_SYSTEM_CLOCK to wait through pthread_cond_timedwait instead.
template <class Pred>
bool wait_ms(std::condition_variable &cv, std::unique_lock<std::mutex> &lk, int ms, Pred pred) {
#ifdef RPA_WAIT_ON_SYSTEM_CLOCK
  return cv.wait_until(lk, std::chrono::system_clock::now() + std::chrono::milliseconds(ms), pred);
#else
  return cv.wait_for(lk, std::chrono::milliseconds(ms), pred);
#endif
}

void wait_ms(std::condition_variable &cv, std::unique_lock<std::mutex> &lk, int ms) {
#ifdef RPA_WAIT_ON_SYSTEM_CLOCK
  (void)cv.wait_until(lk, std::chrono::system_clock::now() + std::chrono::milliseconds(ms));
#else
  (void)cv.wait_for(lk, std::chrono::milliseconds(ms));
#endif
}
}  // namespace

double now_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---- MemLedger ---------------------------------------------------------------------

int64_t MemLedger::outstanding_locked() const {
  return std::max<int64_t>(0, reserved_ - (in_use_ - cached_));
}

void MemLedger::set_limit(int64_t limit) {
  std::lock_guard<std::mutex> g(mu_);
  limit_ = limit;
}

int64_t MemLedger::limit() {
  std::lock_guard<std::mutex> g(mu_);
  return limit_;
}

bool MemLedger::charge(int64_t bytes, bool cached, int64_t *held_out) {
  std::lock_guard<std::mutex> g(mu_);
  const int64_t held = in_use_ + (cached ? outstanding_locked() : 0);
  if (held_out) *held_out = held;
  if (bytes < 0 || held + bytes > limit_) return false;
  in_use_ += bytes;
  if (cached) cached_ += bytes;
  high_water_ = std::max(high_water_, in_use_);
  return true;
}

void MemLedger::refund(int64_t bytes, bool cached) {
  std::lock_guard<std::mutex> g(mu_);
  in_use_ -= bytes;
  if (cached) cached_ -= bytes;
}

bool MemLedger::would_fit(int64_t extra) {
  std::lock_guard<std::mutex> g(mu_);
  return in_use_ + outstanding_locked() + extra <= limit_;
}

int64_t MemLedger::sync_budget() {
  // everything outside the cache belongs to admitted jobs and lies within their
  // reservations
  std::lock_guard<std::mutex> g(mu_);
  return limit_ - std::max<int64_t>(reserved_, in_use_ - cached_);
}

bool MemLedger::try_reserve(int64_t need, int64_t *cached_out) {
  std::lock_guard<std::mutex> g(mu_);
  if (cached_out) *cached_out = cached_;
  // the synchronous calls' caches stay allocated; everything else in use is reserved
  if (need > limit_ - cached_ - reserved_) return false;
  reserved_ += need;
  return true;
}

void MemLedger::unreserve(int64_t need) {
  std::lock_guard<std::mutex> g(mu_);
  reserved_ -= need;
}

MemLedger::Snapshot MemLedger::snapshot() {
  std::lock_guard<std::mutex> g(mu_);
  return Snapshot{limit_, in_use_, high_water_, cached_, reserved_};
}

// ---- FaultPlan ---------------------------------------------------------------------

bool FaultPlan::parse(const char *spec) {
  fail_at_.clear();
  count_ = 0;
  if (!spec || !*spec) return true;
  static const char kAlloc[] = "alloc:";
  if (strncmp(spec, kAlloc, sizeof(kAlloc) - 1) != 0) return false;
  const char *p = spec + sizeof(kAlloc) - 1;
  std::vector<int64_t> at;
  for (;;) {
    char *end = nullptr;
    const long long v = strtoll(p, &end, 10);
    if (end == p || v < 1) {
      return false;
    }
    at.push_back((int64_t)v);
    if (*end == '\0') break;
    if (*end != ',') return false;
    p = end + 1;
  }
  std::sort(at.begin(), at.end());
  at.erase(std::unique(at.begin(), at.end()), at.end());
  fail_at_ = std::move(at);
  return true;
}

bool FaultPlan::alloc_fails() {
  if (fail_at_.empty()) return false;
  const int64_t n = ++count_;
  return std::binary_search(fail_at_.begin(), fail_at_.end(), n);
}

// ---- ServeQueue --------------------------------------------------------------------

ServeQueue::ServeQueue(ServeBackend &be, int nworkers, int recheck_ms, int hold_ms)
    : be_(be),
      nworkers_(std::max(1, nworkers)),
      recheck_ms_(std::max(1, recheck_ms)),
      hold_s_(std::max(0, hold_ms) * 1e-3) {}

ServeQueue::~ServeQueue() { shutdown(); }

void ServeQueue::start_locked() {
  if (started_) return;
  started_ = true;
  be_.start();
  for (int w = 0; w < nworkers_; ++w) workers_.emplace_back(&ServeQueue::worker, this, w);
}

int ServeQueue::submit(void *payload, int64_t need, uint64_t *id) {
  if (!id) return RPA_E_ARG;
  if (need < 0 || need > be_.limit()) return RPA_E_NOMEM;
  Entry *e = new Entry();
  e->need = need;
  e->payload = payload;
  e->t_submit = now_seconds();
  std::lock_guard<std::mutex> g(mu_);
  if (stop_) {
    delete e;
    return RPA_E_CANCELLED;
  }
  e->id = next_id_++;
  *id = e->id;
  jobs_[e->id] = e;
  queue_.push_back(e);
  ++submitted_;
  start_locked();
  cv_work_.notify_one();
  return RPA_OK;
}

ServeQueue::Entry *ServeQueue::pick_locked() {
  const double now = now_seconds();
  for (int attempt = 0; attempt < 2; ++attempt) {
    int64_t cached = 0;
    for (auto it = queue_.begin(); it != queue_.end(); ++it) {
      int64_t c = 0;
      if (be_.try_reserve((*it)->need, &c)) {
        Entry *e = *it;
        queue_.erase(it);
        return e;
      }
      cached = c;
      if (now - (*it)->t_submit > hold_s_) break;   // waited long enough: no job passes it
    }
    // nothing fits: if the synchronous calls' idle cache is in the way, release it (only
    // when no synchronous call runs) and look once more
    if (attempt > 0 || cached == 0 || !be_.release_cache()) break;
  }
  return nullptr;
}

void ServeQueue::worker(int w) {
  void *state = be_.worker_begin(w);
  for (;;) {
    Entry *e = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu_);
      for (;;) {
        if (!queue_.empty()) e = pick_locked();
        if (e || stop_) break;
        if (queue_.empty()) cv_work_.wait(lk);
        else wait_ms(cv_work_, lk, recheck_ms_);
      }
      if (!e) break;   // shutting down with nothing admitted
      ++running_;
    }
    e->t_start = now_seconds();
    std::string err;
    const int rc = be_.run(state, e->payload, &err);
    be_.retire(e->payload);
    {
      std::lock_guard<std::mutex> g(mu_);
      e->status = rc;
      if (rc != RPA_OK) e->err = err.empty() ? std::string("job failed") : err;
      e->t_done = now_seconds();
      e->finished = true;
      be_.unreserve(e->need);
      --running_;
      ++done_;
    }
    cv_done_.notify_all();
    cv_work_.notify_all();
  }
  be_.worker_end(state);
}

int ServeQueue::poll(uint64_t id, int32_t timeout_ms, const std::function<void(const Record &)> &consume) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = jobs_.find(id);
  if (it == jobs_.end() || joined_) return RPA_E_UNKNOWN_JOB;
  if (!it->second->finished) {
    if (timeout_ms == 0) return RPA_PENDING;
    // the predicate looks the id up again: another poller of the same id may consume and
    // free the record while this one waits
    auto ended = [&] {
      auto f = jobs_.find(id);
      return f == jobs_.end() || f->second->finished;
    };
    ++pollers_;
    if (timeout_ms < 0) cv_done_.wait(lk, ended);
    else wait_ms(cv_done_, lk, timeout_ms, ended);
    --pollers_;
    if (pollers_ == 0) cv_done_.notify_all();   // shutdown may be waiting for pollers to leave
    it = jobs_.find(id);
    if (it == jobs_.end()) return RPA_E_UNKNOWN_JOB;
    if (!it->second->finished) return RPA_PENDING;
  }
  Entry *e = it->second;
  const Record r{e->status, e->t_submit, e->t_start, e->t_done, e->need, &e->err, e->payload};
  if (consume) consume(r);
  const int st = e->status;
  jobs_.erase(it);
  be_.destroy(e->payload);
  delete e;
  return st;
}

ServeQueue::Counts ServeQueue::counts() {
  std::lock_guard<std::mutex> g(mu_);
  return Counts{submitted_, done_, running_, (int64_t)queue_.size()};
}

void ServeQueue::kick() {
  std::lock_guard<std::mutex> g(mu_);
  cv_work_.notify_all();
}

void ServeQueue::shutdown() {
  {
    std::lock_guard<std::mutex> g(mu_);
    if (joined_) return;
    stop_ = true;
    const double t = now_seconds();
    for (Entry *e : queue_) {
      e->status = RPA_E_CANCELLED;
      e->err = "cancelled by rpa_finalize";
      e->finished = true;
      e->t_done = t;
    }
    queue_.clear();
  }
  cv_work_.notify_all();
  cv_done_.notify_all();
  for (auto &t : workers_) t.join();
  workers_.clear();
  if (started_) be_.stop();
  std::unique_lock<std::mutex> lk(mu_);
  // every job has finished now; pollers still inside poll are about to return
  cv_done_.wait(lk, [&] { return pollers_ == 0; });
  joined_ = true;
  for (auto &kv : jobs_) {
    be_.destroy(kv.second->payload);
    delete kv.second;
  }
  jobs_.clear();
}

}  // namespace rpa
