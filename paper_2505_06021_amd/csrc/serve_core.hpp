// Host-only core of the serving loop and of the device-memory accounting.
//
// Nothing here touches HIP: the ledger counts bytes, the queue admits jobs against it and
// hands them to worker threads, and what a job does on the device lives behind
// ServeBackend (scheduler.cpp implements it with streams and the point pipeline).  Kept
// apart so that a plain CPU build, with AddressSanitizer, UndefinedBehaviorSanitizer or
// ThreadSanitizer, can drive the same admission, cancellation and failure paths with a
// fake backend (tests/native/serve_core_check.cpp).
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rpa.h"

namespace rpa {

double now_seconds();

// Device-memory accounting of one context (bytes; every member takes the ledger's lock).
// in_use counts every allocation; cached the part held by the grow-only workspaces of
// synchronous calls; reserved the footprints of admitted serving jobs.  A job allocates
// only within its own footprint, so reserved - (in_use - cached) is what admitted jobs
// may still allocate ("outstanding"), and a synchronous call must leave that free.
class MemLedger {
 public:
  struct Snapshot {
    int64_t limit, in_use, high_water, cached, reserved;
  };
  void set_limit(int64_t limit);
  int64_t limit();
  // Account an allocation of `bytes` (cached: a synchronous call's workspace, which must
  // also leave room for the outstanding reservations).  False if it does not fit; then
  // *held_out (if given) is what is in use or reserved.
  bool charge(int64_t bytes, bool cached, int64_t *held_out = nullptr);
  void refund(int64_t bytes, bool cached);
  // Whether a synchronous call may allocate `extra` more bytes now.
  bool would_fit(int64_t extra);
  // What a synchronous call may hold, its own cached workspaces included: the limit minus
  // the reservations (or minus what jobs hold, if that is more).
  int64_t sync_budget();
  // Admit a job of `need` bytes if it fits beside the cached workspaces and the other
  // reservations; the reservation is made in the same critical section as the check.
  // *cached_out (if given) receives the cached bytes seen.
  bool try_reserve(int64_t need, int64_t *cached_out = nullptr);
  void unreserve(int64_t need);
  Snapshot snapshot();

 private:
  int64_t outstanding_locked() const;
  std::mutex mu_;
  int64_t limit_ = 0, in_use_ = 0, high_water_ = 0, cached_ = 0, reserved_ = 0;
};

// Fault injection for tests of the error paths.  Spec "alloc:N[,N2,...]": the N-th
// (1-based) device allocation of the context, and each further listed one, fails with
// RPA_E_NOMEM before any memory is taken.  Thread-safe.
class FaultPlan {
 public:
  // Null or empty spec: no faults.  False (and no faults) for a malformed spec.
  bool parse(const char *spec);
  bool active() const { return !fail_at_.empty(); }
  // Count one allocation; true if this one is to fail.
  bool alloc_fails();

 private:
  std::vector<int64_t> fail_at_;   // ascending
  std::atomic<int64_t> count_{0};
};

// What is device-specific about serving a job.  Calls come from the queue's threads:
// try_reserve / release_cache with the queue's lock held (they must not call back into
// the queue), run and the worker hooks without it.
class ServeBackend {
 public:
  virtual ~ServeBackend() = default;
  virtual int64_t limit() = 0;
  virtual bool try_reserve(int64_t need, int64_t *cached_out) = 0;
  virtual void unreserve(int64_t need) = 0;
  // Free the synchronous calls' idle cached workspaces if no synchronous call is running
  // (never waits); true if anything was freed.
  virtual bool release_cache() = 0;
  // Once, before the first worker starts, and once after the last one has ended.
  virtual void start() {}
  virtual void stop() {}
  // Per-worker state (a stream); null is allowed and is passed back to run.
  virtual void *worker_begin(int w) = 0;
  virtual void worker_end(void *state) = 0;
  // Run the job; a status code, with a message in *err when it is not RPA_OK.
  virtual int run(void *state, void *payload, std::string *err) = 0;
  // The job has finished: free what only the run needed (its inputs).
  virtual void retire(void *payload) = 0;
  // The job's record is gone (polled, or the queue shut down).
  virtual void destroy(void *payload) = 0;
};

// Job queue with HBM admission: worker threads take the first queued job whose footprint
// fits the free part of the limit (skipping ahead of one that does not fit yet, unless
// that one has waited longer than hold_ms: then nothing passes it, so a large job is not
// starved by a stream of small ones), run it through the backend, and release its
// reservation when it ends.  When nothing fits and
// the synchronous calls' idle cache is what blocks, it is released; a worker that still
// finds nothing that fits looks again every recheck interval, since memory freed by a
// synchronous call does not wake it.
class ServeQueue {
 public:
  struct Record {
    int status;
    double t_submit, t_start, t_done;
    int64_t need;
    const std::string *err;
    void *payload;
  };
  struct Counts {
    int64_t submitted, done, running, queued;
  };
  ServeQueue(ServeBackend &be, int nworkers, int recheck_ms = 20, int hold_ms = 60000);
  ~ServeQueue();
  // Queue a job of `need` device bytes.  The queue owns the payload from RPA_OK on
  // (backend.destroy frees it); otherwise the caller keeps it.  RPA_E_NOMEM if the job can
  // never fit, RPA_E_CANCELLED once shutdown has begun.
  int submit(void *payload, int64_t need, uint64_t *id);
  // RPA_E_UNKNOWN_JOB, RPA_PENDING (not finished within timeout_ms; < 0 waits for good),
  // or the job's status, after consume(record) has run (with the queue's lock held) and
  // the job's record and payload are gone.
  int poll(uint64_t id, int32_t timeout_ms, const std::function<void(const Record &)> &consume);
  Counts counts();
  // Wake idle workers to look at the queue again (memory was freed elsewhere).
  void kick();
  // Cancel queued jobs (status RPA_E_CANCELLED, visible to pollers), let running ones
  // finish, join the workers, wait for pollers inside poll to leave, and destroy every
  // record.  Idempotent; no other call may start once it has been called.
  void shutdown();

 private:
  struct Entry {
    uint64_t id = 0;
    int64_t need = 0;
    void *payload = nullptr;
    int status = RPA_PENDING;
    bool finished = false;
    double t_submit = 0, t_start = 0, t_done = 0;
    std::string err;
  };
  void worker(int w);
  Entry *pick_locked();
  void start_locked();

  ServeBackend &be_;
  const int nworkers_;
  const int recheck_ms_;
  const double hold_s_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<Entry *> queue_;
  std::map<uint64_t, Entry *> jobs_;
  std::vector<std::thread> workers_;
  uint64_t next_id_ = 1;
  int64_t submitted_ = 0, done_ = 0, running_ = 0;
  int pollers_ = 0;
  bool stop_ = false, started_ = false, joined_ = false;
};

}  // namespace rpa
