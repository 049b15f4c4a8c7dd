// Serving loop of librpa: a job queue with HBM admission and continuous batching.
//
// rpa_submit copies a job's inputs into host memory owned by the scheduler and queues
// it.  Worker threads, each with its own HIP stream, take queued jobs whose projected
// device footprint fits into the free part of the context's HBM limit (skipping ahead
// of a job that does not fit yet), so jobs that arrive while others run are admitted as
// soon as a worker and memory are free and their kernels overlap on the device.  Each
// job's points run through the same pipeline and kernels as a synchronous rpa_energy
// call on buffers the job owns, so a job's result does not depend on what runs beside it.
// Small contraction launches of jobs in flight (split 16-bit, paired FP64 and paired FP32)
// are fused into one launch per kind (fuser.cpp), which changes when they run, never what
// they compute.  The queue, the admission and the cancellation are host-only
// (serve_core.hpp); this file adds what runs on the device.
#pragma once

#include "runtime.hpp"

namespace rpa {

class Scheduler : private ServeBackend {
 public:
  explicit Scheduler(Ctx &c);
  ~Scheduler() override;
  int submit(const rpa_system *sys, const rpa_freq *freq, rpa_precision prec, uint64_t *id);
  int poll(uint64_t id, int32_t timeout_ms, rpa_result *out, double *eps_qw);
  void fill_stats(rpa_stats *out);
  void shutdown();

  // Device bytes a job of this shape holds while it runs (one q at a time, its B slot
  // holding kc k-points: all of them, or a chunk of a streamed q).
  static int64_t footprint(const HostSmall &hs, int nw, rpa_precision prec, int kc);

 private:
  struct Job;
  // ServeBackend
  int64_t limit() override;
  bool try_reserve(int64_t need, int64_t *cached_out) override;
  void unreserve(int64_t need) override;
  bool release_cache() override;
  void start() override;
  void stop() override;
  void *worker_begin(int w) override;
  void worker_end(void *state) override;
  int run(void *state, void *payload, std::string *err) override;
  void retire(void *payload) override;
  void destroy(void *payload) override;

  Ctx &ctx_;
  std::atomic<Fuser *> fuser_{nullptr};   // cross-job fusion of small contraction launches (null until the first job)
  ServeQueue queue_;
};

}  // namespace rpa
