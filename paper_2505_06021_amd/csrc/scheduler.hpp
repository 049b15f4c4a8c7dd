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
// they compute.
#pragma once

#include "runtime.hpp"

namespace rpa {

class Scheduler {
 public:
  explicit Scheduler(Ctx &c);
  ~Scheduler();
  int submit(const rpa_system *sys, const rpa_freq *freq, rpa_precision prec, uint64_t *id);
  int poll(uint64_t id, int32_t timeout_ms, rpa_result *out, double *eps_qw);
  void fill_stats(rpa_stats *out);
  void shutdown();

  // Device bytes a job of this shape holds while it runs (one q at a time, its B slot
  // holding kc k-points: all of them, or a chunk of a streamed q).
  static int64_t footprint(const HostSmall &hs, int nw, rpa_precision prec, int kc);

 private:
  struct Job;
  void worker(int w);
  Job *pick_locked();

  Ctx &ctx_;
  std::mutex mu_;
  std::condition_variable cv_work_;
  std::condition_variable cv_done_;
  std::deque<Job *> queue_;
  std::map<uint64_t, Job *> jobs_;
  std::vector<std::thread> workers_;
  uint64_t next_id_ = 1;
  int64_t submitted_ = 0, done_ = 0, running_ = 0;
  bool stop_ = false;
  bool started_ = false;
  Fuser *fuser_ = nullptr;   // cross-job fusion of small contraction launches
  void start_locked();
};

}  // namespace rpa
