// Serving loop: job queue, HBM admission, worker streams (see scheduler.hpp).
#include "scheduler.hpp"

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>

namespace rpa {

struct Scheduler::Job {
  uint64_t id = 0;
  // owned host copies of the inputs
  std::vector<int32_t> kq;
  std::vector<double> eps_occ, eps_virt, zeta_k, zeta_q, omega, weight;
  std::vector<char> B, vhalf;
  rpa_system sys{};
  HostSmall hs;
  rpa_precision prec = RPA_FP64;
  int64_t need = 0;
  // outcome
  int status = RPA_PENDING;
  double E = 0.0;
  std::vector<double> eps;
  double t_submit = 0, t_start = 0, t_done = 0;
  bool finished = false;
  std::string err;
};

namespace {
int worker_count() {
  const char *s = getenv("RPA_SERVE_WORKERS");
  int n = s ? atoi(s) : 4;
  return std::max(1, std::min(n, 16));
}

template <class T>
int copy_array(std::vector<T> &dst, const T *src, size_t n, int memspace) {
  dst.resize(n);
  if (n == 0) return RPA_OK;
  if (memspace == RPA_MEM_HOST) {
    memcpy(dst.data(), src, n * sizeof(T));
  } else {
    RPA_HIP(hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost));
  }
  return RPA_OK;
}
}  // namespace

Scheduler::Scheduler(Ctx &c) : ctx_(c) {}

Scheduler::~Scheduler() { shutdown(); }

int64_t Scheduler::footprint(const HostSmall &hs, int nw, rpa_precision prec, int kc) {
  const bool mixed = prec != RPA_FP64;
  const int64_t N = hs.naux;
  // rows of one B slot: a whole q, or a chunk of kc k-points of a streamed q
  const int64_t M = (int64_t)(kc > 0 && kc < hs.nk ? kc : hs.nk) * hs.nocc * hs.nvirt;
  const int64_t belem = hs.is_complex ? 16 : 8;
  const bool bsplit = prec == RPA_BF16X3 || prec == RPA_F16X3;
  const int64_t small = (int64_t)(hs.eps_occ.size() + hs.eps_virt.size() + hs.zeta_k.size()) * 8 +
                        (int64_t)hs.kq.size() * 4 + (int64_t)hs.nq * nw * 32 + 4096 +
                        (int64_t)(hs.nq + nw + 1) * 8 +
                        (bsplit ? bf16_diag_scratch_doubles(M, (int)N) * 8
                         : mixed ? diag_exact_scratch_doubles(M, (int)N, 16) * 8 : 0) +
                        (hs.nbas > 0 ? (int64_t)(hs.c_occ.size() + hs.c_virt.size()) * 8 + 512 +
                                           ao_scratch_bytes(hs.nbas, hs.nocc, hs.naux) + ao_stage_scratch_bytes(hs)
                                     : 0);
  // one q staged at a time: FP64 B (and its FP32 copy, or its prepared split-BF16 copy),
  // V^(1/2), and per point chi0, T, the weight table and the exact diagonal -- the same
  // sizes run_points() budgets
  // (the fp16 operands' scales and maxima: a few KB per slot and per point)
  const int64_t prep = bsplit ? bf16_prepared_elems(M, (int)N) * 2 + (f16_absmax_scratch_doubles(1) + 1) * 8 : 0;
  const int64_t per_q = M * N * belem + N * N * 16 + (hs.is_complex ? 0 : N * N * 8) +
                        (bsplit ? prep : mixed ? M * N * 8 : 0);
  const int64_t per_pt = 2 * N * N * 16 + M * 8 + (mixed ? N * 8 : 0) + trln_blocked_scratch_bytes(1) + 64;
  // split-BF16: prepared right operands and partial tiles of up to four points at a time
  int64_t split_extra = 0;
  if (bsplit) {
    const int r = nw < 4 ? nw : 4;
    Bf16Plan pl;
    bf16_plan(M, (int)N, r, 256, 0, 128, &pl);
    split_extra = r * prep + bf16_partial_elems(pl, r) * 8 + 512;
  }
  // allocation granularity slack per buffer
  return small + per_q + (int64_t)nw * per_pt + split_extra + 24 * 4096;
}

void Scheduler::start_locked() {
  if (started_) return;
  started_ = true;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx_.device) != hipSuccess) ncu = 256;
  fuser_ = fuser_create(ctx_.device, ncu);   // null: every contraction launches alone
  const int n = worker_count();
  for (int w = 0; w < n; ++w) workers_.emplace_back(&Scheduler::worker, this, w);
}

int Scheduler::submit(const rpa_system *sys, const rpa_freq *freq, rpa_precision prec, uint64_t *id) {
  if (!id) return fail(RPA_E_ARG, "job_id pointer is NULL");
  if (prec != RPA_FP64 && prec != RPA_FP32 && prec != RPA_BF16X3 && prec != RPA_F16X3)
    return fail(RPA_E_ARG, "unknown precision %d", (int)prec);
  RPA_HIP(hipSetDevice(ctx_.device));
  std::unique_ptr<Job> j(new Job());
  RPA_TRY(validate_system(sys, j->hs));
  RPA_TRY(validate_freq(freq));
  if (sys->B && sys->memspace == RPA_MEM_DEVICE)
    return fail(RPA_E_ARG, "submitted jobs take B from host memory or from Philox (B = NULL)");
  const HostSmall &hs = j->hs;
  const int64_t N = hs.naux;
  const int64_t M = (int64_t)hs.nk * hs.nocc * hs.nvirt;
  const int64_t belem = hs.is_complex ? 16 : 8;
  j->need = footprint(hs, freq->nw, prec, hs.nk);
  // a job whose whole q does not fit the limit streams its q's one k-point at a time
  if (j->need > ctx_.hbm_limit) j->need = footprint(hs, freq->nw, prec, 1);
  if (j->need > ctx_.hbm_limit)
    return fail(RPA_E_NOMEM, "job needs %lld device bytes, above the limit %lld", (long long)j->need,
                (long long)ctx_.hbm_limit);
  j->kq = hs.kq;
  j->eps_occ = hs.eps_occ;
  j->eps_virt = hs.eps_virt;
  j->zeta_k = hs.zeta_k;
  j->zeta_q = hs.zeta_q;
  j->omega.assign(freq->omega, freq->omega + freq->nw);
  j->weight.assign(freq->weight, freq->weight + freq->nw);
  RPA_TRY(copy_array(j->vhalf, (const char *)sys->vhalf, (size_t)(hs.nq * N * N * belem), sys->memspace));
  if (sys->B) {
    const int64_t bbytes = (int64_t)hs.nq * M * N * belem;
    if (bbytes > ((int64_t)64 << 30))
      return fail(RPA_E_NOMEM, "explicit B of %lld bytes is too large to copy; use Philox (B = NULL)",
                  (long long)bbytes);
    RPA_TRY(copy_array(j->B, (const char *)sys->B, (size_t)bbytes, RPA_MEM_HOST));
  }
  rpa_system &s = j->sys;
  s = *sys;
  s.memspace = RPA_MEM_HOST;
  s.kq = j->kq.data();
  s.eps_occ = j->eps_occ.data();
  s.eps_virt = j->eps_virt.data();
  s.zeta_k = j->zeta_k.data();
  s.zeta_q = j->zeta_q.data();
  s.vhalf = j->vhalf.data();
  s.B = sys->B ? (const void *)j->B.data() : nullptr;
  // atomic-orbital systems: the job's own copies of the projected coefficients
  s.c_occ = j->hs.nbas > 0 ? (const void *)j->hs.c_occ.data() : nullptr;
  s.c_virt = j->hs.nbas > 0 ? (const void *)j->hs.c_virt.data() : nullptr;
  s.S_ao = j->hs.S.empty() ? nullptr : (const void *)j->hs.S.data();
  j->prec = prec;
  j->t_submit = now_seconds();
  std::lock_guard<std::mutex> g(mu_);
  if (stop_) return fail(RPA_E_CANCELLED, "context is shutting down");
  j->id = next_id_++;
  *id = j->id;
  Job *raw = j.release();
  jobs_[raw->id] = raw;
  queue_.push_back(raw);
  ++submitted_;
  start_locked();
  cv_work_.notify_one();
  return RPA_OK;
}

Scheduler::Job *Scheduler::pick_locked() {
  for (int attempt = 0; attempt < 2; ++attempt) {
    // the first queued job whose footprint fits is reserved in the same critical section
    // of the context's memory lock as the check, so a synchronous call planning at the
    // same time already sees the reservation
    int64_t cached = 0;
    for (auto it = queue_.begin(); it != queue_.end(); ++it) {
      if (ctx_.try_reserve((*it)->need, &cached)) {
        Job *j = *it;
        queue_.erase(it);
        return j;
      }
    }
    // nothing fits: if the workspace cache of the synchronous calls is in the way and no
    // synchronous call is running (try_lock never waits), release it and look again
    if (attempt > 0 || cached == 0 || !ctx_.mu.try_lock()) break;
    ctx_.free_cache();
    ctx_.mu.unlock();
  }
  return nullptr;
}

void Scheduler::worker(int w) {
  (void)w;
  (void)hipSetDevice(ctx_.device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  for (;;) {
    Job *j = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_work_.wait(lk, [&] { return stop_ || (!queue_.empty() && (j = pick_locked()) != nullptr); });
      if (!j) {
        if (stop_) break;
        continue;
      }
      ++running_;
    }
    j->t_start = now_seconds();
    int rc;
    if (!st) {
      rc = fail(RPA_E_DEVICE, "worker stream could not be created");
    } else {
      PointJob pj;
      pj.sys = &j->sys;
      pj.hs = &j->hs;
      pj.prec = j->prec;
      for (int q = 0; q < j->hs.nq; ++q)
        for (double om : j->omega) {
          pj.pq.push_back(q);
          pj.pw.push_back(om);
        }
      pj.quadrature = true;
      pj.weight = j->weight;
      pj.max_q_group = 1;
      pj.fuser = fuser_;
      // every precision's small contractions may be fused with other jobs' of their kind
      fuser_register(fuser_, +1);
      rc = run_points(ctx_, st, pj, j->need, false);
      fuser_register(fuser_, -1);
      if (rc == RPA_OK) {
        j->E = pj.E;
        j->eps = std::move(pj.eps);
      }
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      j->status = rc;
      if (rc != RPA_OK) j->err = last_error();
      j->t_done = now_seconds();
      j->finished = true;
      ctx_.unreserve(j->need);
      --running_;
      ++done_;
      // free the inputs now; the record stays until it is polled
      std::vector<char>().swap(j->B);
      std::vector<char>().swap(j->vhalf);
    }
    cv_done_.notify_all();
    cv_work_.notify_all();
  }
  if (st) (void)hipStreamDestroy(st);
}

int Scheduler::poll(uint64_t id, int32_t timeout_ms, rpa_result *out, double *eps_qw) {
  if (!out) return fail(RPA_E_ARG, "result pointer is NULL");
  std::unique_lock<std::mutex> lk(mu_);
  auto it = jobs_.find(id);
  if (it == jobs_.end()) return fail(RPA_E_UNKNOWN_JOB, "job %llu is unknown or already consumed",
                                     (unsigned long long)id);
  Job *j = it->second;
  auto done = [&] { return j->finished; };
  if (!done()) {
    if (timeout_ms == 0) return RPA_PENDING;
    if (timeout_ms < 0) cv_done_.wait(lk, done);
    else if (!cv_done_.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) return RPA_PENDING;
  }
  out->E = j->E;
  out->status = j->status;
  out->npoints = j->hs.nq * (int32_t)j->omega.size();
  out->t_submit = j->t_submit;
  out->t_start = j->t_start;
  out->t_done = j->t_done;
  out->hbm_bytes = j->need;
  if (eps_qw && j->status == RPA_OK) memcpy(eps_qw, j->eps.data(), j->eps.size() * 8);
  const int st = j->status;
  const std::string err = j->err;
  jobs_.erase(it);
  delete j;
  if (st != RPA_OK) set_error("%s", err.c_str());
  return st;
}

void Scheduler::fill_stats(rpa_stats *out) {
  std::lock_guard<std::mutex> g(mu_);
  out->jobs_submitted = submitted_;
  out->jobs_done = done_;
  out->jobs_running = running_;
  out->jobs_queued = (int64_t)queue_.size();
  fuser_stats(fuser_, &out->fused_launches, &out->fused_groups, &out->solo_groups);
}

void Scheduler::shutdown() {
  {
    std::lock_guard<std::mutex> g(mu_);
    if (stop_ && workers_.empty()) return;
    stop_ = true;
    for (Job *j : queue_) {
      j->status = RPA_E_CANCELLED;
      j->err = "cancelled by rpa_finalize";
      j->finished = true;
      j->t_done = now_seconds();
    }
    queue_.clear();
  }
  cv_work_.notify_all();
  cv_done_.notify_all();
  for (auto &t : workers_) t.join();
  workers_.clear();
  fuser_destroy(fuser_);
  fuser_ = nullptr;
  std::lock_guard<std::mutex> g(mu_);
  for (auto &kv : jobs_) delete kv.second;
  jobs_.clear();
}

}  // namespace rpa
