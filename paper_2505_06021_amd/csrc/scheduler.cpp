// Serving loop: job queue, HBM admission, worker streams (see scheduler.hpp).
#include "scheduler.hpp"

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>

namespace rpa {

struct Scheduler::Job {
  // owned host copies of the inputs
  std::vector<int32_t> kq;
  std::vector<double> eps_occ, eps_virt, zeta_k, zeta_q, omega, weight;
  std::vector<char> B, vhalf;
  rpa_system sys{};
  HostSmall hs;
  rpa_precision prec = RPA_FP64;
  int64_t need = 0;   // device footprint, reserved while the job runs
  // outcome
  double E = 0.0;
  std::vector<double> eps;
};

namespace {
int worker_count() {
  const char *s = getenv("RPA_SERVE_WORKERS");
  int n = s ? atoi(s) : 4;
  return std::max(1, std::min(n, 16));
}

// How long a queued job may be passed by later jobs that fit before it (milliseconds).
int hold_ms() {
  const char *s = getenv("RPA_SERVE_HOLD_MS");
  return s ? std::max(0, atoi(s)) : 60000;
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

Scheduler::Scheduler(Ctx &c) : ctx_(c), queue_(*this, worker_count(), 20, hold_ms()) {}

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
  const int64_t lim = ctx_.mem.limit();
  int64_t need = footprint(hs, freq->nw, prec, hs.nk);
  // a job whose whole q does not fit the limit streams its q's one k-point at a time
  if (need > lim) need = footprint(hs, freq->nw, prec, 1);
  if (need > lim)
    return fail(RPA_E_NOMEM, "job needs %lld device bytes, above the limit %lld", (long long)need,
                (long long)lim);
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
  j->need = need;
  const int rc = queue_.submit(j.get(), need, id);
  if (rc == RPA_E_CANCELLED) return fail(rc, "context is shutting down");
  if (rc != RPA_OK) return fail(rc, "job of %lld device bytes refused", (long long)need);
  j.release();   // the queue owns it now
  return RPA_OK;
}

// ---- ServeBackend: what a job does on the device ------------------------------------

int64_t Scheduler::limit() { return ctx_.mem.limit(); }

bool Scheduler::try_reserve(int64_t need, int64_t *cached_out) { return ctx_.mem.try_reserve(need, cached_out); }

void Scheduler::unreserve(int64_t need) { ctx_.mem.unreserve(need); }

bool Scheduler::release_cache() {
  // only when no synchronous call is running: try_lock never waits
  if (!ctx_.mu.try_lock()) return false;
  const bool any = !ctx_.cache.empty();
  ctx_.free_cache();
  ctx_.mu.unlock();
  return any;
}

void Scheduler::start() {
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx_.device) != hipSuccess) ncu = 256;
  fuser_.store(fuser_create(ctx_.device, ncu));   // null: every contraction launches alone
}

void Scheduler::stop() {
  fuser_destroy(fuser_.exchange(nullptr));
}

void *Scheduler::worker_begin(int) {
  (void)hipSetDevice(ctx_.device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  return (void *)st;
}

void Scheduler::worker_end(void *state) {
  if (state) (void)hipStreamDestroy((hipStream_t)state);
}

int Scheduler::run(void *state, void *payload, std::string *err) {
  Job *j = (Job *)payload;
  hipStream_t st = (hipStream_t)state;
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
    pj.fuser = fuser_.load();
    // every precision's small contractions may be fused with other jobs' of their kind
    fuser_register(pj.fuser, +1);
    rc = run_points(ctx_, st, pj, j->need, false);   // within the job's reservation
    fuser_register(pj.fuser, -1);
    if (rc == RPA_OK) {
      j->E = pj.E;
      j->eps = std::move(pj.eps);
    }
  }
  if (rc != RPA_OK) *err = last_error();
  return rc;
}

void Scheduler::retire(void *payload) {
  Job *j = (Job *)payload;
  std::vector<char>().swap(j->B);
  std::vector<char>().swap(j->vhalf);
}

void Scheduler::destroy(void *payload) { delete (Job *)payload; }

int Scheduler::poll(uint64_t id, int32_t timeout_ms, rpa_result *out, double *eps_qw) {
  if (!out) return fail(RPA_E_ARG, "result pointer is NULL");
  std::string err;
  const int st = queue_.poll(id, timeout_ms, [&](const ServeQueue::Record &r) {
    const Job *j = (const Job *)r.payload;
    out->E = j->E;
    out->status = r.status;
    out->npoints = j->hs.nq * (int32_t)j->omega.size();
    out->t_submit = r.t_submit;
    out->t_start = r.t_start;
    out->t_done = r.t_done;
    out->hbm_bytes = r.need;
    if (eps_qw && r.status == RPA_OK) memcpy(eps_qw, j->eps.data(), j->eps.size() * 8);
    err = *r.err;
  });
  if (st == RPA_E_UNKNOWN_JOB)
    return fail(st, "job %llu is unknown or already consumed", (unsigned long long)id);
  if (st != RPA_OK && st != RPA_PENDING) set_error("%s", err.c_str());
  return st;
}

void Scheduler::fill_stats(rpa_stats *out) {
  const ServeQueue::Counts n = queue_.counts();
  out->jobs_submitted = n.submitted;
  out->jobs_done = n.done;
  out->jobs_running = n.running;
  out->jobs_queued = n.queued;
  fuser_stats(fuser_.load(), &out->fused_launches, &out->fused_groups, &out->solo_groups);
}

void Scheduler::shutdown() { queue_.shutdown(); }

}  // namespace rpa
