// Fused contraction launches of concurrent serving jobs.
//
// A serving job runs its own pipeline on its own stream.  A small job's contraction
// fills only part of the GPU (at N_aux = 200 a point is 3 tiles of 128 x 128 in split-BF16,
// ten 64 x 64 tiles in FP64), so when several jobs are in flight, their small contraction
// launches are collected here and issued as one launch of several groups: the groups'
// workgroups share the CUs, the per-launch overhead is paid once, and every group computes
// exactly what it would alone (same plan, same per-workgroup work), so results do not
// depend on fusion.  Three kinds of contraction are fused, each only with its own kind:
// the split 16-bit contraction (up to BF16_MAX_GROUPS groups of one tile edge and one
// format), and the paired FP64 and FP32 contractions (two frequencies of a q per
// workgroup; up to CHI0_MAX_GROUPS groups).  Launches big enough to fill the GPU by
// themselves go straight to the job's stream: fusing them would hold small jobs back until
// the big one ends.
//
// Protocol: the job records an event on its stream (operands prepared), posts its group
// and blocks; the fuser thread waits up to RPA_FUSE_WINDOW_US (default 300) for more
// groups (or until every registered job has posted), makes its own stream wait for each
// group's event, launches, records a completion event, and releases the posters, whose
// streams then wait for that event.
#include <algorithm>
#include <chrono>
#include <string>

#include "runtime.hpp"

namespace rpa {

enum FuseKind { kFuseHerk16 = 0, kFuseF64 = 1, kFuseF32 = 2 };

struct Fuser {
  struct Item {
    int kind = kFuseHerk16;
    Bf16Group g;            // kFuseHerk16
    Chi0Group c64{};        // kFuseF64
    Chi0F32Group c32{};     // kFuseF32
    bool cplx = true;
    hipEvent_t ready = nullptr;
    hipEvent_t done = nullptr;
    int rc = RPA_OK;
    std::string err;
    bool launched = false;
  };
  struct Pending {   // a fused launch whose events are released once it has completed
    hipEvent_t done;
    std::vector<hipEvent_t> ready;
    int waiters;     // posters that have not yet enqueued their wait on `done`
  };

  int device = 0;
  int64_t max_wg = 1024;     // groups with more workgroups launch alone
  int64_t window_us = 300;
  hipStream_t stream = nullptr;
  std::mutex mu;
  std::condition_variable cv_items, cv_launched;
  std::deque<Item *> items;
  std::deque<Pending> pending;
  int registered = 0;
  bool stop = false;
  std::thread th;
  int64_t launches = 0, fused_groups = 0, solo_groups = 0;

  void run();
  void reap_locked();
};

void Fuser::reap_locked() {
  while (!pending.empty()) {
    Pending &p = pending.front();
    if (p.waiters > 0 || hipEventQuery(p.done) != hipSuccess) break;
    (void)hipEventDestroy(p.done);
    for (hipEvent_t e : p.ready) (void)hipEventDestroy(e);
    pending.pop_front();
  }
}

void Fuser::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_items.wait(lk, [&] { return stop || !items.empty(); });
    if (stop && items.empty()) break;
    // gather: until every registered job has posted, the launch is full, or the window ends
    const auto t_end = std::chrono::steady_clock::now() + std::chrono::microseconds(window_us);
    cv_items.wait_until(lk, t_end, [&] { return stop || (int)items.size() >= std::max(1, registered) ||
                                                (int)items.size() >= BF16_MAX_GROUPS; });
    // the first item's kind and launch parameters decide which items go together
    std::vector<Item *> batch;
    const Item &f0 = *items.front();
    const int kind = f0.kind;
    const bool cplx = f0.cplx;
    const int tn = f0.g.pl.tn;
    const bool f16 = f0.g.f16;
    const int cap = kind == kFuseHerk16 ? BF16_MAX_GROUPS : CHI0_MAX_GROUPS;
    for (auto it = items.begin(); it != items.end() && (int)batch.size() < cap;) {
      const Item &c = **it;
      const bool same = c.kind == kind && c.cplx == cplx &&
                        (kind != kFuseHerk16 || (c.g.pl.tn == tn && c.g.f16 == f16));
      if (same) {
        batch.push_back(*it);
        it = items.erase(it);
      } else {
        ++it;
      }
    }
    // smallest groups first: their workgroups are dispatched first
    auto wgs = [](const Item *a) -> int64_t {
      if (a->kind == kFuseHerk16) return (int64_t)a->g.pl.ntiles * a->g.pl.nsplit * a->g.npts;
      return chi0_paired_workgroups(a->kind == kFuseF64 ? a->c64.a : a->c32.a);
    };
    std::sort(batch.begin(), batch.end(), [&](const Item *a, const Item *b) { return wgs(a) < wgs(b); });
    std::vector<Bf16Group> groups;
    std::vector<Chi0Group> g64;
    std::vector<Chi0F32Group> g32;
    Pending pend{};
    hipError_t e = hipSuccess;
    for (Item *it : batch) {
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, it->ready, 0);
      groups.push_back(it->g);
      g64.push_back(it->c64);
      g32.push_back(it->c32);
      pend.ready.push_back(it->ready);
    }
    if (e == hipSuccess) {
      if (kind == kFuseHerk16) e = launch_bf16_herk_groups(stream, groups.data(), (int)groups.size(), cplx);
      else if (kind == kFuseF64) e = launch_chi0_f64_paired_groups(stream, g64.data(), (int)g64.size(), cplx);
      else e = launch_chi0_f32_paired_groups(stream, g32.data(), (int)g32.size());
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pend.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(pend.done, stream);
    const int rc = e == hipSuccess ? RPA_OK : RPA_E_DEVICE;
    ++launches;
    fused_groups += (int64_t)batch.size();
    pend.waiters = rc == RPA_OK ? (int)batch.size() : 0;
    for (Item *it : batch) {
      it->rc = rc;
      if (rc != RPA_OK) it->err = hipGetErrorString(e);
      it->done = rc == RPA_OK ? pend.done : nullptr;
      it->launched = true;
    }
    if (rc == RPA_OK) {
      pending.push_back(pend);
    } else {
      // nothing waits on these events once the posters see the error; the stream
      // synchronisation below makes them safe to destroy
      (void)hipStreamSynchronize(stream);
      if (pend.done) (void)hipEventDestroy(pend.done);
      for (hipEvent_t r : pend.ready) (void)hipEventDestroy(r);
    }
    cv_launched.notify_all();
    reap_locked();
  }
}

Fuser *fuser_create(int device, int ncu) {
  Fuser *f = new Fuser();
  f->device = device;
  f->max_wg = 4LL * (ncu > 0 ? ncu : 256);
  if (const char *w = getenv("RPA_FUSE_WINDOW_US")) f->window_us = std::max(0, atoi(w));
  if (hipStreamCreateWithFlags(&f->stream, hipStreamNonBlocking) != hipSuccess) {
    delete f;
    return nullptr;
  }
  f->th = std::thread(&Fuser::run, f);
  return f;
}

void fuser_destroy(Fuser *f) {
  if (!f) return;
  {
    std::lock_guard<std::mutex> g(f->mu);
    f->stop = true;
  }
  f->cv_items.notify_all();
  f->th.join();
  (void)hipStreamSynchronize(f->stream);
  {
    std::lock_guard<std::mutex> g(f->mu);
    for (Fuser::Pending &p : f->pending) p.waiters = 0;
    f->reap_locked();
  }
  (void)hipStreamDestroy(f->stream);
  delete f;
}

void fuser_register(Fuser *f, int delta) {
  if (!f) return;
  {
    std::lock_guard<std::mutex> g(f->mu);
    f->registered += delta;
  }
  f->cv_items.notify_all();
}

void fuser_stats(Fuser *f, int64_t *launches, int64_t *fused_groups, int64_t *solo_groups) {
  if (!f) {
    *launches = *fused_groups = *solo_groups = 0;
    return;
  }
  std::lock_guard<std::mutex> g(f->mu);
  *launches = f->launches;
  *fused_groups = f->fused_groups;
  *solo_groups = f->solo_groups;
}

namespace {
// Post an item (prepared by the caller) and block until the fuser has launched it; the
// caller's stream then waits for the launch.
int post_and_wait(Fuser *f, hipStream_t st, Fuser::Item &it) {
  RPA_HIP(hipEventCreateWithFlags(&it.ready, hipEventDisableTiming));
  {
    hipError_t e = hipEventRecord(it.ready, st);
    if (e != hipSuccess) {
      (void)hipEventDestroy(it.ready);
      return fail(RPA_E_DEVICE, "hipEventRecord: %s", hipGetErrorString(e));
    }
  }
  std::unique_lock<std::mutex> lk(f->mu);
  f->items.push_back(&it);
  f->cv_items.notify_all();
  f->cv_launched.wait(lk, [&] { return it.launched; });
  if (it.rc != RPA_OK) return fail(it.rc, "fused contraction launch: %s", it.err.c_str());
  const hipError_t e = hipStreamWaitEvent(st, it.done, 0);
  // this poster no longer needs the completion event (the wait is enqueued)
  for (Fuser::Pending &p : f->pending)
    if (p.done == it.done) --p.waiters;
  f->reap_locked();
  if (e != hipSuccess) return fail(RPA_E_DEVICE, "hipStreamWaitEvent: %s", hipGetErrorString(e));
  return RPA_OK;
}

void count_solo(Fuser *f) {
  if (!f) return;
  std::lock_guard<std::mutex> lk(f->mu);
  ++f->solo_groups;
}
}  // namespace

int fused_herk(Fuser *f, hipStream_t st, const Bf16Group &g, bool cplx) {
  const int64_t wg = (int64_t)g.pl.ntiles * g.pl.nsplit * g.npts;
  if (!f || wg >= f->max_wg) {
    count_solo(f);
    RPA_HIP(launch_bf16_herk_groups(st, &g, 1, cplx));
    return RPA_OK;
  }
  Fuser::Item it;
  it.kind = kFuseHerk16;
  it.g = g;
  it.cplx = cplx;
  return post_and_wait(f, st, it);
}

int fused_chi0_f64(Fuser *f, hipStream_t st, const Chi0Args &a, int npts, bool cplx, int cfg) {
  // the paired configuration with a pair table is fused; anything else launches alone
  const bool paired = cfg == 4 && a.pairs != nullptr && a.npairs > 0;
  if (!f || !paired || chi0_paired_workgroups(a) >= f->max_wg) {
    count_solo(f);
    RPA_HIP(launch_chi0_f64(st, a, npts, cplx, cfg));
    return RPA_OK;
  }
  Fuser::Item it;
  it.kind = kFuseF64;
  it.c64 = Chi0Group{a, npts};
  it.cplx = cplx;
  return post_and_wait(f, st, it);
}

int fused_chi0_f32(Fuser *f, hipStream_t st, const Chi0Args &a, int npts, const float2 *B32, const double *diag,
                   int tile) {
  const bool paired = tile == kF32T64W2 && a.pairs != nullptr && a.npairs > 0;
  if (!f || !paired || chi0_paired_workgroups(a) >= f->max_wg) {
    count_solo(f);
    RPA_HIP(launch_chi0_mixed(st, a, npts, B32, diag, 1, tile));
    return RPA_OK;
  }
  Fuser::Item it;
  it.kind = kFuseF32;
  it.c32 = Chi0F32Group{a, npts, B32, diag};
  it.cplx = true;
  return post_and_wait(f, st, it);
}

}  // namespace rpa
