// Host runtime of librpa: errors, device-memory accounting, validation and the
// (q, w) point pipeline (B generation or staging -> chi0 -> Pi -> Tr ln).
#include "runtime.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>

namespace rpa {

// ---- errors ---------------------------------------------------------------------
namespace {
thread_local char g_err[1024] = {0};
}

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char *last_error() { return g_err; }

int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

// ---- device memory ----------------------------------------------------------------
int Ctx::alloc(DevBuf &b, int64_t bytes, const char *what, bool cached) {
  if (bytes <= 0) bytes = 256;
  if (faults.alloc_fails()) return fail(RPA_E_NOMEM, "%s: allocation failure injected by RPA_FAULT", what);
  int64_t held = 0;
  if (!mem.charge(bytes, cached, &held))
    return fail(RPA_E_NOMEM, "%s: %lld bytes requested, %lld of %lld in use or reserved", what, (long long)bytes,
                (long long)held, (long long)mem.limit());
  hipError_t e = hipMalloc(&b.p, (size_t)bytes);
  if (e == hipSuccess && poison) {
    // a fill kernel on the legacy stream, waited for here: nothing else knows this buffer yet
    e = launch_poison_fill(nullptr, b.p, bytes);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
      (void)hipFree(b.p);
      mem.refund(bytes, cached);
      b.p = nullptr;
      return fail(RPA_E_DEVICE, "%s: poison fill failed: %s", what, hipGetErrorString(e));
    }
  }
  if (e != hipSuccess) {
    mem.refund(bytes, cached);
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? RPA_E_NOMEM : RPA_E_DEVICE, "%s: hipMalloc(%lld) failed: %s",
                what, (long long)bytes, hipGetErrorString(e));
  }
  b.bytes = bytes;
  b.cached = cached;
  return RPA_OK;
}

void Ctx::release(DevBuf &b) {
  if (!b.p) return;
  (void)hipFree(b.p);
  mem.refund(b.bytes, b.cached);
  b.p = nullptr;
  b.bytes = 0;
  b.cached = false;
}

int Ctx::workspace(const char *name, int64_t bytes, void **out) {
  DevBuf &b = cache[name];
  if (b.p && b.bytes >= bytes) {
    *out = b.p;
    return RPA_OK;
  }
  if (b.p) {
    RPA_HIP(hipStreamSynchronize(stream));
    release(b);
  }
  RPA_TRY(alloc(b, bytes, name, true));
  *out = b.p;
  return RPA_OK;
}

hipStream_t Ctx::aux_stream() {
  if (!aux && hipStreamCreateWithFlags(&aux, hipStreamNonBlocking) != hipSuccess) aux = nullptr;
  return aux;
}

void Ctx::free_cache() {
  for (auto &kv : cache) release(kv.second);
  cache.clear();
}

int Ctx::prof_begin(hipStream_t s, int k) {
  if (!profile) return RPA_OK;
  hipEvent_t a, b;
  RPA_HIP(hipEventCreate(&a));
  RPA_HIP(hipEventCreate(&b));
  RPA_HIP(hipEventRecord(a, s));
  prof_pending.push_back({k, {a, b}});
  return RPA_OK;
}

int Ctx::prof_end(hipStream_t s) {
  if (!profile || prof_pending.empty()) return RPA_OK;
  RPA_HIP(hipEventRecord(prof_pending.back().second.second, s));
  return RPA_OK;
}

int Ctx::prof_collect() {
  for (auto &p : prof_pending) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, p.second.first, p.second.second);
    if (e == hipSuccess) {
      prof_ms[p.first] += ms;
      prof_launches[p.first] += 1;
    }
    (void)hipEventDestroy(p.second.first);
    (void)hipEventDestroy(p.second.second);
  }
  prof_pending.clear();
  return RPA_OK;
}

// ---- validation -----------------------------------------------------------------
namespace {
int copy_in(void *dst, const void *src, size_t bytes, int memspace) {
  if (memspace == RPA_MEM_HOST) {
    memcpy(dst, src, bytes);
    return RPA_OK;
  }
  RPA_HIP(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
  return RPA_OK;
}
}  // namespace

int validate_freq(const rpa_freq *f) {
  if (!f) return fail(RPA_E_ARG, "freq is NULL");
  if (f->nw < 1 || f->nw > 4096) return fail(RPA_E_ARG, "nw = %d out of range [1, 4096]", f->nw);
  if (!f->omega || !f->weight) return fail(RPA_E_ARG, "freq arrays are NULL");
  for (int j = 0; j < f->nw; ++j)
    if (!std::isfinite(f->omega[j]) || !std::isfinite(f->weight[j]) || f->omega[j] < 0.0)
      return fail(RPA_E_ARG, "frequency node %d is not a finite non-negative value", j);
  return RPA_OK;
}

int validate_system(const rpa_system *sys, HostSmall &hs) {
  if (!sys) return fail(RPA_E_ARG, "system is NULL");
  if (sys->memspace != RPA_MEM_HOST && sys->memspace != RPA_MEM_DEVICE)
    return fail(RPA_E_ARG, "memspace %d is neither host nor device", sys->memspace);
  if (sys->nk < 1 || sys->nq < 1 || sys->nocc < 1 || sys->nvirt < 1 || sys->naux < 1)
    return fail(RPA_E_ARG, "sizes must be >= 1 (nk %d nq %d nocc %d nvirt %d naux %d)", sys->nk,
                sys->nq, sys->nocc, sys->nvirt, sys->naux);
  if (sys->naux > 16384) return fail(RPA_E_ARG, "naux %d above the supported 16384", sys->naux);
  const int64_t M = (int64_t)sys->nk * sys->nocc * sys->nvirt;
  if (M > ((int64_t)1 << 31) - 64) return fail(RPA_E_ARG, "nk*nocc*nvirt = %lld too large", (long long)M);
  if (sys->is_complex != 0 && sys->is_complex != 1) return fail(RPA_E_ARG, "is_complex must be 0 or 1");
  if (!sys->kq || !sys->eps_occ || !sys->eps_virt || !sys->vhalf)
    return fail(RPA_E_ARG, "kq, eps_occ, eps_virt and vhalf must be non-NULL");
  if (!sys->B && !(sys->sigma > 0.0 && std::isfinite(sys->sigma)))
    return fail(RPA_E_ARG, "B is NULL (Philox) but sigma = %g is not positive", sys->sigma);
  hs.nk = sys->nk; hs.nq = sys->nq; hs.nocc = sys->nocc; hs.nvirt = sys->nvirt; hs.naux = sys->naux;
  hs.is_complex = sys->is_complex;
  if (sys->nk_occ < 0 || sys->nk_occ > (1 << 24))
    return fail(RPA_E_ARG, "nk_occ %d outside [0, 2^24]", sys->nk_occ);
  const int32_t nk_occ = sys->nk_occ > 0 ? sys->nk_occ : sys->nk;
  hs.kq.resize((size_t)sys->nq * sys->nk);
  hs.eps_occ.resize((size_t)nk_occ * sys->nocc);
  hs.eps_virt.resize((size_t)sys->nk * sys->nvirt);
  RPA_TRY(copy_in(hs.kq.data(), sys->kq, hs.kq.size() * 4, sys->memspace));
  RPA_TRY(copy_in(hs.eps_occ.data(), sys->eps_occ, hs.eps_occ.size() * 8, sys->memspace));
  RPA_TRY(copy_in(hs.eps_virt.data(), sys->eps_virt, hs.eps_virt.size() * 8, sys->memspace));
  hs.zeta_k.assign(sys->nk, 1.0 / sys->nk);
  hs.zeta_q.assign(sys->nq, 1.0 / sys->nq);
  if (sys->zeta_k) RPA_TRY(copy_in(hs.zeta_k.data(), sys->zeta_k, (size_t)sys->nk * 8, sys->memspace));
  if (sys->zeta_q) RPA_TRY(copy_in(hs.zeta_q.data(), sys->zeta_q, (size_t)sys->nq * 8, sys->memspace));
  for (size_t i = 0; i < hs.kq.size(); ++i)
    if (hs.kq[i] < 0 || hs.kq[i] >= nk_occ)
      return fail(RPA_E_ARG, "kq[%zu] = %d outside [0, nk_occ = %d)", i, hs.kq[i], nk_occ);
  for (double v : hs.eps_occ) if (!std::isfinite(v)) return fail(RPA_E_ARG, "eps_occ not finite");
  for (double v : hs.eps_virt) if (!std::isfinite(v)) return fail(RPA_E_ARG, "eps_virt not finite");
  for (double v : hs.zeta_k) if (!std::isfinite(v)) return fail(RPA_E_ARG, "zeta_k not finite");
  for (double v : hs.zeta_q) if (!std::isfinite(v)) return fail(RPA_E_ARG, "zeta_q not finite");
  hs.nbas = 0;
  hs.c_occ.clear();
  hs.c_virt.clear();
  if (sys->nbas != 0) {
    if (sys->nbas < 1 || sys->nbas > 4096) return fail(RPA_E_ARG, "nbas %d outside [1, 4096]", sys->nbas);
    if (!sys->is_complex) return fail(RPA_E_ARG, "atomic-orbital systems must be complex");
    if (sys->B) return fail(RPA_E_ARG, "an atomic-orbital system builds B itself: B must be NULL");
    if (!sys->c_occ || !sys->c_virt) return fail(RPA_E_ARG, "c_occ and c_virt must be non-NULL when nbas > 0");
    hs.nbas = sys->nbas;
    hs.c_occ.resize((size_t)nk_occ * sys->nbas * sys->nocc * 2);
    hs.c_virt.resize((size_t)sys->nk * sys->nbas * sys->nvirt * 2);
    RPA_TRY(copy_in(hs.c_occ.data(), sys->c_occ, hs.c_occ.size() * 8, sys->memspace));
    RPA_TRY(copy_in(hs.c_virt.data(), sys->c_virt, hs.c_virt.size() * 8, sys->memspace));
    for (double v : hs.c_occ) if (!std::isfinite(v)) return fail(RPA_E_ARG, "c_occ not finite");
    for (double v : hs.c_virt) if (!std::isfinite(v)) return fail(RPA_E_ARG, "c_virt not finite");
    hs.S.clear();
    hs.eps_d = 0.0;
    if (sys->S_ao) {
      // raw coefficients: the projector of Sec. 2.3 runs on the device
      if (nk_occ != sys->nk)
        return fail(RPA_E_ARG, "the device projector takes regular grids (nk_occ = nk); project dual-grid coefficients first");
      if (sys->nbas > 1024) return fail(RPA_E_ARG, "the device projector takes nbas <= 1024 (nbas %d)", sys->nbas);
      if (!(sys->eps_d >= 0.0) || !std::isfinite(sys->eps_d)) return fail(RPA_E_ARG, "eps_d must be finite and >= 0");
      hs.eps_d = sys->eps_d;
      hs.S.resize((size_t)sys->nk * sys->nbas * sys->nbas * 2);
      RPA_TRY(copy_in(hs.S.data(), sys->S_ao, hs.S.size() * 8, sys->memspace));
      for (double v : hs.S) if (!std::isfinite(v)) return fail(RPA_E_ARG, "S_ao not finite");
    }
  }
  // insulators only (closed-shell occupations 2/0): every transition energy positive
  double min_occ_gap = INFINITY;
  for (int q = 0; q < sys->nq; ++q)
    for (int k = 0; k < sys->nk; ++k) {
      const int kq = hs.kq[(size_t)q * sys->nk + k];
      double emax_occ = -INFINITY, emin_virt = INFINITY;
      for (int i = 0; i < sys->nocc; ++i) emax_occ = std::max(emax_occ, hs.eps_occ[(size_t)kq * sys->nocc + i]);
      for (int a = 0; a < sys->nvirt; ++a) emin_virt = std::min(emin_virt, hs.eps_virt[(size_t)k * sys->nvirt + a]);
      min_occ_gap = std::min(min_occ_gap, emin_virt - emax_occ);
    }
  if (!(min_occ_gap > 0.0))
    return fail(RPA_E_ARG, "smallest transition energy %g <= 0: only insulators are supported", min_occ_gap);
  return RPA_OK;
}

// ---- atomic-orbital coefficients ------------------------------------------------------
int64_t ao_stage_scratch_bytes(const HostSmall &hs) {
  if (hs.nbas <= 0 || hs.S.empty()) return 256;
  const int64_t nn = (int64_t)hs.nbas * hs.nbas;
  // S, T, the raw coefficients and the projector's own scratch
  return (int64_t)hs.nk * nn * 16 * 2 + (int64_t)(hs.c_occ.size() + hs.c_virt.size()) * 8 +
         projector_scratch_bytes(hs.nk, hs.nbas) + 1024;
}

int stage_ao_coefficients(hipStream_t st, const HostSmall &hs, double2 *d_cocc, double2 *d_cvirt, void *scratch) {
  if (hs.S.empty()) {
    RPA_HIP(hipMemcpyAsync(d_cocc, hs.c_occ.data(), hs.c_occ.size() * 8, hipMemcpyHostToDevice, st));
    RPA_HIP(hipMemcpyAsync(d_cvirt, hs.c_virt.data(), hs.c_virt.size() * 8, hipMemcpyHostToDevice, st));
    return RPA_OK;
  }
  const int64_t nn = (int64_t)hs.nbas * hs.nbas;
  char *p = (char *)scratch;
  double2 *S = (double2 *)p;
  p += hs.nk * nn * 16;
  double2 *T = (double2 *)p;
  p += hs.nk * nn * 16;
  double2 *raw_o = (double2 *)p;
  p += (int64_t)hs.c_occ.size() * 8;
  double2 *raw_v = (double2 *)p;
  p += (int64_t)hs.c_virt.size() * 8;
  void *pscr = (void *)(((uintptr_t)p + 255) / 256 * 256);
  RPA_HIP(hipMemcpyAsync(S, hs.S.data(), hs.S.size() * 8, hipMemcpyHostToDevice, st));
  RPA_HIP(hipMemcpyAsync(raw_o, hs.c_occ.data(), hs.c_occ.size() * 8, hipMemcpyHostToDevice, st));
  RPA_HIP(hipMemcpyAsync(raw_v, hs.c_virt.data(), hs.c_virt.size() * 8, hipMemcpyHostToDevice, st));
  RPA_HIP(launch_projector(st, S, hs.nk, hs.nbas, hs.eps_d, pscr, T));
  RPA_HIP(launch_project_coeff(st, T, raw_o, hs.nk, hs.nbas, hs.nocc, d_cocc));
  RPA_HIP(launch_project_coeff(st, T, raw_v, hs.nk, hs.nbas, hs.nvirt, d_cvirt));
  return RPA_OK;
}

// ---- the point pipeline -------------------------------------------------------------
// Lanes of a synchronous call: 1 by default, RPA_LANES=2 for two.  Two lanes measured
// +1.7% (FP64) and +4.4% (split-BF16) points/s on the 3x3x1 N_aux 384 slab, but their
// contractions overlap each other, so per-kernel event times no longer isolate a kernel.
int lanes_wanted() {
  const char *e = getenv("RPA_LANES");
  return (e && atoi(e) == 2) ? 2 : 1;
}

bool trln_single() {
  // read at every call, so that a process can switch between the two factorisations
  const char *e = getenv("RPA_TRLN_SINGLE");
  return e && atoi(e) != 0;
}

namespace {

struct Arena {
  // All device buffers of one run_points() call come from a single slab: planned first,
  // then allocated at once.  In cache mode the slab is the context's grow-only
  // "pipeline" workspace; when it has to grow, every cached buffer is released first, so
  // the call never holds more than its own plan plus what other users hold.
  Ctx &ctx;
  bool use_cache;
  DevBuf owned;
  std::vector<std::pair<int64_t, void **>> reqs;
  int64_t total = 0;
  Arena(Ctx &c, bool cache) : ctx(c), use_cache(cache) {}
  ~Arena() { ctx.release(owned); }
  void plan(int64_t bytes, void **out) {
    reqs.push_back({total, out});
    total += (std::max<int64_t>(bytes, 1) + 255) / 256 * 256;
  }
  int commit(hipStream_t st) {
    void *base;
    if (use_cache) {
      DevBuf &b = ctx.cache["pipeline"];
      if (!b.p || b.bytes < total) {
        RPA_HIP(hipStreamSynchronize(st));
        ctx.free_cache();
        RPA_TRY(ctx.alloc(ctx.cache["pipeline"], total, "pipeline workspace", true));
      }
      base = ctx.cache["pipeline"].p;
    } else {
      RPA_TRY(ctx.alloc(owned, total, "job workspace"));
      base = owned.p;
    }
    for (auto &r : reqs) *r.second = (char *)base + r.first;
    return RPA_OK;
  }
};

}  // namespace

int run_points(Ctx &ctx, hipStream_t st, PointJob &job, int64_t budget, bool use_cache) {
  const rpa_system *sys = job.sys;
  const HostSmall &hs = *job.hs;
  const int N = hs.naux;
  const int64_t M = (int64_t)hs.nk * hs.nocc * hs.nvirt;
  const bool cplx = hs.is_complex != 0;
  const int64_t npts = (int64_t)job.pq.size();
  job.eps.assign((size_t)npts, 0.0);
  if (npts == 0) return RPA_OK;
  const bool mixed = job.prec != RPA_FP64;

  const int64_t nn = (int64_t)N * N;
  const int64_t belem = cplx ? 16 : 8;
  const bool b_direct = sys->B && sys->memspace == RPA_MEM_DEVICE;
  const bool vh_direct = sys->memspace == RPA_MEM_DEVICE && cplx;
  const int64_t vh_slot = vh_direct ? 0 : nn * 16;
  // split-BF16 and split-FP16 keep a prepared (split, padded) copy of each B slab instead
  // of the FP32 copy of the FP32 path, plus per point in flight a prepared right operand
  // and the partial tiles of the row splits; fp16 operands carry power-of-two scales (one
  // per B slot, one per point)
  const bool bsplit = job.prec == RPA_BF16X3 || job.prec == RPA_F16X3;
  const bool f16 = job.prec == RPA_F16X3;
  const int64_t f16_slot = f16 ? (f16_absmax_scratch_doubles(1) + 1) * 8 : 0;   // slab maxima and scale
  const int nov = hs.nocc * hs.nvirt;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx.device) != hipSuccess) ncu = 256;
  // Sizes that follow the rows of one B slot: a whole q (kc = nk k-points), or, when one q
  // does not fit the budget, a chunk of kc k-points: the q is then streamed chunk by
  // chunk (B of each chunk generated or copied into the slot, contracted for every point
  // of the batch, and the chunks' chi0 added in chunk order).
  int kc = hs.nk;
  int64_t Mc = M, b_slot = 0, prep_bytes = 0, b32_slot = 0, per_pt = 0, diag_scratch = 0;
  auto set_rows = [&](int k) {
    kc = k;
    Mc = (int64_t)k * nov;
    b_slot = b_direct ? 0 : Mc * N * belem;
    prep_bytes = bsplit ? bf16_prepared_elems(Mc, N) * 2 : 0;
    b32_slot = bsplit ? prep_bytes : mixed ? Mc * N * 8 : 0;   // the slots' stride in d_B32
    per_pt = 2 * nn * 16 + Mc * 8 + (mixed ? (int64_t)N * 8 : 0) + trln_blocked_scratch_bytes(1) + 64;
    diag_scratch = bsplit ? bf16_diag_scratch_doubles(Mc, N) * 8 : mixed ? diag_exact_scratch_doubles(Mc, N, 16) * 8 : 0;
  };
  set_rows(hs.nk);
  auto bsplit_bytes = [&](int64_t r) -> int64_t {
    if (!bsplit || r <= 0) return 0;
    Bf16Plan pl;
    bf16_plan(Mc, N, (int)r, ncu, 0, 128, &pl);
    return r * (prep_bytes + f16_slot) + bf16_partial_elems(pl, (int)r) * 8 + 512;
  };
  // atomic-orbital systems: the projected coefficients and the transform's scratch
  const int64_t ao_bytes = hs.nbas > 0 ? (int64_t)(hs.c_occ.size() + hs.c_virt.size()) * 8 + 512 +
                                             ao_scratch_bytes(hs.nbas, hs.nocc, hs.naux) + ao_stage_scratch_bytes(hs)
                                       : 0;
  const int64_t small = (int64_t)(hs.eps_occ.size() + hs.eps_virt.size() + hs.zeta_k.size()) * 8 +
                        (int64_t)hs.kq.size() * 4 + npts * 32 + 4096 + ao_bytes;

  // distinct q's in order of first appearance; points grouped by q
  std::vector<int32_t> qs;
  std::vector<std::vector<int64_t>> by_q(hs.nq);
  for (int64_t p = 0; p < npts; ++p) {
    const int q = job.pq[(size_t)p];
    if (q < 0 || q >= hs.nq) return fail(RPA_E_ARG, "point %lld: q = %d outside [0, nq)", (long long)p, q);
    if (!std::isfinite(job.pw[(size_t)p]) || job.pw[(size_t)p] < 0.0)
      return fail(RPA_E_ARG, "point %lld: omega is not finite and non-negative", (long long)p);
    if (by_q[q].empty()) qs.push_back(q);
    by_q[q].push_back(p);
  }

  // q-group size and point batch under the budget.  With two lanes (RPA_LANES=2) a
  // synchronous call runs its batches alternately on the context's stream and a second
  // one, with separate batch buffers, so one batch's sandwich and Cholesky overlap the
  // other's contraction.
  int64_t avail = budget - small;
  int gq = (int)qs.size();
  if (job.max_q_group > 0) gq = std::min(gq, job.max_q_group);
  auto pts_of = [&](int g0, int g) {
    int64_t c = 0;
    for (int i = g0; i < g0 + g && i < (int)qs.size(); ++i) c += (int64_t)by_q[qs[i]].size();
    return c;
  };
  // fixed per-lane buffers: one point's split-BF16 operands and the exact-diagonal scratch
  int64_t one_split = 0;
  int nlanes = (use_cache && lanes_wanted() > 1 && npts >= 8) ? 2 : 1;
  hipStream_t lane_st[2] = {st, nullptr};
  if (nlanes == 2) {
    lane_st[1] = ctx.aux_stream();
    if (!lane_st[1]) nlanes = 1;
  }
  int64_t rest = 0, pbatch = 0, rbatch = 0;
  for (;;) {
    one_split = bsplit_bytes(1) + diag_scratch;
    const int64_t lane_min = nlanes * (per_pt + one_split);
    gq = (int)qs.size();
    if (job.max_q_group > 0) gq = std::min(gq, job.max_q_group);
    if (kc < hs.nk) gq = 1;
    // device bytes per q slot: B, V^(1/2), the reduced-precision copy and the fp16
    // operand's maxima and scale
    const int64_t per_slot = b_slot + vh_slot + b32_slot + f16_slot;
    while (gq > 1 && gq * per_slot + nlanes * std::min<int64_t>(pts_of(0, gq), 256) * per_pt +
                         nlanes * one_split > avail)
      --gq;
    rest = avail - gq * per_slot;
    if (rest < lane_min && nlanes == 2) {
      nlanes = 1;
      continue;
    }
    if (rest < lane_min && kc > 1) {
      // one q does not fit: stream it in chunks of fewer k-points (one lane: the lanes
      // would share the chunk slot)
      set_rows((kc + 1) / 2);
      nlanes = 1;
      continue;
    }
    if (rest < lane_min)
      return fail(RPA_E_NOMEM, "one k-point of one q of this system needs %lld bytes, budget is %lld",
                  (long long)(per_slot + per_pt + one_split + small), (long long)budget);
    const int64_t pb_cap = (rest / nlanes - one_split) / per_pt;
    int64_t max_group_pts = 0;
    for (size_t g0 = 0; g0 < qs.size(); g0 += gq) max_group_pts = std::max(max_group_pts, pts_of((int)g0, gq));
    // at most 16384 points per batch: the point index is a grid dimension of the kernels
    pbatch = std::min<int64_t>({pb_cap, (max_group_pts + nlanes - 1) / nlanes, (int64_t)16384});
    // points per split-BF16 sub-launch: as many as the rest of the budget holds
    // (a synchronous call takes one launch for a whole batch where memory allows: fewer
    // row splits, so less partial traffic, and each B slab is read once per run of its
    // points; a served job keeps launches of at most 16 points, which the fuser can merge
    // with other jobs' and which let concurrent jobs interleave)
    rbatch = bsplit ? std::min<int64_t>(pbatch, use_cache ? 128 : 16) : 0;
    while (rbatch > 1 && pbatch * per_pt + bsplit_bytes(rbatch) + diag_scratch > rest / nlanes) rbatch = rbatch * 3 / 4;
    if (bsplit && rbatch < 1) rbatch = 1;
    break;
  }
  // FP64 and FP32: two more partial planes per lane (up to four row splits per launch)
  // where the budget holds them; one plane (two splits) otherwise.  A streamed q keeps
  // each later chunk's chi0 in the first plane before adding it in.
  const int tplanes = (!bsplit && pbatch * per_pt + one_split + 2 * pbatch * nn * 16 <= rest / nlanes) ? kBatchSplits - 1 : 1;
  const bool streamed = kc < hs.nk;
  const int nchunks = (hs.nk + kc - 1) / kc;
  const int max_split = streamed ? tplanes : tplanes + 1;

  Arena ar(ctx, use_cache);
  const bool prof = use_cache && ctx.profile;   // timing only on the synchronous path
  double *d_eo, *d_ev, *d_zk, *d_eps;
  int32_t *d_kq, *d_info;
  void *d_B = nullptr, *d_vh = nullptr, *d_vstage = nullptr;
  ar.plan((int64_t)hs.eps_occ.size() * 8, (void **)&d_eo);
  ar.plan((int64_t)hs.eps_virt.size() * 8, (void **)&d_ev);
  ar.plan((int64_t)hs.zeta_k.size() * 8, (void **)&d_zk);
  ar.plan((int64_t)hs.kq.size() * 4, (void **)&d_kq);
  ar.plan(npts * 8, (void **)&d_eps);
  ar.plan(npts * 4, (void **)&d_info);
  double2 *d_cocc = nullptr, *d_cvirt = nullptr;
  void *d_aoscr = nullptr, *d_aostage = nullptr;
  if (hs.nbas > 0) {
    ar.plan((int64_t)hs.c_occ.size() * 8, (void **)&d_cocc);
    ar.plan((int64_t)hs.c_virt.size() * 8, (void **)&d_cvirt);
    ar.plan(ao_stage_scratch_bytes(hs), &d_aostage);
    ar.plan(ao_scratch_bytes(hs.nbas, hs.nocc, hs.naux), &d_aoscr);
  }
  if (b_slot) ar.plan(gq * b_slot, &d_B);
  if (vh_slot) ar.plan(gq * vh_slot, &d_vh);
  if (vh_slot && !cplx && sys->memspace == RPA_MEM_HOST) ar.plan(nn * 8, &d_vstage);
  float2 *d_B32 = nullptr;
  if (mixed) ar.plan(gq * b32_slot, (void **)&d_B32);
  Bf16Plan rplan{};
  int bf16_tn = 0;   // split-BF16 tile edge, chosen on the first contraction
  if (bsplit) bf16_plan(Mc, N, (int)rbatch, ncu, 0, 128, &rplan);
  double *d_bpart = nullptr, *d_lscale = nullptr;   // fp16: slab maxima and scales per slot
  if (f16) {
    ar.plan(f16_absmax_scratch_doubles(gq) * 8, (void **)&d_bpart);
    ar.plan((int64_t)gq * 8, (void **)&d_lscale);
  }
  // per-lane batch buffers
  struct LaneBufs {
    PointDesc *pts = nullptr;
    int32_t *amap = nullptr;
    void *chi = nullptr, *T = nullptr, *tscr = nullptr;
    double *w = nullptr, *diag = nullptr, *dscr = nullptr;
    unsigned short *R = nullptr;
    float2 *part = nullptr;
    double *wpart = nullptr, *rscale = nullptr;   // fp16: weight maxima and scales per point
  } lanes[2];
  for (int l = 0; l < nlanes; ++l) {
    LaneBufs &lb = lanes[l];
    ar.plan(pbatch * (int64_t)sizeof(PointDesc), (void **)&lb.pts);
    ar.plan(5 * pbatch * 4, (void **)&lb.amap);   // three maps and the pair table
    ar.plan(pbatch * nn * 16, &lb.chi);
    ar.plan(pbatch * M * 8, (void **)&lb.w);
    if (mixed) {
      ar.plan(pbatch * N * 8, (void **)&lb.diag);
      ar.plan(diag_scratch, (void **)&lb.dscr);
    }
    if (bsplit) {
      ar.plan(rbatch * prep_bytes, (void **)&lb.R);
      ar.plan(bf16_partial_elems(rplan, (int)rbatch) * 8, (void **)&lb.part);
    }
    if (f16) {
      ar.plan(f16_absmax_scratch_doubles((int)rbatch) * 8, (void **)&lb.wpart);
      ar.plan(rbatch * 8, (void **)&lb.rscale);
    }
    ar.plan(pbatch * nn * 16 * tplanes, &lb.T);
    ar.plan(trln_blocked_scratch_bytes((int32_t)pbatch), &lb.tscr);
  }
  double *d_qw = nullptr;
  ar.plan((int64_t)(hs.nq + 4097) * 8, (void **)&d_qw);
  RPA_TRY(ar.commit(st));
  const bool single_wg_trln = trln_single();
  // lane events: staging done (lane 1 waits), lane 1 finished (the caller's stream waits)
  struct Events {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  if (nlanes == 2) {
    RPA_HIP(hipEventCreateWithFlags(&ev.e[0], hipEventDisableTiming));
    RPA_HIP(hipEventCreateWithFlags(&ev.e[1], hipEventDisableTiming));
  }

  RPA_HIP(hipMemcpyAsync(d_eo, hs.eps_occ.data(), hs.eps_occ.size() * 8, hipMemcpyHostToDevice, st));
  RPA_HIP(hipMemcpyAsync(d_ev, hs.eps_virt.data(), hs.eps_virt.size() * 8, hipMemcpyHostToDevice, st));
  RPA_HIP(hipMemcpyAsync(d_zk, hs.zeta_k.data(), hs.zeta_k.size() * 8, hipMemcpyHostToDevice, st));
  RPA_HIP(hipMemcpyAsync(d_kq, hs.kq.data(), hs.kq.size() * 4, hipMemcpyHostToDevice, st));
  if (hs.nbas > 0) {
    RPA_TRY(stage_ao_coefficients(st, hs, d_cocc, d_cvirt, d_aostage));
  }

  // B rows of the k-points [k0, k1) of q into slot s on stream S: generated (Philox, or
  // the MO transform of an atomic-orbital system), or copied from the caller's host B; then
  // the slot's reduced-precision copy (FP32, or the prepared split operand with its scale)
  auto stage_b = [&](hipStream_t S, int s, int q, int k0, int k1) -> int {
    const int64_t rows = (int64_t)(k1 - k0) * nov;
    const int64_t off = ((int64_t)q * M + (int64_t)k0 * nov) * N * belem;   // in a caller's B
    const char *src;
    if (!b_direct) {
      char *dst = (char *)d_B + (int64_t)s * b_slot;
      if (!sys->B) {
        if (prof) RPA_TRY(ctx.prof_begin(S, RPA_K_PHILOX));
        if (hs.nbas > 0) {
          // the MO transform of the pair-fit coefficients, one k block at a time
          const int64_t cstride = (int64_t)hs.nbas * hs.nocc, vstride = (int64_t)hs.nbas * hs.nvirt;
          const int64_t per_k = (int64_t)nov * N;
          for (int ik = k0; ik < k1; ++ik)
            RPA_HIP(launch_ao_B(S, sys->philox_seed, sys->sigma, hs.nk, q, ik, hs.nbas, hs.nocc, hs.nvirt, N,
                                d_cocc + (int64_t)hs.kq[(size_t)q * hs.nk + ik] * cstride,
                                d_cvirt + (int64_t)ik * vstride, d_aoscr,
                                reinterpret_cast<double2 *>(dst) + (int64_t)(ik - k0) * per_k));
        } else {
          RPA_HIP(launch_philox_B(S, sys->philox_seed, sys->sigma, hs.nk, q, k0, k1, hs.nocc, hs.nvirt, N, cplx,
                                  dst));
        }
        if (prof) RPA_TRY(ctx.prof_end(S));
      } else {
        RPA_HIP(hipMemcpyAsync(dst, (const char *)sys->B + off, (size_t)(rows * N * belem), hipMemcpyHostToDevice, S));
      }
      src = dst;
    } else {
      src = (const char *)sys->B + off;
    }
    if (mixed) {
      if (prof) RPA_TRY(ctx.prof_begin(S, RPA_K_CHI0_AUX));
      if (f16) {
        // the slab's largest |Re|, |Im| and from it the left operand's scale
        double *bp = d_bpart + f16_absmax_scratch_doubles(1) * s;
        RPA_HIP(launch_absmax_blocks(S, (const double *)src, rows * N * (cplx ? 2 : 1), 0, 1, bp));
        RPA_HIP(launch_f16_scales(S, bp, nullptr, nullptr, 1, d_lscale + s));
      }
      if (bsplit)
        RPA_HIP(launch_bf16_prepare(S, src, cplx, rows, N, nullptr, 1,
                                    (unsigned short *)((char *)d_B32 + (int64_t)s * b32_slot), nullptr, nullptr,
                                    f16 ? d_lscale + s : nullptr, f16));
      else
        RPA_HIP(launch_to_f32(S, src, d_B32 + (int64_t)s * Mc * N, rows * N, cplx));
      if (prof) RPA_TRY(ctx.prof_end(S));
    }
    return RPA_OK;
  };

  // host copies of every batch's descriptors stay alive until the final synchronisation
  std::deque<std::vector<PointDesc>> keep_pts;
  std::deque<std::vector<int32_t>> keep_maps;
  int64_t batch_no = 0;
  for (size_t g0 = 0; g0 < qs.size(); g0 += (size_t)gq) {
    const int ng = (int)std::min<size_t>((size_t)gq, qs.size() - g0);
    if (g0 > 0) {   // slots are reused by this group
      RPA_HIP(hipStreamSynchronize(st));
      if (nlanes == 2) RPA_HIP(hipStreamSynchronize(lane_st[1]));
    }
    // stage B (whole q's; streamed q's chunk by chunk below) and V^(1/2) of the group's
    // q's into slots
    for (int s = 0; s < ng; ++s) {
      const int q = qs[g0 + s];
      if (!streamed) RPA_TRY(stage_b(st, s, q, 0, hs.nk));
      if (vh_slot) {
        double2 *dst = (double2 *)((char *)d_vh + (int64_t)s * vh_slot);
        if (cplx) {
          RPA_HIP(hipMemcpyAsync(dst, (const char *)sys->vhalf + (int64_t)q * nn * 16, (size_t)(nn * 16),
                                 hipMemcpyHostToDevice, st));
        } else if (sys->memspace == RPA_MEM_HOST) {
          RPA_HIP(hipMemcpyAsync(d_vstage, (const char *)sys->vhalf + (int64_t)q * nn * 8, (size_t)(nn * 8),
                                 hipMemcpyHostToDevice, st));
          RPA_HIP(launch_widen(st, (const double *)d_vstage, dst, nn));
        } else {
          RPA_HIP(launch_widen(st, (const double *)sys->vhalf + (int64_t)q * nn, dst, nn));
        }
      }
    }
    if (nlanes == 2) {
      RPA_HIP(hipEventRecord(ev.e[0], st));
      RPA_HIP(hipStreamWaitEvent(lane_st[1], ev.e[0], 0));
    }
    // the group's points in batches, alternating between the lanes
    std::vector<int64_t> gp;
    std::vector<int> gslot;
    for (int s = 0; s < ng; ++s)
      for (int64_t p : by_q[qs[g0 + s]]) {
        gp.push_back(p);
        gslot.push_back(s);
      }
    for (size_t b0 = 0; b0 < gp.size(); b0 += (size_t)pbatch, ++batch_no) {
      const int lane = (int)(batch_no % nlanes);
      hipStream_t S = lane_st[lane];
      LaneBufs &lb = lanes[lane];
      const int nb = (int)std::min<size_t>((size_t)pbatch, gp.size() - b0);
      keep_pts.emplace_back(nb);
      keep_maps.emplace_back(5 * (size_t)nb);
      std::vector<PointDesc> &hp = keep_pts.back();
      int32_t *vmap = keep_maps.back().data();      // V^(1/2) slot of each batch entry
      int32_t *imap = vmap + nb;                     // identity (chi0 / T slot)
      int32_t *emap = vmap + 2 * nb;                 // output position of each batch entry
      for (int i = 0; i < nb; ++i) {
        const int64_t p = gp[b0 + i];
        const int s = gslot[b0 + i];
        const int q = job.pq[(size_t)p];
        hp[i].q = q;
        // the FP64 contraction reads a caller's device B by q and staged slabs by slot;
        // the reduced-precision contraction always reads the slot's FP32 copy
        hp[i].bslot = (b_direct && !mixed) ? q : s;
        hp[i].omega = job.pw[(size_t)p];
        vmap[i] = vh_direct ? q : s;
        imap[i] = i;
        emap[i] = (int32_t)p;
      }
      // consecutive points on one slab (the frequencies of a q) pair up for the paired
      // FP64 contraction kernel
      int32_t *pairs = vmap + 3 * nb;
      int32_t npairs = 0;
      for (int i = 0; i < nb;) {
        const bool two = i + 1 < nb && hp[i + 1].bslot == hp[i].bslot;
        pairs[2 * npairs] = i;
        pairs[2 * npairs + 1] = two ? i + 1 : -1;
        ++npairs;
        i += two ? 2 : 1;
      }
      RPA_HIP(hipMemcpyAsync(lb.pts, hp.data(), nb * sizeof(PointDesc), hipMemcpyHostToDevice, S));
      RPA_HIP(hipMemcpyAsync(lb.amap, vmap, (3 * (size_t)nb + 2 * (size_t)npairs) * 4, hipMemcpyHostToDevice, S));
      const int32_t *d_vmap = lb.amap, *d_imap = lb.amap + nb, *d_emap = lb.amap + 2 * nb;
      double *d_w = lb.w, *d_diag = lb.diag, *d_dscr = lb.dscr;
      unsigned short *d_R = lb.R;
      float2 *d_part = lb.part;
      void *d_chi = lb.chi, *d_T = lb.T, *d_tscr = lb.tscr;
      PointDesc *d_pts = lb.pts;

      // the contraction, once per chunk of the q's k-points (one chunk unless the q is
      // streamed); chunk c > 0 goes to the first T plane and is added to chi0 in order
      for (int c = 0; c < nchunks; ++c) {
      const int k0 = c * kc, k1 = std::min(hs.nk, k0 + kc);
      const int64_t rows = (int64_t)(k1 - k0) * nov;
      if (streamed) RPA_TRY(stage_b(S, 0, hp[0].q, k0, k1));   // one q per group: slot 0
      void *out_c = c == 0 ? d_chi : d_T;
      // FP64 rows of this chunk that point i of the batch contracts
      auto fp64_rows = [&](int i) -> const char * {
        if (b_direct)
          return (const char *)sys->B + ((int64_t)job.pq[(size_t)gp[b0 + i]] * M + (int64_t)k0 * nov) * N * belem;
        return (const char *)d_B + (int64_t)hp[i].bslot * b_slot;
      };
      Chi0Args ca{};
      // a caller's device B is read in place (the FP64 contraction by q, at the chunk's
      // first row); staged slots, FP32 copies and prepared operands by slot
      ca.B = b_direct ? (const void *)((const char *)sys->B + (int64_t)k0 * nov * N * belem) : d_B;
      ca.b_slot_stride = (b_direct && !mixed) ? M * N : Mc * N;
      ca.eps_occ = d_eo;
      ca.eps_virt = d_ev;
      ca.kq = d_kq;
      ca.zeta_k = d_zk;
      ca.pts = d_pts;
      ca.wtab = d_w;
      ca.out = (double2 *)out_c;
      ca.out_stride = nn;
      ca.nk = hs.nk; ca.nocc = hs.nocc; ca.nvirt = hs.nvirt; ca.N = N; ca.M = rows;
      ca.k0 = k0;
      ca.ksplit = 1;
      ca.partial = (double2 *)d_T + (c == 0 ? 0 : (int64_t)nb * nn);
      ca.pairs = lb.amap + 3 * nb;
      ca.npairs = npairs;
      int cfg = 1;   // FP64 tile configuration (the tuner's choice, made after the weights)
      if (prof) RPA_TRY(ctx.prof_begin(S, RPA_K_CHI0_AUX));
      RPA_HIP(launch_chi0_weights(S, ca, nb));
      // row splits of the contraction (FP64 up to four, reduced precision two) where they
      // fill the last round of workgroups better (counting the workgroups of a concurrent
      // lane); the later splits' results go to the T buffer's planes, which are free
      // until the sandwich.  RPA_CHI0_KSPLIT fixes the count (tests, timing).
      auto pick_split = [&](int64_t tn, int64_t slots, int64_t units, int max_split) {
        const int64_t T = (N + tn - 1) / tn;
        int ks = chi0_pick_ksplit(T * (T + 1) / 2 * units * nlanes, slots, rows, max_split);
        if (const char *e = getenv("RPA_CHI0_KSPLIT")) {
          const int v = atoi(e);
          if (v >= 1) ks = std::min(v, max_split);
        }
        return ks;
      };
      int ks_of[8] = {1, 1, 1, 1, 1, 1, 1, 1};   // FP64: the split count of each configuration
      if (!mixed) {
        for (int c = 0; c < chi0_cfg_count() && c < 8; ++c)
          ks_of[c] = pick_split(chi0_cfg_tile(c), (int64_t)chi0_cfg_slots_per_cu(c) * ncu,
                                chi0_cfg_points_per_wg(c) == 2 ? npairs : nb, max_split);
        RPA_TRY(tune_chi0_cfg(S, ca, nb, cplx, &cfg, ks_of));
      }
      int f32_tile = kF32T64;   // FP32 configuration (64- or 128-wide, or 64-wide paired)
      if (mixed && !bsplit) {
        // the exact FP64 diagonal first: the tile tuner launches the contraction
        int i0 = 0;
        while (i0 < nb) {
          int i1 = i0 + 1;
          while (i1 < nb && hp[i1].bslot == hp[i0].bslot) ++i1;
          RPA_HIP(launch_diag_exact(S, fp64_rows(i0), cplx, rows, N, d_w + (int64_t)i0 * rows, i1 - i0, d_dscr,
                                    d_diag + (int64_t)i0 * N));
          i0 = i1;
        }
        const int f32_cfgs[3] = {kF32T64, kF32T128, kF32T64W2};
        int f32_ks[3];
        for (int c = 0; c < 3; ++c) {
          const int e = f32_cfg_edge(f32_cfgs[c]);
          f32_ks[c] = pick_split(e, (e == 128 ? 1LL : 2LL) * ncu, f32_cfg_points_per_wg(f32_cfgs[c]) == 2 ? npairs : nb,
                                 max_split);
        }
        RPA_TRY(tune_f32_tile(S, ca, nb, cplx, d_B32, d_diag, &f32_tile, f32_ks));
        ca.ksplit = f32_ks[f32_tile == kF32T128 ? 1 : f32_tile == kF32T64W2 ? 2 : 0];
      } else if (bsplit) {
        ca.ksplit = 1;   // the split-BF16 plan makes its own row splits
      } else {
        ca.ksplit = ks_of[cfg];
      }
      if (mixed) {
        // the exact FP64 diagonal: FP32 above, split-BF16 in the operand preparation
        if (bsplit) {
          // sub-launches of up to rbatch points: prepare their right operands (per run of
          // points on one B slab), then contract and reduce
          for (int r0 = 0; r0 < nb; r0 += (int)rbatch) {
            const int r1 = std::min<int>(nb, r0 + (int)rbatch);
            if (f16) {
              // each point's right-operand scale from its slab's maximum and its own
              // largest weight
              RPA_HIP(launch_absmax_blocks(S, d_w + (int64_t)r0 * rows, rows, rows, r1 - r0, lb.wpart));
              RPA_HIP(launch_f16_scales(S, d_bpart, lb.wpart, d_pts + r0, r1 - r0, lb.rscale));
            }
            int i0 = r0;
            while (i0 < r1) {
              int i1 = i0 + 1;
              while (i1 < r1 && hp[i1].bslot == hp[i0].bslot) ++i1;
              RPA_HIP(launch_bf16_prepare(S, fp64_rows(i0), cplx, rows, N, d_w + (int64_t)i0 * rows, i1 - i0,
                                          d_R + (int64_t)(i0 - r0) * (prep_bytes / 2), d_dscr,
                                          d_diag + (int64_t)i0 * N, f16 ? lb.rscale + (i0 - r0) : nullptr, f16));
              i0 = i1;
            }
            const int64_t max_part = bf16_partial_elems(rplan, (int)rbatch);
            if (bf16_tn == 0) {
              // the tile edge of this shape, timed once on the first sub-batch
              Bf16Group tg{};
              tg.L = (const unsigned short *)d_B32;
              tg.l_stride = prep_bytes / 2;
              tg.R = d_R;
              tg.r_stride = prep_bytes / 2;
              tg.pts = d_pts + r0;
              tg.part = d_part;
              tg.npts = r1 - r0;
              tg.f16 = f16;
              RPA_TRY(tune_bf16_tile(S, tg, rows, N, ncu, max_part, cplx, &bf16_tn));
            }
            Bf16Plan pl;
            bf16_plan(rows, N, r1 - r0, ncu, max_part, bf16_tn, &pl);
            Bf16Group grp{};
            grp.L = (const unsigned short *)d_B32;
            grp.l_stride = prep_bytes / 2;
            grp.R = d_R;
            grp.r_stride = prep_bytes / 2;
            grp.pts = d_pts + r0;
            grp.part = d_part;
            grp.pl = pl;
            grp.npts = r1 - r0;
            grp.f16 = f16;
            if (prof) RPA_TRY(ctx.prof_end(S));
            if (prof) RPA_TRY(ctx.prof_begin(S, RPA_K_CHI0));
            RPA_TRY(fused_herk(job.fuser, S, grp, cplx));
            if (prof) RPA_TRY(ctx.prof_end(S));
            if (prof) RPA_TRY(ctx.prof_begin(S, RPA_K_CHI0_AUX));
            RPA_HIP(launch_bf16_reduce(S, pl, d_part, r1 - r0, N, d_diag + (int64_t)r0 * N,
                                       (double2 *)out_c + (int64_t)r0 * nn, nn, d_pts + r0,
                                       f16 ? d_lscale : nullptr, f16 ? lb.rscale : nullptr));
            if (prof) RPA_TRY(ctx.prof_end(S));
            if (prof && r1 < nb) RPA_TRY(ctx.prof_begin(S, RPA_K_CHI0_AUX));
          }
        } else {
          if (prof) RPA_TRY(ctx.prof_end(S));
          if (prof) RPA_TRY(ctx.prof_begin(S, RPA_K_CHI0));
          RPA_TRY(fused_chi0_f32(job.fuser, S, ca, nb, d_B32, d_diag, f32_tile));
        }
      } else {
        if (prof) RPA_TRY(ctx.prof_end(S));
        if (prof) RPA_TRY(ctx.prof_begin(S, RPA_K_CHI0));
        RPA_TRY(fused_chi0_f64(job.fuser, S, ca, nb, cplx, cfg));
      }
      if (prof && !bsplit) RPA_TRY(ctx.prof_end(S));
      if (c > 0) {
        if (prof) RPA_TRY(ctx.prof_begin(S, RPA_K_OTHER));
        RPA_HIP(launch_split_add(S, (const double2 *)d_T, 1, (int64_t)nb * nn, (double2 *)d_chi));
        if (prof) RPA_TRY(ctx.prof_end(S));
      }
      }

      const double2 *vh = vh_direct ? (const double2 *)sys->vhalf : (const double2 *)d_vh;
      GemmArgs g1{};   // T = chi0 V^(1/2)
      g1.A = (const double2 *)d_chi; g1.a_stride = nn; g1.a_map = d_imap; g1.a_div = 1;
      g1.B = vh; g1.b_stride = nn; g1.b_map = d_vmap; g1.b_div = 1;
      g1.C = (double2 *)d_T; g1.c_stride = nn; g1.N = N; g1.lower_only = 0;
      if (prof) RPA_TRY(ctx.prof_begin(S, RPA_K_PI));
      RPA_HIP(launch_zgemm_f64(S, g1, nb));
      GemmArgs g2{};   // Pi = V^(1/2) T, lower triangle, into the chi0 buffer
      g2.A = vh; g2.a_stride = nn; g2.a_map = d_vmap; g2.a_div = 1;
      g2.B = (const double2 *)d_T; g2.b_stride = nn; g2.b_map = d_imap; g2.b_div = 1;
      g2.C = (double2 *)d_chi; g2.c_stride = nn; g2.N = N; g2.lower_only = 1;
      g2.negate = single_wg_trln ? 0 : 1;   // the blocked factorisation takes W = -Pi
      RPA_HIP(launch_zgemm_f64(S, g2, nb));
      if (prof) RPA_TRY(ctx.prof_end(S));
      if (prof) RPA_TRY(ctx.prof_begin(S, RPA_K_TRLN));
      if (single_wg_trln) {
        RPA_HIP(launch_trln_f64(S, (double2 *)d_chi, nn, N, nb, d_eps, d_info, d_emap));
      } else {
        RPA_HIP(launch_trln_blocked(S, (double2 *)d_chi, nn, N, nb, d_eps, d_info, d_emap, d_tscr));
      }
      if (prof) RPA_TRY(ctx.prof_end(S));
    }
  }
  if (nlanes == 2) {   // everything after this point runs on the caller's stream
    RPA_HIP(hipEventRecord(ev.e[1], lane_st[1]));
    RPA_HIP(hipStreamWaitEvent(st, ev.e[1], 0));
  }
  if (job.quadrature) {
    // E = sum_q zeta_q sum_j W_j eps(q, w_j) / (2 pi) over the full q-major grid, on the device
    const int nq = hs.nq, nw = (int)job.weight.size();
    if ((int64_t)nq * nw != npts) return fail(RPA_E_INTERNAL, "quadrature needs the full point grid");
    if (nw > 4096) return fail(RPA_E_ARG, "nw = %d above 4096", nw);
    std::vector<double> &hq = job.qstage;
    hq.assign(hs.zeta_q.begin(), hs.zeta_q.end());
    hq.insert(hq.end(), job.weight.begin(), job.weight.end());
    RPA_HIP(hipMemcpyAsync(d_qw, hq.data(), (size_t)(nq + nw) * 8, hipMemcpyHostToDevice, st));
    if (prof) RPA_TRY(ctx.prof_begin(st, RPA_K_OTHER));
    RPA_HIP(launch_quadrature(st, d_eps, d_qw, d_qw + nq, nq, nw, d_qw + nq + nw));
    if (prof) RPA_TRY(ctx.prof_end(st));
    RPA_HIP(hipMemcpyAsync(&job.E, d_qw + nq + nw, 8, hipMemcpyDeviceToHost, st));
  }
  std::vector<int32_t> info((size_t)npts);
  RPA_HIP(hipMemcpyAsync(job.eps.data(), d_eps, (size_t)npts * 8, hipMemcpyDeviceToHost, st));
  RPA_HIP(hipMemcpyAsync(info.data(), d_info, (size_t)npts * 4, hipMemcpyDeviceToHost, st));
  RPA_HIP(hipStreamSynchronize(st));
  if (prof) RPA_TRY(ctx.prof_collect());
  for (int64_t p = 0; p < npts; ++p)
    if (info[(size_t)p] >= 0)
      return fail(RPA_E_NOTSPD, "1 - Pi is not positive definite at point %lld (q %d, omega %g), column %d",
                  (long long)p, job.pq[(size_t)p], job.pw[(size_t)p], info[(size_t)p]);
  return RPA_OK;
}

}  // namespace rpa
