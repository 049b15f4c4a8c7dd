// extern "C" entry points of librpa (declared in include/rpa.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <new>
#include <vector>

#include "runtime.hpp"
#include "scheduler.hpp"

using namespace rpa;

namespace {

int check_ctx(rpa_ctx *ctx) {
  if (!ctx) return fail(RPA_E_ARG, "ctx is NULL");
  return RPA_OK;
}

int set_device(Ctx &c) {
  RPA_HIP(hipSetDevice(c.device));
  return RPA_OK;
}

// Device bytes a synchronous call may plan with (its own cached workspaces count as
// available; what admitted serving jobs have reserved does not).
int64_t budget_of(Ctx &c) { return c.mem.sync_budget(); }

// Copy `bytes` between a caller array in `memspace` and a device buffer.
int to_device(void *dst, const void *src, size_t bytes, int memspace, hipStream_t s) {
  RPA_HIP(hipMemcpyAsync(dst, src, bytes,
                         memspace == RPA_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
  return RPA_OK;
}
int from_device(void *dst, const void *src, size_t bytes, int memspace, hipStream_t s) {
  RPA_HIP(hipMemcpyAsync(dst, src, bytes,
                         memspace == RPA_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  return RPA_OK;
}

// Stage n*n real or complex caller data as complex on the device (widening real input).
int stage_complex(Ctx &c, const char *name, const void *src, int64_t count, int is_complex,
                  int memspace, double2 **out) {
  void *buf;
  RPA_TRY(c.workspace(name, count * 16, &buf));
  if (is_complex) {
    RPA_TRY(to_device(buf, src, (size_t)count * 16, memspace, c.stream));
  } else {
    void *tmp;
    std::string tname = std::string(name) + "_real";
    RPA_TRY(c.workspace(tname.c_str(), count * 8, &tmp));
    RPA_TRY(to_device(tmp, src, (size_t)count * 8, memspace, c.stream));
    RPA_HIP(launch_widen(c.stream, (const double *)tmp, (double2 *)buf, count));
  }
  *out = (double2 *)buf;
  return RPA_OK;
}

// Write a complex device result to the caller (narrowing to real if needed).
int deliver_complex(Ctx &c, void *dst, const double2 *src, int64_t count, int is_complex, int memspace) {
  if (is_complex) {
    RPA_TRY(from_device(dst, src, (size_t)count * 16, memspace, c.stream));
  } else {
    void *tmp;
    RPA_TRY(c.workspace("deliver_real", count * 8, &tmp));
    RPA_HIP(launch_narrow(c.stream, src, (double *)tmp, count));
    RPA_TRY(from_device(dst, tmp, (size_t)count * 8, memspace, c.stream));
  }
  return RPA_OK;
}

}  // namespace

extern "C" {

int rpa_init(rpa_ctx **out, int device, uint64_t hbm_limit_bytes) {
  if (!out) return fail(RPA_E_ARG, "ctx pointer is NULL");
  *out = nullptr;
  int ndev = 0;
  RPA_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(RPA_E_ARG, "device %d not in [0, %d)", device, ndev);
  RPA_HIP(hipSetDevice(device));
  RPA_TRY(noalloc_setup(device));   // address of the fixed scratch of rpa_chi0_noalloc
  size_t free_b = 0, total_b = 0;
  RPA_HIP(hipMemGetInfo(&free_b, &total_b));
  rpa_ctx *ctx = new (std::nothrow) rpa_ctx();
  if (!ctx) return fail(RPA_E_NOMEM, "host allocation of the context failed");
  Ctx &c = ctx->c;
  c.device = device;
  c.mem.set_limit(hbm_limit_bytes ? (int64_t)hbm_limit_bytes : (int64_t)(0.9 * (double)free_b));
  // debugging modes, read once per context
  const char *fault = getenv("RPA_FAULT");
  if (!c.faults.parse(fault)) {
    delete ctx;
    return fail(RPA_E_ARG, "RPA_FAULT=%s: expected alloc:N[,N2,...] with N >= 1", fault);
  }
  const char *poison = getenv("RPA_POISON");
  c.poison = poison && atoi(poison) != 0;
  hipError_t e = hipStreamCreateWithFlags(&c.own_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete ctx;
    return fail(RPA_E_DEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
  }
  c.stream = c.own_stream;
  c.sched.reset(new Scheduler(c));
  *out = ctx;
  return RPA_OK;
}

int rpa_finalize(rpa_ctx *ctx) {
  RPA_TRY(check_ctx(ctx));
  Ctx &c = ctx->c;
  (void)hipSetDevice(c.device);
  if (c.sched) c.sched->shutdown();
  c.sched.reset();
  {
    std::lock_guard<std::mutex> g(c.mu);
    (void)hipStreamSynchronize(c.stream);
    c.free_cache();
  }
  if (c.own_stream) (void)hipStreamDestroy(c.own_stream);
  if (c.aux) (void)hipStreamDestroy(c.aux);
  delete ctx;
  return RPA_OK;
}

const char *rpa_last_error(const rpa_ctx *) { return last_error(); }

int rpa_set_stream(rpa_ctx *ctx, void *hip_stream) {
  RPA_TRY(check_ctx(ctx));
  std::lock_guard<std::mutex> g(ctx->c.mu);
  ctx->c.stream = hip_stream ? (hipStream_t)hip_stream : ctx->c.own_stream;
  return RPA_OK;
}

int rpa_chi0(rpa_ctx *ctx, const rpa_system *sys, int32_t iq, double omega, rpa_precision prec,
             void *chi0) {
  RPA_TRY(check_ctx(ctx));
  Ctx &c = ctx->c;
  std::lock_guard<std::mutex> g(c.mu);
  RPA_TRY(set_device(c));
  HostSmall hs;
  RPA_TRY(validate_system(sys, hs));
  if (!chi0) return fail(RPA_E_ARG, "chi0 output is NULL");
  if (iq < 0 || iq >= hs.nq) return fail(RPA_E_ARG, "iq = %d outside [0, nq)", iq);
  if (!std::isfinite(omega) || omega < 0.0) return fail(RPA_E_ARG, "omega must be finite and >= 0");
  if (prec != RPA_FP64 && prec != RPA_FP32 && prec != RPA_BF16X3 && prec != RPA_F16X3)
    return fail(RPA_E_ARG, "unknown precision %d", (int)prec);
  const int N = hs.naux;
  const int64_t M = (int64_t)hs.nk * hs.nocc * hs.nvirt;
  const bool cplx = hs.is_complex != 0;
  const int64_t belem = cplx ? 16 : 8;
  const void *B = sys->B;
  if (!B || sys->memspace == RPA_MEM_HOST) {
    void *buf;
    RPA_TRY(c.workspace("B", M * N * belem, &buf));
    if (!B && hs.nbas > 0) {
      // atomic-orbital system: the MO transform of the pair-fit coefficients, per k block
      void *cbuf, *scr;
      const int64_t cbytes = (int64_t)(hs.c_occ.size() + hs.c_virt.size()) * 8;
      RPA_TRY(c.workspace("ao_coeff", cbytes, &cbuf));
      RPA_TRY(c.workspace("ao_scratch", ao_scratch_bytes(hs.nbas, hs.nocc, N), &scr));
      double2 *co = reinterpret_cast<double2 *>(cbuf);
      double2 *cv = co + hs.c_occ.size() / 2;
      void *pstage;
      RPA_TRY(c.workspace("ao_stage", ao_stage_scratch_bytes(hs), &pstage));
      RPA_TRY(stage_ao_coefficients(c.stream, hs, co, cv, pstage));
      const int64_t per_k = (int64_t)hs.nocc * hs.nvirt * N;
      for (int ik = 0; ik < hs.nk; ++ik)
        RPA_HIP(launch_ao_B(c.stream, sys->philox_seed, sys->sigma, hs.nk, iq, ik, hs.nbas, hs.nocc, hs.nvirt, N,
                            co + (int64_t)hs.kq[(size_t)iq * hs.nk + ik] * hs.nbas * hs.nocc,
                            cv + (int64_t)ik * hs.nbas * hs.nvirt, scr,
                            reinterpret_cast<double2 *>(buf) + (int64_t)ik * per_k));
    } else if (!B) {
      RPA_HIP(launch_philox_B(c.stream, sys->philox_seed, sys->sigma, hs.nk, iq, 0, hs.nk, hs.nocc,
                              hs.nvirt, N, cplx, buf));
    } else {
      RPA_HIP(hipMemcpyAsync(buf, (const char *)B + (int64_t)iq * M * N * belem, (size_t)(M * N * belem),
                             hipMemcpyHostToDevice, c.stream));
    }
    B = buf;
  } else {
    B = (const char *)B + (int64_t)iq * M * N * belem;
  }
  // eps_occ | eps_virt | zeta_k | kq | (pad to 16) | PointDesc, one upload
  const int64_t nsmall = (int64_t)(hs.eps_occ.size() + hs.eps_virt.size() + hs.zeta_k.size());
  const int64_t pd_off = ((nsmall * 8 + (int64_t)hs.kq.size() * 4) + 15) / 16 * 16;
  std::vector<char> hsm((size_t)(pd_off + (int64_t)sizeof(PointDesc)));
  char *hp = hsm.data();
  memcpy(hp, hs.eps_occ.data(), hs.eps_occ.size() * 8);
  memcpy(hp + hs.eps_occ.size() * 8, hs.eps_virt.data(), hs.eps_virt.size() * 8);
  memcpy(hp + (hs.eps_occ.size() + hs.eps_virt.size()) * 8, hs.zeta_k.data(), hs.zeta_k.size() * 8);
  memcpy(hp + nsmall * 8, hs.kq.data(), hs.kq.size() * 4);
  PointDesc pd{iq, 0, omega};
  memcpy(hp + pd_off, &pd, sizeof(pd));
  void *d_all;
  RPA_TRY(c.workspace("chi0_args", (int64_t)hsm.size() + 64, &d_all));
  RPA_HIP(hipMemcpyAsync(d_all, hsm.data(), hsm.size(), hipMemcpyHostToDevice, c.stream));
  char *da = (char *)d_all;
  double2 *out;
  const bool direct = cplx && sys->memspace == RPA_MEM_DEVICE;
  if (direct) out = (double2 *)chi0;
  else RPA_TRY(c.workspace("chi0_out", (int64_t)N * N * 16, (void **)&out));
  double *wt;
  RPA_TRY(c.workspace("chi0_wtab", M * 8, (void **)&wt));
  Chi0Args a{};
  a.B = B;
  a.b_slot_stride = 0;
  a.eps_occ = (const double *)da;
  a.eps_virt = (const double *)(da + hs.eps_occ.size() * 8);
  a.zeta_k = (const double *)(da + (hs.eps_occ.size() + hs.eps_virt.size()) * 8);
  a.kq = (const int32_t *)(da + nsmall * 8);
  a.pts = (const PointDesc *)(da + pd_off);
  a.wtab = wt;
  a.ksplit = 1;
  a.out = out;
  a.out_stride = (int64_t)N * N;   // one point; also the stride of the partial planes
  a.nk = hs.nk; a.nocc = hs.nocc; a.nvirt = hs.nvirt; a.N = N; a.M = M;
  RPA_HIP(launch_chi0_weights(c.stream, a, 1));
  // one point fills few workgroups: the FP64 and FP32 contractions split their rows (up
  // to kMaxSplit ways, each split at least 512 rows) so that the launch fills the GPU;
  // the later splits go to partial planes summed in split order.  RPA_CHI0_KSPLIT fixes
  // the count.
  int ncu_all = 0;
  if (hipDeviceGetAttribute(&ncu_all, hipDeviceAttributeMultiprocessorCount, c.device) != hipSuccess) ncu_all = 256;
  auto split_for = [&](int64_t tn, int64_t slots_per_cu) {
    const int64_t T = (N + tn - 1) / tn;
    int ks = chi0_pick_ksplit(T * (T + 1) / 2, slots_per_cu * ncu_all, M, kMaxSplit);
    if (const char *e = getenv("RPA_CHI0_KSPLIT")) {
      const int v = atoi(e);
      if (v >= 1) ks = std::min(v, kMaxSplit);
    }
    return ks;
  };
  // the partial planes of the largest split count that the HBM limit still holds (an
  // existing buffer of the same name is reused); every count is capped to it
  auto plan_planes = [&](int *ks_of, int n) -> int {
    int ks_max = 1;
    for (int i = 0; i < n; ++i) ks_max = std::max(ks_max, ks_of[i]);
    const int64_t plane = (int64_t)N * N * 16;
    auto it = c.cache.find("chi0_partial");
    const int64_t have = it != c.cache.end() ? it->second.bytes : 0;   // reused if large enough
    while (ks_max > 1 && !c.mem.would_fit(std::max<int64_t>(0, (int64_t)(ks_max - 1) * plane - have))) --ks_max;
    for (int i = 0; i < n; ++i) ks_of[i] = std::min(ks_of[i], ks_max);
    if (ks_max > 1) return c.workspace("chi0_partial", (int64_t)(ks_max - 1) * plane, (void **)&a.partial);
    return RPA_OK;
  };
  if (prec == RPA_BF16X3 || prec == RPA_F16X3) {
    // prepared left (unweighted) and right (weighted) operands, then the split contraction
    const bool f16 = prec == RPA_F16X3;
    double *dg, *scr;
    unsigned short *lr;
    float2 *part;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c.device) != hipSuccess) ncu = 256;
    Bf16Plan pl;
    bf16_plan(M, N, 1, ncu, 0, 128, &pl);   // the larger of the two tiles' partial buffers
    const int64_t pe = bf16_prepared_elems(M, N);
    const int64_t max_part = bf16_partial_elems(pl, 1);
    RPA_TRY(c.workspace("chi0_bf16_ops", 2 * pe * 2, (void **)&lr));
    RPA_TRY(c.workspace("chi0_bf16_part", max_part * 8, (void **)&part));
    RPA_TRY(c.workspace("chi0_diag", (int64_t)N * 8, (void **)&dg));
    RPA_TRY(c.workspace("chi0_diag_scratch", bf16_diag_scratch_doubles(M, N) * 8, (void **)&scr));
    double *sc = nullptr;   // fp16: [slab maxima | weight maxima | left scale | right scale]
    if (f16) {
      const int64_t nb = f16_absmax_scratch_doubles(1);
      RPA_TRY(c.workspace("chi0_f16_scales", (2 * nb + 2) * 8, (void **)&sc));
      RPA_HIP(launch_absmax_blocks(c.stream, (const double *)B, M * N * (cplx ? 2 : 1), 0, 1, sc));
      RPA_HIP(launch_absmax_blocks(c.stream, wt, M, M, 1, sc + nb));
      RPA_HIP(launch_f16_scales(c.stream, sc, nullptr, nullptr, 1, sc + 2 * nb));
      RPA_HIP(launch_f16_scales(c.stream, sc, sc + nb, a.pts, 1, sc + 2 * nb + 1));
    }
    const double *lsc = f16 ? sc + 2 * f16_absmax_scratch_doubles(1) : nullptr;
    const double *rsc = f16 ? lsc + 1 : nullptr;
    RPA_HIP(launch_bf16_prepare(c.stream, B, cplx, M, N, nullptr, 1, lr, nullptr, nullptr, lsc, f16));
    RPA_HIP(launch_bf16_prepare(c.stream, B, cplx, M, N, wt, 1, lr + pe, scr, dg, rsc, f16));
    Bf16Group g{};
    g.L = lr;
    g.l_stride = 0;
    g.R = lr + pe;
    g.r_stride = pe;
    g.pts = a.pts;
    g.part = part;
    g.npts = 1;
    g.f16 = f16;
    int tn = 128;
    RPA_TRY(tune_bf16_tile(c.stream, g, M, N, ncu, max_part, cplx, &tn));
    bf16_plan(M, N, 1, ncu, max_part, tn, &g.pl);
    RPA_HIP(launch_bf16_herk_groups(c.stream, &g, 1, cplx));
    RPA_HIP(launch_bf16_reduce(c.stream, g.pl, part, 1, N, dg, out, 0, a.pts, lsc, rsc));
  } else if (prec != RPA_FP64) {
    float2 *b32;
    double *dg, *scr;
    RPA_TRY(c.workspace("chi0_B32", M * N * 8, (void **)&b32));
    RPA_TRY(c.workspace("chi0_diag", (int64_t)N * 8, (void **)&dg));
    RPA_TRY(c.workspace("chi0_diag_scratch", diag_exact_scratch_doubles(M, N, 1) * 8, (void **)&scr));
    RPA_HIP(launch_to_f32(c.stream, B, b32, M * N, cplx));
    RPA_HIP(launch_diag_exact(c.stream, B, cplx, M, N, wt, 1, scr, dg));
    const int f32_cfgs[3] = {kF32T64, kF32T128, kF32T64W2};
    int ks_of[3];
    for (int ci = 0; ci < 3; ++ci) {
      const int e = f32_cfg_edge(f32_cfgs[ci]);
      ks_of[ci] = split_for(e, e == 128 ? 1 : 2);
    }
    RPA_TRY(plan_planes(ks_of, 3));
    int tile = kF32T64;
    RPA_TRY(tune_f32_tile(c.stream, a, 1, cplx, b32, dg, &tile, ks_of));
    a.ksplit = ks_of[tile == kF32T128 ? 1 : tile == kF32T64W2 ? 2 : 0];
    RPA_HIP(launch_chi0_mixed(c.stream, a, 1, b32, dg, (int)prec, tile));
  } else {
    int ks_of[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    const int ncfg = std::min(chi0_cfg_count(), 8);
    for (int cf = 0; cf < ncfg; ++cf) ks_of[cf] = split_for(chi0_cfg_tile(cf), chi0_cfg_slots_per_cu(cf));
    RPA_TRY(plan_planes(ks_of, ncfg));
    int cfg = 1;
    RPA_TRY(tune_chi0_cfg(c.stream, a, 1, cplx, &cfg, ks_of));
    a.ksplit = ks_of[cfg];
    RPA_HIP(launch_chi0_f64(c.stream, a, 1, cplx, cfg));
  }
  if (!direct) RPA_TRY(deliver_complex(c, chi0, out, (int64_t)N * N, hs.is_complex, sys->memspace));
  RPA_HIP(hipStreamSynchronize(c.stream));
  return RPA_OK;
}

int rpa_pi(rpa_ctx *ctx, int32_t n, int32_t is_complex, int32_t memspace, const void *vhalf,
           const void *chi0, void *pi) {
  RPA_TRY(check_ctx(ctx));
  Ctx &c = ctx->c;
  std::lock_guard<std::mutex> g(c.mu);
  RPA_TRY(set_device(c));
  if (n < 1 || n > 16384) return fail(RPA_E_ARG, "n = %d out of range", n);
  if (is_complex != 0 && is_complex != 1) return fail(RPA_E_ARG, "is_complex must be 0 or 1");
  if (memspace != RPA_MEM_HOST && memspace != RPA_MEM_DEVICE) return fail(RPA_E_ARG, "bad memspace");
  if (!vhalf || !chi0 || !pi) return fail(RPA_E_ARG, "NULL array");
  const int64_t nn = (int64_t)n * n;
  double2 *dv, *dc, *dt, *dp;
  RPA_TRY(stage_complex(c, "pi_v", vhalf, nn, is_complex, memspace, &dv));
  RPA_TRY(stage_complex(c, "pi_c", chi0, nn, is_complex, memspace, &dc));
  RPA_TRY(c.workspace("pi_t", nn * 16, (void **)&dt));
  RPA_TRY(c.workspace("pi_p", nn * 16, (void **)&dp));
  GemmArgs g1{};
  g1.A = dc; g1.a_div = 1; g1.B = dv; g1.b_div = 1; g1.C = dt; g1.N = n;
  RPA_HIP(launch_zgemm_f64(c.stream, g1, 1));
  GemmArgs g2{};
  g2.A = dv; g2.a_div = 1; g2.B = dt; g2.b_div = 1; g2.C = dp; g2.N = n;
  RPA_HIP(launch_zgemm_f64(c.stream, g2, 1));
  RPA_TRY(deliver_complex(c, pi, dp, nn, is_complex, memspace));
  RPA_HIP(hipStreamSynchronize(c.stream));
  return RPA_OK;
}

int rpa_trln(rpa_ctx *ctx, int32_t n, int32_t batch, int32_t is_complex, int32_t memspace,
             const void *pi, double *out) {
  RPA_TRY(check_ctx(ctx));
  Ctx &c = ctx->c;
  std::lock_guard<std::mutex> g(c.mu);
  RPA_TRY(set_device(c));
  if (n < 1 || n > 16384) return fail(RPA_E_ARG, "n = %d out of range", n);
  if (batch < 0 || batch > (1 << 20)) return fail(RPA_E_ARG, "batch = %d out of range", batch);
  if (is_complex != 0 && is_complex != 1) return fail(RPA_E_ARG, "is_complex must be 0 or 1");
  if (memspace != RPA_MEM_HOST && memspace != RPA_MEM_DEVICE) return fail(RPA_E_ARG, "bad memspace");
  if (batch == 0) return RPA_OK;
  if (!pi || !out) return fail(RPA_E_ARG, "NULL array");
  const int64_t nn = (int64_t)n * n;
  double2 *dp;
  RPA_TRY(stage_complex(c, "trln_pi", pi, nn * batch, is_complex, memspace, &dp));
  double *de;
  int32_t *di;
  RPA_TRY(c.workspace("trln_eps", (int64_t)batch * 8, (void **)&de));
  RPA_TRY(c.workspace("trln_info", (int64_t)batch * 4, (void **)&di));
  if (trln_single()) {
    RPA_HIP(launch_trln_f64(c.stream, dp, nn, n, batch, de, di, nullptr));
  } else {
    void *scr;
    RPA_TRY(c.workspace("trln_scratch", trln_blocked_scratch_bytes(batch), &scr));
    RPA_HIP(launch_negate(c.stream, dp, nn, n, batch));
    RPA_HIP(launch_trln_blocked(c.stream, dp, nn, n, batch, de, di, nullptr, scr));
  }
  std::vector<int32_t> info((size_t)batch);
  RPA_HIP(hipMemcpyAsync(info.data(), di, (size_t)batch * 4, hipMemcpyDeviceToHost, c.stream));
  RPA_TRY(from_device(out, de, (size_t)batch * 8, memspace, c.stream));
  RPA_HIP(hipStreamSynchronize(c.stream));
  for (int b = 0; b < batch; ++b)
    if (info[b] >= 0)
      return fail(RPA_E_NOTSPD, "1 - Pi is not positive definite for matrix %d (column %d)", b, info[b]);
  return RPA_OK;
}

int rpa_energy(rpa_ctx *ctx, const rpa_system *sys, const rpa_freq *freq, rpa_precision prec,
               double *E, double *eps_qw) {
  RPA_TRY(check_ctx(ctx));
  Ctx &c = ctx->c;
  std::lock_guard<std::mutex> g(c.mu);
  RPA_TRY(set_device(c));
  HostSmall hs;
  RPA_TRY(validate_system(sys, hs));
  RPA_TRY(validate_freq(freq));
  if (!E) return fail(RPA_E_ARG, "E is NULL");
  if (prec != RPA_FP64 && prec != RPA_FP32 && prec != RPA_BF16X3 && prec != RPA_F16X3)
    return fail(RPA_E_ARG, "unknown precision %d", (int)prec);
  PointJob job;
  job.sys = sys;
  job.hs = &hs;
  job.prec = prec;
  for (int q = 0; q < hs.nq; ++q)
    for (int j = 0; j < freq->nw; ++j) {
      job.pq.push_back(q);
      job.pw.push_back(freq->omega[j]);
    }
  job.quadrature = true;
  job.weight.assign(freq->weight, freq->weight + freq->nw);
  RPA_TRY(run_points(c, c.stream, job, budget_of(c), true));
  *E = job.E;
  if (eps_qw) memcpy(eps_qw, job.eps.data(), job.eps.size() * 8);
  return RPA_OK;
}

int rpa_points(rpa_ctx *ctx, const rpa_system *sys, int32_t npts, const int32_t *iq, const double *w,
               rpa_precision prec, double *eps) {
  RPA_TRY(check_ctx(ctx));
  Ctx &c = ctx->c;
  std::lock_guard<std::mutex> g(c.mu);
  RPA_TRY(set_device(c));
  HostSmall hs;
  RPA_TRY(validate_system(sys, hs));
  if (npts < 0) return fail(RPA_E_ARG, "npts < 0");
  if (npts == 0) return RPA_OK;
  if (!iq || !w || !eps) return fail(RPA_E_ARG, "NULL array");
  if (prec != RPA_FP64 && prec != RPA_FP32 && prec != RPA_BF16X3 && prec != RPA_F16X3)
    return fail(RPA_E_ARG, "unknown precision %d", (int)prec);
  PointJob job;
  job.sys = sys;
  job.hs = &hs;
  job.prec = prec;
  job.pq.assign(iq, iq + npts);
  job.pw.assign(w, w + npts);
  RPA_TRY(run_points(c, c.stream, job, budget_of(c), true));
  memcpy(eps, job.eps.data(), (size_t)npts * 8);
  return RPA_OK;
}

int rpa_projector(rpa_ctx *ctx, int32_t nk, int32_t nbas, double eps_d, int32_t memspace, const void *S,
                  void *T) {
  RPA_TRY(check_ctx(ctx));
  Ctx &c = ctx->c;
  std::lock_guard<std::mutex> g(c.mu);
  RPA_TRY(set_device(c));
  if (nk < 1 || nk > 65535 || nbas < 1 || nbas > 1024) return fail(RPA_E_ARG, "nk %d or nbas %d out of range", nk, nbas);
  if (!(eps_d >= 0.0) || !std::isfinite(eps_d)) return fail(RPA_E_ARG, "eps_d must be finite and >= 0");
  if (memspace != RPA_MEM_HOST && memspace != RPA_MEM_DEVICE) return fail(RPA_E_ARG, "bad memspace");
  if (!S || !T) return fail(RPA_E_ARG, "NULL array");
  const int64_t bytes = (int64_t)nk * nbas * nbas * 16;
  void *ds, *dt, *scr;
  RPA_TRY(c.workspace("proj_S", bytes, &ds));
  RPA_TRY(c.workspace("proj_T", bytes, &dt));
  RPA_TRY(c.workspace("proj_scratch", projector_scratch_bytes(nk, nbas), &scr));
  RPA_TRY(to_device(ds, S, (size_t)bytes, memspace, c.stream));
  RPA_HIP(launch_projector(c.stream, (const double2 *)ds, nk, nbas, eps_d, scr, (double2 *)dt));
  RPA_TRY(from_device(T, dt, (size_t)bytes, memspace, c.stream));
  RPA_HIP(hipStreamSynchronize(c.stream));
  return RPA_OK;
}

int rpa_philox_B(rpa_ctx *ctx, uint64_t seed, double sigma, int32_t nk, int32_t iq, int32_t ik,
                 int32_t nocc, int32_t nvirt, int32_t naux, int32_t is_complex, int32_t memspace,
                 void *out) {
  RPA_TRY(check_ctx(ctx));
  Ctx &c = ctx->c;
  std::lock_guard<std::mutex> g(c.mu);
  RPA_TRY(set_device(c));
  if (nk < 1 || iq < 0 || ik < 0 || ik >= nk || nocc < 1 || nvirt < 1 || naux < 1)
    return fail(RPA_E_ARG, "bad block indices or sizes");
  if (memspace != RPA_MEM_HOST && memspace != RPA_MEM_DEVICE) return fail(RPA_E_ARG, "bad memspace");
  if (!out) return fail(RPA_E_ARG, "out is NULL");
  const int64_t count = (int64_t)nocc * nvirt * naux;
  const int64_t bytes = count * (is_complex ? 16 : 8);
  void *dst = out;
  if (memspace == RPA_MEM_HOST) RPA_TRY(c.workspace("philox_out", bytes, &dst));
  RPA_HIP(launch_philox_B(c.stream, seed, sigma, nk, iq, ik, ik + 1, nocc, nvirt, naux, is_complex != 0, dst));
  if (memspace == RPA_MEM_HOST) RPA_HIP(hipMemcpyAsync(out, dst, (size_t)bytes, hipMemcpyDeviceToHost, c.stream));
  RPA_HIP(hipStreamSynchronize(c.stream));
  return RPA_OK;
}

int rpa_philox_words(rpa_ctx *ctx, uint64_t seed, int32_t nk, int32_t iq, int32_t ik, uint64_t e0,
                     int64_t count, int32_t memspace, uint32_t *out) {
  RPA_TRY(check_ctx(ctx));
  Ctx &c = ctx->c;
  std::lock_guard<std::mutex> g(c.mu);
  RPA_TRY(set_device(c));
  if (nk < 1 || iq < 0 || ik < 0 || ik >= nk || count < 0) return fail(RPA_E_ARG, "bad block or count");
  if (memspace != RPA_MEM_HOST && memspace != RPA_MEM_DEVICE) return fail(RPA_E_ARG, "bad memspace");
  if (count == 0) return RPA_OK;
  if (!out) return fail(RPA_E_ARG, "out is NULL");
  void *dst = out;
  if (memspace == RPA_MEM_HOST) RPA_TRY(c.workspace("philox_words", count * 16, &dst));
  RPA_HIP(launch_philox_words(c.stream, seed, nk, iq, ik, e0, count, (uint32_t *)dst));
  if (memspace == RPA_MEM_HOST) RPA_HIP(hipMemcpyAsync(out, dst, (size_t)count * 16, hipMemcpyDeviceToHost, c.stream));
  RPA_HIP(hipStreamSynchronize(c.stream));
  return RPA_OK;
}

int rpa_submit(rpa_ctx *ctx, const rpa_system *sys, const rpa_freq *freq, rpa_precision prec,
               uint64_t *job_id) {
  RPA_TRY(check_ctx(ctx));
  return ctx->c.sched->submit(sys, freq, prec, job_id);
}

int rpa_poll(rpa_ctx *ctx, uint64_t job_id, int32_t timeout_ms, rpa_result *out, double *eps_qw) {
  RPA_TRY(check_ctx(ctx));
  return ctx->c.sched->poll(job_id, timeout_ms, out, eps_qw);
}

int rpa_get_stats(rpa_ctx *ctx, rpa_stats *out) {
  RPA_TRY(check_ctx(ctx));
  if (!out) return fail(RPA_E_ARG, "out is NULL");
  Ctx &c = ctx->c;
  const MemLedger::Snapshot m = c.mem.snapshot();
  out->hbm_limit = m.limit;
  out->hbm_in_use = m.in_use;
  out->hbm_high_water = m.high_water;
  c.sched->fill_stats(out);
  return RPA_OK;
}

int rpa_profile(rpa_ctx *ctx, int32_t enable) {
  RPA_TRY(check_ctx(ctx));
  Ctx &c = ctx->c;
  std::lock_guard<std::mutex> g(c.mu);
  c.prof_collect();
  c.profile = enable != 0;
  for (int k = 0; k < RPA_K_COUNT; ++k) {
    c.prof_launches[k] = 0;
    c.prof_ms[k] = 0.0;
  }
  return RPA_OK;
}

int rpa_profile_read(rpa_ctx *ctx, rpa_kernel_times *out) {
  RPA_TRY(check_ctx(ctx));
  if (!out) return fail(RPA_E_ARG, "out is NULL");
  Ctx &c = ctx->c;
  std::lock_guard<std::mutex> g(c.mu);
  for (int k = 0; k < RPA_K_COUNT; ++k) {
    out->launches[k] = c.prof_launches[k];
    out->ms[k] = c.prof_ms[k];
  }
  return RPA_OK;
}

int rpa_tuned(char *buf, int32_t len, int32_t *needed) {
  const int n = tuned_entries(buf, len);
  if (needed) *needed = n;
  return RPA_OK;
}

}  // extern "C"
