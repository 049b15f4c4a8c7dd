// rpa_chi0_noalloc: the FP64 chi0 of one (q, omega) point without any device allocation.
//
// The contraction's scratch (the system's band energies, weights and k (+) q map, the
// point descriptor, the per-row weight table w_m zeta_k and the partial planes of the row
// splits) lives in one file-scope device array of kNoallocScratchBytes.  Host code never
// passes the array's name to a kernel or a copy: its device address is looked up once per
// device with hipGetSymbolAddress when a context is created there, and that address is
// used everywhere.  Every call on a device shares that device's array; calls on one
// context are serialised by the context's lock, calls through two contexts of one device
// at the same time race on it.  Nothing in the array has to start at zero: every region
// a call reads was written earlier in the same call (the weight table by its kernel, the
// partial planes by the contraction's later row splits, which store rather than add).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>

#include "runtime.hpp"

namespace rpa {

namespace {

__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }

}  // namespace

int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(RPA_E_ARG, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return RPA_OK;
  void *ptr = nullptr;
  // the caller has made `device` current
  RPA_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return fail(RPA_E_DEVICE, "no device address for the fixed scratch array on device %d", device);
  g_scratch_ptr[device] = ptr;
  return RPA_OK;
}

namespace {
void *scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_ptr[device];
}
}  // namespace

}  // namespace rpa

using namespace rpa;

extern "C" int rpa_chi0_noalloc(rpa_ctx *ctx, const rpa_system *sys, int32_t iq, double omega,
                                rpa_precision prec, void *chi0) {
  if (!ctx) return fail(RPA_E_ARG, "ctx is NULL");
  Ctx &c = ctx->c;
  std::lock_guard<std::mutex> g(c.mu);
  RPA_HIP(hipSetDevice(c.device));
  if (prec != RPA_FP64) return fail(RPA_E_ARG, "rpa_chi0_noalloc computes FP64 only (precision %d)", (int)prec);
  if (!sys) return fail(RPA_E_ARG, "system is NULL");
  if (sys->memspace != RPA_MEM_DEVICE || !sys->B || sys->is_complex != 1 || sys->nbas != 0)
    return fail(RPA_E_ARG, "rpa_chi0_noalloc takes a complex system with B given, all arrays in device memory");
  if (!chi0) return fail(RPA_E_ARG, "chi0 output is NULL");
  HostSmall hs;
  RPA_TRY(validate_system(sys, hs));
  if (iq < 0 || iq >= hs.nq) return fail(RPA_E_ARG, "iq = %d outside [0, nq)", iq);
  if (!std::isfinite(omega) || omega < 0.0) return fail(RPA_E_ARG, "omega must be finite and >= 0");
  char *base = (char *)scratch_of(c.device);
  if (!base) return fail(RPA_E_DEVICE, "the fixed scratch of device %d was not set up", c.device);

  const int N = hs.naux;
  const int64_t M = (int64_t)hs.nk * hs.nocc * hs.nvirt;
  // scratch layout: eps_occ | eps_virt | zeta_k | kq | PointDesc, then the weight table,
  // then as many partial planes as fit
  const int64_t n_eo = (int64_t)hs.eps_occ.size(), n_ev = (int64_t)hs.eps_virt.size(), n_zk = hs.nk;
  const int64_t kq_off = (n_eo + n_ev + n_zk) * 8;
  const int64_t pd_off = (kq_off + (int64_t)hs.kq.size() * 4 + 15) / 16 * 16;
  const int64_t w_off = round256(pd_off + (int64_t)sizeof(PointDesc));
  const int64_t part_off = round256(w_off + M * 8);
  if (part_off > kNoallocScratchBytes)
    return fail(RPA_E_NOMEM,
                "rpa_chi0_noalloc: this system needs %lld bytes of scratch (band energies and one weight per "
                "contraction row), above the fixed %lld",
                (long long)part_off, (long long)kNoallocScratchBytes);
  const int64_t plane = (int64_t)N * N * 16;
  const int64_t planes_fit = (kNoallocScratchBytes - part_off) / plane;

  PointDesc pd{iq, 0, omega};
  hipStream_t st = c.stream;
  RPA_HIP(hipMemcpyAsync(base, hs.eps_occ.data(), (size_t)n_eo * 8, hipMemcpyHostToDevice, st));
  RPA_HIP(hipMemcpyAsync(base + n_eo * 8, hs.eps_virt.data(), (size_t)n_ev * 8, hipMemcpyHostToDevice, st));
  RPA_HIP(hipMemcpyAsync(base + (n_eo + n_ev) * 8, hs.zeta_k.data(), (size_t)n_zk * 8, hipMemcpyHostToDevice, st));
  RPA_HIP(hipMemcpyAsync(base + kq_off, hs.kq.data(), hs.kq.size() * 4, hipMemcpyHostToDevice, st));
  RPA_HIP(hipMemcpyAsync(base + pd_off, &pd, sizeof(pd), hipMemcpyHostToDevice, st));

  const int64_t belem = 16;
  Chi0Args a{};
  a.B = (const char *)sys->B + (int64_t)iq * M * N * belem;
  a.b_slot_stride = 0;
  a.eps_occ = (const double *)base;
  a.eps_virt = (const double *)(base + n_eo * 8);
  a.zeta_k = (const double *)(base + (n_eo + n_ev) * 8);
  a.kq = (const int32_t *)(base + kq_off);
  a.pts = (const PointDesc *)(base + pd_off);
  a.wtab = (double *)(base + w_off);
  a.out = (double2 *)chi0;
  a.out_stride = (int64_t)N * N;
  a.nk = hs.nk; a.nocc = hs.nocc; a.nvirt = hs.nvirt; a.N = N; a.M = M;
  a.ksplit = 1;
  RPA_HIP(launch_chi0_weights(st, a, 1));

  // the configuration the tuner chose for this shape in this process (or the fixed or
  // default one); nothing is timed here
  const int cfg = chi0_cfg_lookup(a, 1, true);
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c.device) != hipSuccess) ncu = 256;
  const int64_t T = (N + chi0_cfg_tile(cfg) - 1) / chi0_cfg_tile(cfg);
  int ks = chi0_pick_ksplit(T * (T + 1) / 2, (int64_t)chi0_cfg_slots_per_cu(cfg) * ncu, M, kMaxSplit);
  if (const char *e = getenv("RPA_CHI0_KSPLIT")) {
    const int v = atoi(e);
    if (v >= 1) ks = std::min(v, kMaxSplit);
  }
  ks = (int)std::min<int64_t>(ks, planes_fit + 1);
  a.ksplit = ks;
  a.partial = ks > 1 ? (double2 *)(base + part_off) : nullptr;
  RPA_HIP(launch_chi0_f64(st, a, 1, true, cfg));
  RPA_HIP(hipStreamSynchronize(st));
  return RPA_OK;
}
