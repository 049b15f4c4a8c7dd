// Host runtime of librpa: context, device-memory accounting, errors, staging of the
// system description, and the (q, w) point pipeline shared by the synchronous entry
// points and the serving scheduler.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rpa.h"
#include "common.hpp"
#include "serve_core.hpp"

namespace rpa {

// ---- errors -------------------------------------------------------------------
void set_error(const char *fmt, ...);
const char *last_error();
int fail(int code, const char *fmt, ...);

#define RPA_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::rpa::fail(RPA_E_DEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                         __FILE__, __LINE__);                                           \
  } while (0)

#define RPA_TRY(expr)          \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != RPA_OK) return rc_; \
  } while (0)


class Scheduler;

// ---- device memory -------------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  int64_t bytes = 0;
  bool cached = false;   // a workspace of synchronous calls (counted in Ctx::cached_bytes)
};

struct Ctx {
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;     // stream of synchronous calls
  std::mutex mu;                    // serialises synchronous calls on this context
  // Device-memory accounting (limit, in use, cached workspaces, job reservations).
  MemLedger mem;
  // RPA_FAULT: injected allocation failures; RPA_POISON=1: every new device allocation is
  // filled with 0xFF bytes (NaN in every floating-point format used here) before use.
  FaultPlan faults;
  bool poison = false;
  // Grow-only workspaces of synchronous calls.  The map itself is only read or changed
  // by a thread holding `mu`; other threads read cached_bytes instead.
  std::map<std::string, DevBuf> cache;
  std::unique_ptr<Scheduler> sched;
  // kernel timing of synchronous calls (rpa_profile)
  bool profile = false;
  int64_t prof_launches[RPA_K_COUNT] = {0};
  double prof_ms[RPA_K_COUNT] = {0};
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_pending;
  // Record the start / end of a kernel of kind k on stream s (no-op unless profiling).
  int prof_begin(hipStream_t s, int k);
  int prof_end(hipStream_t s);
  // After the stream has been synchronised: fold pending event pairs into the totals.
  int prof_collect();

  // second stream of synchronous calls (created on first use; null if that fails)
  hipStream_t aux_stream();
  hipStream_t aux = nullptr;

  // Allocate `bytes` of device memory.  A cached (synchronous-call) allocation must also
  // leave room for what admitted serving jobs may still allocate; a job's allocation is
  // part of its own reservation.
  int alloc(DevBuf &b, int64_t bytes, const char *what, bool cached = false);
  void release(DevBuf &b);
  // Cached workspace of at least `bytes` (device), reused across synchronous calls.
  int workspace(const char *name, int64_t bytes, void **out);
  void free_cache();
};

// ---- staged system ----------------------------------------------------------------
// Host-side copy of the small arrays of a system (always made, for validation) plus
// device copies; large arrays (B, V^(1/2)) are referenced or staged by the pipeline.
struct HostSmall {
  int32_t nk, nq, nocc, nvirt, naux, is_complex;
  std::vector<int32_t> kq;
  std::vector<double> eps_occ, eps_virt, zeta_k, zeta_q;
  // atomic-orbital systems: basis size and the projected KS coefficients (complex,
  // interleaved), [nk_occ][nbas][nocc] and [nk][nbas][nvirt]
  int32_t nbas = 0;
  std::vector<double> c_occ, c_virt;
  // raw coefficients to be projected on the device (Sec. 2.3): the overlaps S(k),
  // [nk][nbas][nbas] complex interleaved, and the threshold; S empty: c is projected already
  std::vector<double> S;
  double eps_d = 0.0;
};

// Device bytes stage_ao_coefficients needs beside the two coefficient buffers.
int64_t ao_stage_scratch_bytes(const HostSmall &hs);
// Upload the atomic-orbital coefficients of hs into d_cocc ([nk_occ][nbas][nocc]) and
// d_cvirt ([nk][nbas][nvirt]); with overlaps in hs, apply the periodic projector T(k) on
// the device first (scratch: ao_stage_scratch_bytes).
int stage_ao_coefficients(hipStream_t st, const HostSmall &hs, double2 *d_cocc, double2 *d_cvirt, void *scratch);

int validate_system(const rpa_system *sys, HostSmall &hs);
int validate_freq(const rpa_freq *f);

// Bytes of device memory the pipeline needs for a group of `gq` q-points of a system,
// `npts` (q, w) points in flight, and whether B must be staged.
struct PlanSizes {
  int64_t small_bytes, vhalf_bytes, b_slot_bytes, point_bytes;
};
PlanSizes plan_sizes(const HostSmall &hs, bool b_on_device_complex, bool b_device_real);

// One evaluation job over a list of (q, w) points of one system, used by rpa_energy,
// rpa_points and the scheduler.  Device memory comes from the context's workspace cache
// (use_cache, synchronous calls) or from buffers owned by the call.
// ---- fused split-BF16 contraction launches of concurrent serving jobs (fuser.cpp) ----
struct Fuser;
Fuser *fuser_create(int device, int ncu);
void fuser_destroy(Fuser *f);
// A job that may post groups registers (+1) when it starts and unregisters (-1) when done.
void fuser_register(Fuser *f, int delta);
void fuser_stats(Fuser *f, int64_t *launches, int64_t *fused_groups, int64_t *solo_groups);
// Launch the contraction group g, whose operands stream st prepares: alone on st if it
// fills the GPU by itself (or f is null), else fused with the groups other jobs post at
// about the same time; st waits for the launch either way.
int fused_herk(Fuser *f, hipStream_t st, const Bf16Group &g, bool cplx);
// The same for the FP64 contraction (configuration cfg; only the paired configuration 4
// is fused) and the FP32 contraction (tile configuration; only kF32T64W2 is fused).
int fused_chi0_f64(Fuser *f, hipStream_t st, const Chi0Args &a, int npts, bool cplx, int cfg);
int fused_chi0_f32(Fuser *f, hipStream_t st, const Chi0Args &a, int npts, const float2 *B32, const double *diag,
                   int tile);

struct PointJob {
  const rpa_system *sys;     // caller's description (pointers valid during run)
  const HostSmall *hs;
  rpa_precision prec;
  std::vector<int32_t> pq;   // q of every point
  std::vector<double> pw;    // omega of every point
  std::vector<double> eps;   // output eps per point (host)
  // rpa_energy: the points are the full q-major grid and the quadrature runs on the device
  bool quadrature = false;
  std::vector<double> weight;   // W_j
  std::vector<double> qstage;   // host staging of zeta_q and W_j
  double E = 0.0;
  int max_q_group = 0;          // > 0: at most this many q's staged at once
  Fuser *fuser = nullptr;       // serving: small contractions may be fused across jobs
};

int run_points(Ctx &ctx, hipStream_t stream, PointJob &job, int64_t mem_budget, bool use_cache);

// Tile and K-step configuration (launch_chi0_f64's cfg) of the FP64 chi0 contraction for
// this launch shape: fixed by the environment, else timed once per shape bucket and
// cached (tuner.cpp).  a.out must hold npts outputs; its contents are overwritten.
// ksplit_of[c] (null: all 1) is the row split count the launch would use with
// configuration c; the candidates are timed with it (a.partial holds its planes).
int tune_chi0_cfg(hipStream_t st, const Chi0Args &a, int npts, bool cplx, int *cfg_out,
                  const int *ksplit_of = nullptr);
// Tile edge (64 or 128) of the split-BF16 contraction of group g (operands prepared on
// st, g.part large enough for the candidates' truncated launches: at most max_part
// elements): fixed by RPA_BF16_TILE, else timed once per shape bucket and cached.
int tune_bf16_tile(hipStream_t st, const Bf16Group &g, int64_t M, int N, int64_t slots, int64_t max_part, bool cplx,
                   int *tn_out);
// Configuration (kF32T64, kF32T128, kF32T64W2) of the FP32 contraction of npts points
// (a.out and a.partial hold them; they are overwritten): fixed by RPA_F32_TILE (64, 128,
// 64w2), else timed once per shape bucket and cached.  ksplit_of (null: all 1) gives the
// row split count of each configuration in that order; the candidates are timed with it.
int tune_f32_tile(hipStream_t st, const Chi0Args &a, int npts, bool cplx, const float2 *B32, const double *diag,
                  int *tile_out, const int *ksplit_of = nullptr);
// The FP64 configuration tune_chi0_cfg would give this shape without timing anything:
// the environment's fixed choice, else the choice already made (or loaded) for its shape
// bucket, else the default (t64k16).
int chi0_cfg_lookup(const Chi0Args &a, int npts, bool cplx);
// Fixed device scratch of rpa_chi0_noalloc (noalloc.hip): its size, and the per-device
// lookup of its address (called by rpa_init with the device current).
constexpr int64_t kNoallocScratchBytes = (int64_t)64 << 20;
int noalloc_setup(int device);
// "bucket configuration" lines of the choices made so far; returns the full length.
int tuned_entries(char *buf, int len);
// RPA_TRLN_SINGLE=1 selects the one-workgroup-per-matrix Cholesky instead of the blocked one.
bool trln_single();

}  // namespace rpa

struct rpa_ctx {
  rpa::Ctx c;
};
