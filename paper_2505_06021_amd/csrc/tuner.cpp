// Autotuner of the chi0 contractions' tile shapes: the FP64 contraction's tile and
// K-step depth, the FP32 contraction's configuration (64- or 128-wide tiles, or 64-wide
// tiles with two frequencies per workgroup) and the split-BF16 contraction's tile edge
// (RPA_F32_TILE=64|128|64w2 and RPA_BF16_TILE=64|128 fix them; RPA_TUNE_VERBOSE=1 prints
// the candidates' timings).
//
// Candidates (launch_chi0_f64 configurations): 64-wide tiles with 8, 16 or 32 rows per
// LDS step (two workgroups per CU), 128-wide tiles with 16-row steps (one per CU), and
// 64-wide tiles with 16-row steps contracting two frequencies of a q per workgroup (only
// where the launch's pair table pairs some points).
// The first launch of a shape bucket (real/complex, N rounded up to 64, points per
// launch, order of magnitude of M) times every candidate on a truncated contraction (the
// first 4096 rows, one row split) written into the launch's own output, which the real
// launch then overwrites in full (the kernels store, they never accumulate), so tuning
// never changes a result; all candidates sum the same products in the same row order.
// Every later launch of the bucket in the process uses the choice.  RPA_CHI0_CFG=<name>
// (t64k8, t64k16, t64k32, t128k16, t64k16w2) or the older RPA_CHI0_KT=8|16|32 fixes the
// configuration (read on every launch); RPA_TUNE=0 keeps t64k16; RPA_TUNE_CACHE names a
// text file that keeps the choices across processes ("bucket name" lines).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.hpp"

namespace rpa {
namespace {

constexpr int kDefaultCfg = 1;   // 64-wide tiles, 16-row steps
constexpr int kTuneReps = 4;     // timing rounds per candidate (the first one warms up)
constexpr int kBf16TuneReps = 3;           // split-BF16: fewer, longer rounds
constexpr double kBf16TuneMs = 5.0;        // split-BF16: time budget of one timed launch

std::mutex g_tune_mu;
std::map<std::string, int> g_tuned;
bool g_loaded = false;

int cfg_by_name(const std::string &n) {
  for (int c = 0; c < chi0_cfg_count(); ++c)
    if (n == chi0_cfg_name(c)) return c;
  return -1;
}

void load_cache_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char *p = getenv("RPA_TUNE_CACHE");
  if (!p) return;
  std::ifstream f(p);
  std::string key, name;
  while (f >> key >> name) {
    if (key.compare(0, 5, "bf16_") == 0) {
      if (name == "t64" || name == "t128") g_tuned[key] = name == "t64" ? 64 : 128;
      continue;
    }
    if (key.compare(0, 4, "f32_") == 0) {
      for (int c : {kF32T64, kF32T128, kF32T64W2})
        if (name == f32_cfg_name(c)) g_tuned[key] = c;
      continue;
    }
    const int c = cfg_by_name(name);
    if (c >= 0) g_tuned[key] = c;
  }
}

std::string entry_name(const std::string &key, int v) {
  if (key.compare(0, 5, "bf16_") == 0) return v == 64 ? "t64" : "t128";
  if (key.compare(0, 4, "f32_") == 0) return f32_cfg_name(v);
  return chi0_cfg_name(v);
}

void store_cache_locked() {
  const char *p = getenv("RPA_TUNE_CACHE");
  if (!p) return;
  std::ofstream f(p, std::ios::trunc);
  for (auto &kv : g_tuned) f << kv.first << " " << entry_name(kv.first, kv.second) << "\n";
}

std::string bucket(const Chi0Args &a, int npts, bool cplx) {
  int mlog = 0;
  for (int64_t m = a.M; m > 1; m >>= 1) ++mlog;
  std::ostringstream k;
  k << "f64_" << (cplx ? "c" : "r") << "_N" << ((a.N + 63) / 64) * 64 << "_p" << (npts > 512 ? 512 : npts) << "_m"
    << mlog;
  return k.str();
}

// -1 when the environment leaves the choice to the tuner
int fixed_cfg() {
  if (const char *e = getenv("RPA_CHI0_CFG")) {
    const int c = cfg_by_name(e);
    if (c >= 0) return c;
  }
  if (const char *e = getenv("RPA_CHI0_KT")) {
    const int v = atoi(e);
    if (v == 8) return 0;
    if (v == 16) return 1;
    if (v == 32) return 2;
  }
  const char *t = getenv("RPA_TUNE");
  return (t && t[0] == '0') ? kDefaultCfg : -1;
}

}  // namespace

int tune_chi0_cfg(hipStream_t st, const Chi0Args &a, int npts, bool cplx, int *cfg_out, const int *ksplit_of) {
  const int f = fixed_cfg();
  if (f >= 0) {
    *cfg_out = f;
    return RPA_OK;
  }
  const std::string key = bucket(a, npts, cplx);
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_cache_locked();
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) {
    *cfg_out = it->second;
    return RPA_OK;
  }
  // time each configuration on the first rows of the contraction with the row split
  // count the launch would use with it (so the candidates fill the GPU as the real
  // launches do), 4096 rows per split (enough K steps for a steady state, few enough that
  // tuning costs a fraction of one launch); compare time per row
  // kTuneReps rounds, the first to warm code and caches, the candidates in alternating
  // order; each candidate keeps its best time (clock and power drift between rounds)
  std::vector<float> tmin(chi0_cfg_count(), 1e30f);
  hipEvent_t e0, e1;
  RPA_HIP(hipEventCreate(&e0));
  RPA_HIP(hipEventCreate(&e1));
  for (int rep = 0; rep < kTuneReps; ++rep) {
    for (int ci = 0; ci < chi0_cfg_count(); ++ci) {
      const int c = rep % 2 ? chi0_cfg_count() - 1 - ci : ci;
      if (chi0_cfg_points_per_wg(c) == 2 && (a.pairs == nullptr || a.npairs == npts)) continue;
      Chi0Args t = a;
      t.ksplit = ksplit_of ? ksplit_of[c] : 1;
      t.M = a.M < 4096LL * t.ksplit ? a.M : 4096LL * t.ksplit;
      RPA_HIP(hipEventRecord(e0, st));
      RPA_HIP(launch_chi0_f64(st, t, npts, cplx, c));
      RPA_HIP(hipEventRecord(e1, st));
      RPA_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      RPA_HIP(hipEventElapsedTime(&ms, e0, e1));
      ms /= (float)t.M;
      if (rep > 0 && ms < tmin[c]) tmin[c] = ms;
      if (rep == kTuneReps - 1 && getenv("RPA_TUNE_VERBOSE"))
        fprintf(stderr, "[tune] %s %s: %.3e ms per row (%d splits, %lld rows)\n", key.c_str(), chi0_cfg_name(c),
                tmin[c], t.ksplit, (long long)t.M);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int best = kDefaultCfg;
  for (int c = 0; c < chi0_cfg_count(); ++c)
    if (tmin[c] < tmin[best]) best = c;
  g_tuned[key] = best;
  store_cache_locked();
  *cfg_out = best;
  return RPA_OK;
}

int chi0_cfg_lookup(const Chi0Args &a, int npts, bool cplx) {
  const int f = fixed_cfg();
  if (f >= 0) return f;
  const std::string key = bucket(a, npts, cplx);
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_cache_locked();
  auto it = g_tuned.find(key);
  return it != g_tuned.end() ? it->second : kDefaultCfg;
}

int tune_bf16_tile(hipStream_t st, const Bf16Group &g, int64_t M, int N, int64_t slots, int64_t max_part, bool cplx,
                   int *tn_out) {
  if (const char *e = getenv("RPA_BF16_TILE")) {
    const int v = atoi(e);
    if (v == 64 || v == 128) {
      *tn_out = v;
      return RPA_OK;
    }
  }
  if (const char *t = getenv("RPA_TUNE"))
    if (t[0] == '0') {
      *tn_out = 128;
      return RPA_OK;
    }
  int mlog = 0;
  for (int64_t m = M; m > 1; m >>= 1) ++mlog;
  std::ostringstream k;
  k << "bf16_" << (cplx ? "c" : "r") << "_N" << ((N + 63) / 64) * 64 << "_p" << (g.npts > 512 ? 512 : g.npts) << "_m"
    << mlog;
  const std::string key = k.str();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_cache_locked();
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) {
    *tn_out = it->second;
    return RPA_OK;
  }
  // time both tile edges with their real plan (split count and full split length: a
  // 128-wide tile writes a four times larger partial tile at the end of its split, so
  // shortened splits favour the 64-wide one) on the group's first npts_t points: all of
  // them when the launch is short (its last round of workgroups then weighs as in the
  // real launch), else as many as take about kBf16TuneMs.  Into the group's partial
  // buffer (which the real launch overwrites wherever the reduction reads); compare time
  // per point.
  const double issued_pt = (cplx ? 4.0 : 1.0) * 3.0 * (double)M * N * (N + 1.0);
  const double est_ms = issued_pt * g.npts / 1.0e12;   // at about 1 PFLOP/s issued
  int npts_t = g.npts;
  if (est_ms > kBf16TuneMs) npts_t = std::max(1, (int)(g.npts * kBf16TuneMs / est_ms));
  const int cands[2] = {128, 64};
  float tmin[2] = {1e30f, 1e30f};
  hipEvent_t e0, e1;
  RPA_HIP(hipEventCreate(&e0));
  RPA_HIP(hipEventCreate(&e1));
  for (int rep = 0; rep < kBf16TuneReps; ++rep) {
    for (int cj = 0; cj < 2; ++cj) {
      const int ci = rep % 2 ? 1 - cj : cj;
      const int tn = cands[ci];
      Bf16Group t = g;
      bf16_plan(M, N, g.npts, slots, max_part, tn, &t.pl);
      if (max_part > 0 && bf16_partial_elems(t.pl, g.npts) > max_part) continue;
      t.npts = npts_t;
      RPA_HIP(hipEventRecord(e0, st));
      RPA_HIP(launch_bf16_herk_groups(st, &t, 1, cplx));
      RPA_HIP(hipEventRecord(e1, st));
      RPA_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      RPA_HIP(hipEventElapsedTime(&ms, e0, e1));
      ms /= (float)npts_t;
      if (rep > 0 && ms < tmin[ci]) tmin[ci] = ms;
      if (rep == kBf16TuneReps - 1 && getenv("RPA_TUNE_VERBOSE"))
        fprintf(stderr, "[tune] %s t%d: %.4f ms per point (%d of %d points, %d splits x %d steps, %d tiles)\n",
                key.c_str(), tn, tmin[ci], npts_t, g.npts, t.pl.nsplit, t.pl.kc_per_split, t.pl.ntiles);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int best = tmin[1] < tmin[0] ? cands[1] : cands[0];
  g_tuned[key] = best;
  store_cache_locked();
  *tn_out = best;
  return RPA_OK;
}

int tune_f32_tile(hipStream_t st, const Chi0Args &a, int npts, bool cplx, const float2 *B32, const double *diag,
                  int *tile_out, const int *ksplit_of) {
  if (const char *e = getenv("RPA_F32_TILE")) {
    const std::string v = e;
    if (v == "64" || v == "128" || v == "64w2") {
      *tile_out = v == "64" ? kF32T64 : v == "128" ? kF32T128 : kF32T64W2;
      return RPA_OK;
    }
  }
  if (const char *t = getenv("RPA_TUNE"))
    if (t[0] == '0') {
      *tile_out = kF32T64;
      return RPA_OK;
    }
  int mlog = 0;
  for (int64_t m = a.M; m > 1; m >>= 1) ++mlog;
  std::ostringstream k;
  k << "f32_" << (cplx ? "c" : "r") << "_N" << ((a.N + 63) / 64) * 64 << "_p" << (npts > 512 ? 512 : npts) << "_m"
    << mlog;
  const std::string key = k.str();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_cache_locked();
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) {
    *tile_out = it->second;
    return RPA_OK;
  }
  // the three configurations, each with the row split count the launch would give it and
  // 8192 rows per split, into the launch's own output and partial planes (overwritten by
  // the real launch); long enough that each workgroup reaches its steady state (short
  // runs favour the 64-wide tile); compare time per row
  const int cands[3] = {kF32T64, kF32T128, kF32T64W2};
  float tmin[3] = {1e30f, 1e30f, 1e30f};
  hipEvent_t e0, e1;
  RPA_HIP(hipEventCreate(&e0));
  RPA_HIP(hipEventCreate(&e1));
  for (int rep = 0; rep < kTuneReps; ++rep) {
    for (int cj = 0; cj < 3; ++cj) {
      const int ci = rep % 2 ? 2 - cj : cj;
      const int tile = cands[ci];
      if (f32_cfg_points_per_wg(tile) == 2 && (a.pairs == nullptr || a.npairs == npts)) continue;
      Chi0Args t = a;
      t.ksplit = ksplit_of ? ksplit_of[ci] : 1;
      t.M = a.M < 8192LL * t.ksplit ? a.M : 8192LL * t.ksplit;
      RPA_HIP(hipEventRecord(e0, st));
      RPA_HIP(launch_chi0_mixed(st, t, npts, B32, diag, 1, tile));
      RPA_HIP(hipEventRecord(e1, st));
      RPA_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      RPA_HIP(hipEventElapsedTime(&ms, e0, e1));
      ms /= (float)t.M;
      if (rep > 0 && ms < tmin[ci]) tmin[ci] = ms;
      if (rep == kTuneReps - 1 && getenv("RPA_TUNE_VERBOSE"))
        fprintf(stderr, "[tune] %s %s: %.3e ms per row (%d splits, %lld rows, %d points)\n", key.c_str(),
                f32_cfg_name(tile), tmin[ci], t.ksplit, (long long)t.M, npts);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int bi = 0;
  for (int ci = 1; ci < 3; ++ci)
    if (tmin[ci] < tmin[bi]) bi = ci;
  const int best = cands[bi];
  g_tuned[key] = best;
  store_cache_locked();
  *tile_out = best;
  return RPA_OK;
}

int tuned_entries(char *buf, int len) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  std::string s;
  for (auto &kv : g_tuned) s += kv.first + " " + entry_name(kv.first, kv.second) + "\n";
  if (buf && len > 0) {
    strncpy(buf, s.c_str(), (size_t)len - 1);
    buf[len - 1] = 0;
  }
  return (int)s.size();
}

}  // namespace rpa
