// Autotuner of the FP64 chi0 contraction's tile shape and K-step depth.
//
// Candidates (launch_chi0_f64 configurations): 64-wide tiles with 8, 16 or 32 rows per
// LDS step (two workgroups per CU) and 128-wide tiles with 16-row steps (one per CU).
// The first launch of a shape bucket (real/complex, N rounded up to 64, points per
// launch, order of magnitude of M) times every candidate on a truncated contraction (the
// first 4096 rows, one row split) written into the launch's own output, which the real
// launch then overwrites in full (the kernels store, they never accumulate), so tuning
// never changes a result; all candidates sum the same products in the same row order.
// Every later launch of the bucket in the process uses the choice.  RPA_CHI0_CFG=<name>
// (t64k8, t64k16, t64k32, t128k16) or the older RPA_CHI0_KT=8|16|32 fixes the
// configuration (read on every launch); RPA_TUNE=0 keeps t64k16; RPA_TUNE_CACHE names a
// text file that keeps the choices across processes ("bucket name" lines).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "runtime.hpp"

namespace rpa {
namespace {

constexpr int kDefaultCfg = 1;   // 64-wide tiles, 16-row steps

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
    const int c = cfg_by_name(name);
    if (c >= 0) g_tuned[key] = c;
  }
}

void store_cache_locked() {
  const char *p = getenv("RPA_TUNE_CACHE");
  if (!p) return;
  std::ofstream f(p, std::ios::trunc);
  for (auto &kv : g_tuned) f << kv.first << " " << chi0_cfg_name(kv.second) << "\n";
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

int tune_chi0_cfg(hipStream_t st, const Chi0Args &a, int npts, bool cplx, int *cfg_out) {
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
  // time each configuration on the first rows of the contraction (enough K steps for a
  // steady state, few enough that tuning costs a fraction of one launch)
  Chi0Args t = a;
  t.M = a.M < 4096 ? a.M : 4096;
  t.ksplit = 1;
  float best_ms = 1e30f;
  int best = kDefaultCfg;
  hipEvent_t e0, e1;
  RPA_HIP(hipEventCreate(&e0));
  RPA_HIP(hipEventCreate(&e1));
  for (int rep = 0; rep < 2; ++rep) {   // the first round warms code and caches
    for (int c = 0; c < chi0_cfg_count(); ++c) {
      RPA_HIP(hipEventRecord(e0, st));
      RPA_HIP(launch_chi0_f64(st, t, npts, cplx, c));
      RPA_HIP(hipEventRecord(e1, st));
      RPA_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      RPA_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep == 1 && ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g_tuned[key] = best;
  store_cache_locked();
  *cfg_out = best;
  return RPA_OK;
}

int tuned_entries(char *buf, int len) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  std::string s;
  for (auto &kv : g_tuned) s += kv.first + " " + chi0_cfg_name(kv.second) + "\n";
  if (buf && len > 0) {
    strncpy(buf, s.c_str(), (size_t)len - 1);
    buf[len - 1] = 0;
  }
  return (int)s.size();
}

}  // namespace rpa
