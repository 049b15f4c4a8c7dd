// Autotuner of the FP64 chi0 contraction's K-step depth (rows staged per LDS stage).
//
// The first launch of a shape bucket (real/complex, N rounded up to the 64-wide tile,
// points per launch, order of magnitude of M) times the contraction for each candidate
// depth on a truncated contraction (the first 4096 rows, one row split) written into the
// launch's own output, which the real launch then overwrites in full (the kernel stores,
// it never accumulates), so tuning never changes a result; every later launch of the
// bucket in the process uses the same choice.  RPA_CHI0_KT=8|16|32 fixes the depth (read
// on every launch, no tuning); RPA_TUNE=0 keeps the default depth of 16; RPA_TUNE_CACHE
// names a text file that keeps the choices across processes ("key depth" lines).
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

std::mutex g_tune_mu;
std::map<std::string, int> g_tuned;
bool g_loaded = false;

const char *cache_path() { return getenv("RPA_TUNE_CACHE"); }

void load_cache_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char *p = cache_path();
  if (!p) return;
  std::ifstream f(p);
  std::string key;
  int kt;
  while (f >> key >> kt)
    if (kt == 8 || kt == 16 || kt == 32) g_tuned[key] = kt;
}

void store_cache_locked() {
  const char *p = cache_path();
  if (!p) return;
  std::ofstream f(p, std::ios::trunc);
  for (auto &kv : g_tuned) f << kv.first << " " << kv.second << "\n";
}

std::string bucket(const Chi0Args &a, int npts, bool cplx) {
  int mlog = 0;
  for (int64_t m = a.M; m > 1; m >>= 1) ++mlog;
  std::ostringstream k;
  k << "f64_" << (cplx ? "c" : "r") << "_N" << ((a.N + 63) / 64) * 64 << "_p" << (npts > 512 ? 512 : npts) << "_m"
    << mlog;
  return k.str();
}

}  // namespace

static int chi0_kt_fixed() {
  const char *e = getenv("RPA_CHI0_KT");
  const int v = e ? atoi(e) : 0;
  if (v == 8 || v == 16 || v == 32) return v;
  const char *t = getenv("RPA_TUNE");
  return (t && t[0] == '0') ? 16 : 0;
}

int tune_chi0_kt(hipStream_t st, const Chi0Args &a, int npts, bool cplx, int *kt_out) {
  const int f = chi0_kt_fixed();
  if (f) {
    *kt_out = f;
    return RPA_OK;
  }
  const std::string key = bucket(a, npts, cplx);
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_cache_locked();
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) {
    *kt_out = it->second;
    return RPA_OK;
  }
  // time each depth on the first rows of the contraction (enough K steps for a steady
  // state, few enough that tuning costs a fraction of one launch)
  Chi0Args t = a;
  t.M = a.M < 4096 ? a.M : 4096;
  t.ksplit = 1;
  const int cands[3] = {8, 16, 32};
  float best_ms = 1e30f;
  int best = 16;
  hipEvent_t e0, e1;
  RPA_HIP(hipEventCreate(&e0));
  RPA_HIP(hipEventCreate(&e1));
  for (int rep = 0; rep < 2; ++rep) {          // the first round warms code and caches
    for (int kt : cands) {
      RPA_HIP(hipEventRecord(e0, st));
      RPA_HIP(launch_chi0_f64(st, t, npts, cplx, kt));
      RPA_HIP(hipEventRecord(e1, st));
      RPA_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      RPA_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep == 1 && ms < best_ms) {
        best_ms = ms;
        best = kt;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g_tuned[key] = best;
  store_cache_locked();
  *kt_out = best;
  return RPA_OK;
}

int tuned_entries(char *buf, int len) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  std::string s;
  for (auto &kv : g_tuned) s += kv.first + " " + std::to_string(kv.second) + "\n";
  if (buf && len > 0) {
    strncpy(buf, s.c_str(), (size_t)len - 1);
    buf[len - 1] = 0;
  }
  return (int)s.size();
}

}  // namespace rpa
