// Device generator of the fit coefficients B^P_ia(k,q): Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) and an FP64
// Box-Muller transform.  Coefficients are regenerated on demand instead of being
// stored, as the paper does with its on-the-fly MO transform of the fit coefficients
// (Sec. "RPA Algorithm"): large systems stream B through HBM one q at a time.
#include "common.hpp"

namespace rpa {
namespace {

constexpr uint32_t kM0 = 0xD2511F53u;   // Philox4x32 round multipliers
constexpr uint32_t kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u;   // Weyl key increments
constexpr uint32_t kW1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += kW0; k1 += kW1; }
    const uint32_t hi0 = __umulhi(kM0, c.x), lo0 = kM0 * c.x;
    const uint32_t hi1 = __umulhi(kM1, c.z), lo1 = kM1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ __forceinline__ double uniform52(uint32_t a, uint32_t b) {
  const uint64_t x = ((uint64_t)(a >> 6) << 26) | (uint64_t)(b >> 6);
  return ((double)x + 0.5) * 0x1p-52;
}

// `stream` is the third counter word: 0 for B, 1 for the pair-fit coefficients C of
// atomic-orbital systems (same key, independent stream).
template <bool CPLX>
__global__ __launch_bounds__(256) void philox_B_kernel(uint64_t seed, double sigma, int32_t nk,
                                                       int32_t iq, int32_t k0, int64_t per_k,
                                                       void *out, uint32_t stream) {
  const uint32_t key0 = (uint32_t)seed;
  const uint32_t key_hi = (uint32_t)(seed >> 32);
  // blockIdx.y is the k of the slab (no 64-bit division per element)
  const int32_t kk = (int32_t)blockIdx.y;
  const uint32_t key1 = key_hi + (uint32_t)(iq * nk + k0 + kk);
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < per_k;
       e0 += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t e = (uint64_t)e0;
    const int64_t g = (int64_t)kk * per_k + e0;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)e, (uint32_t)(e >> 32), stream, 0u), key0, key1);
    const double u1 = uniform52(w.x, w.y);
    const double u2 = uniform52(w.z, w.w);
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    if (CPLX) {
      const double sc = sigma * 0.70710678118654752440 * r;
      reinterpret_cast<double2 *>(out)[g] = make_double2(sc * cs, sc * sn);
    } else {
      reinterpret_cast<double *>(out)[g] = sigma * r * cs;
    }
  }
}

__global__ __launch_bounds__(256) void philox_words_kernel(uint64_t seed, int32_t key1_off,
                                                           uint64_t e0, int64_t count,
                                                           uint32_t *out) {
  const uint32_t key0 = (uint32_t)seed;
  const uint32_t key1 = (uint32_t)(seed >> 32) + (uint32_t)key1_off;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < count;
       g += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t e = e0 + (uint64_t)g;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)e, (uint32_t)(e >> 32), 0u, 0u), key0, key1);
    reinterpret_cast<uint4 *>(out)[g] = w;
  }
}

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_philox_B(hipStream_t s, uint64_t seed, double sigma, int32_t nk, int32_t iq,
                           int32_t k0, int32_t k1, int32_t nocc, int32_t nvirt, int32_t naux,
                           bool cplx, void *out) {
  const int64_t per_k = (int64_t)nocc * nvirt * naux;
  const int64_t total = per_k * (k1 - k0);
  if (total <= 0) return hipSuccess;
  if (k1 - k0 > 65535) return hipErrorInvalidValue;
  // about 64K workgroups over all k slabs together
  int64_t bx = (per_k + 255) / 256, cap = 65536 / (k1 - k0);
  if (cap < 64) cap = 64;
  if (bx > cap) bx = cap;
  const dim3 grid((unsigned)bx, (unsigned)(k1 - k0));
  if (cplx)
    hipLaunchKernelGGL(philox_B_kernel<true>, grid, dim3(256), 0, s, seed, sigma, nk, iq, k0, per_k, out, 0u);
  else
    hipLaunchKernelGGL(philox_B_kernel<false>, grid, dim3(256), 0, s, seed, sigma, nk, iq, k0, per_k, out, 0u);
  return hipGetLastError();
}

hipError_t launch_philox_C(hipStream_t s, uint64_t seed, double sigma, int32_t nk, int32_t iq, int32_t ik,
                           int32_t nbas, int32_t naux, void *out) {
  const int64_t per = (int64_t)nbas * nbas * naux;
  if (per <= 0) return hipSuccess;
  int64_t bx = (per + 255) / 256;
  if (bx > 65536) bx = 65536;
  hipLaunchKernelGGL(philox_B_kernel<true>, dim3((unsigned)bx, 1u), dim3(256), 0, s, seed, sigma, nk, iq, ik, per,
                     out, 1u);
  return hipGetLastError();
}

hipError_t launch_philox_words(hipStream_t s, uint64_t seed, int32_t nk, int32_t iq, int32_t ik,
                               uint64_t e0, int64_t count, uint32_t *out) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(philox_words_kernel, dim3(grid_for(count)), dim3(256), 0, s, seed,
                     iq * nk + ik, e0, count, out);
  return hipGetLastError();
}

}  // namespace rpa
