// eps = ln det(1 - Pi) + Re Tr Pi for a batch of Hermitian Pi, FP64.
//
// The paper takes ln det(1 - Z) for every (q, w) point (Algorithm 1) without saying
// how; here 1 - Pi is Hermitian positive definite (Pi <= 0 because w < 0), so a
// Cholesky factor L gives ln det = 2 sum ln L_ii.  The kernel factors
// W = -Pi with the identity kept implicit: the pivot of column c is 1 + d_c, where
// d_c is the updated diagonal of W, and 2 ln L_cc = log1p(d_c), which keeps full
// relative accuracy when Pi is small (large w) and ln det nearly cancels Tr Pi.
//
// One workgroup (8 waves) per matrix, right-looking blocked factorisation with
// 16-column panels: the diagonal block is factored in LDS, the panel below it is
// solved row-per-thread, and the trailing lower triangle is updated with
// v_mfma_f64_16x16x4f64 in 16 x 16 complex tiles spread over the waves.  The matrix
// is factored in place (the caller passes a scratch copy).
#include "common.hpp"

namespace rpa {
namespace {

constexpr int NB = 16;
constexpr int NT = 512;
constexpr int NWAVES = NT / 64;

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void tile_of(int t, int &tr, int &tc) {
  int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  tr = r;
  tc = t - r * (r + 1) / 2;
}

__global__ __launch_bounds__(NT) void trln_kernel(double2 *pi, int64_t stride, int n, double *eps,
                                                  int32_t *info, const int32_t *out_map) {
  __shared__ double2 D[NB][NB + 1];
  __shared__ double Ldiag[NB];
  __shared__ double red[NT];

  double2 *A = pi + (int64_t)blockIdx.x * stride;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;

  // Tr Pi and W = -Pi on the lower triangle
  double tr_part = 0.0;
  for (int r = 0; r < n; ++r) {
    for (int c = tid; c <= r; c += NT) {
      const double2 v = A[(int64_t)r * n + c];
      if (c == r) tr_part += v.x;
      A[(int64_t)r * n + c] = make_double2(-v.x, -v.y);
    }
  }
  red[tid] = tr_part;

  double logacc = 0.0;
  int failcol = -1;
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = min(NB, n - j0);
    __syncthreads();
    if (tid < NB * NB) {
      const int r = tid / NB, c = tid % NB;
      if (r < jb && c <= r) D[r][c] = A[(int64_t)(j0 + r) * n + j0 + c];
    }
    __syncthreads();
    for (int c = 0; c < jb; ++c) {
      const double d = D[c][c].x;
      const double piv = 1.0 + d;
      if (!(piv > 0.0) || !(piv < INFINITY)) {
        failcol = j0 + c;
        break;
      }
      const double l = sqrt(piv);
      if (tid == 0) {
        Ldiag[c] = l;
        logacc += log1p(d);
      }
      if (tid > c && tid < jb) {
        const double2 v = D[tid][c];
        D[tid][c] = make_double2(v.x / l, v.y / l);
      }
      __syncthreads();
      if (tid < NB * NB) {
        const int r = tid / NB, s = tid % NB;
        if (s > c && s <= r && r < jb) {
          const double2 x = D[r][c], y = D[s][c];
          // x * conj(y)
          D[r][s].x -= x.x * y.x + x.y * y.y;
          D[r][s].y -= x.y * y.x - x.x * y.y;
        }
      }
      __syncthreads();
    }
    if (failcol >= 0) break;

    // panel: L21 = W21 L11^{-H}, one row per thread
    for (int r = j0 + jb + tid; r < n; r += NT) {
      double2 x[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t)
        x[t] = (t < jb) ? A[(int64_t)r * n + j0 + t] : make_double2(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c < jb) {
          double2 v = x[c];
#pragma unroll
          for (int t = 0; t < NB; ++t) {
            if (t < c) {
              const double2 y = D[c][t];
              // v -= x_t * conj(y)
              v.x -= x[t].x * y.x + x[t].y * y.y;
              v.y -= x[t].y * y.x - x[t].x * y.y;
            }
          }
          const double il = 1.0 / Ldiag[c];
          x[c] = make_double2(v.x * il, v.y * il);
        }
      }
#pragma unroll
      for (int t = 0; t < NB; ++t)
        if (t < jb) A[(int64_t)r * n + j0 + t] = x[t];
    }
    __syncthreads();

    // trailing update of the lower triangle: W22 -= L21 L21^H
    const int r0 = j0 + jb;
    const int nt = (n - r0 + 15) / 16;
    const int ntiles = nt * (nt + 1) / 2;
    for (int t = wave; t < ntiles; t += NWAVES) {
      int tr, tc;
      tile_of(t, tr, tc);
      const int R0 = r0 + tr * 16, S0 = r0 + tc * 16;
      d4 accR = d4{0.0, 0.0, 0.0, 0.0}, accI = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < NB / 4; ++ks) {
        const int kc = ks * 4 + lk;
        const bool kin = kc < jb;
        const double2 x = (kin && R0 + li < n) ? A[(int64_t)(R0 + li) * n + j0 + kc] : make_double2(0.0, 0.0);
        const double2 y = (kin && S0 + li < n) ? A[(int64_t)(S0 + li) * n + j0 + kc] : make_double2(0.0, 0.0);
        // x * conj(y) = (xr yr + xi yi) + i (xi yr - xr yi)
        accR = mfma(x.x, y.x, accR);
        accR = mfma(x.y, y.y, accR);
        accI = mfma(x.y, y.x, accI);
        accI = mfma(-x.x, y.y, accI);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = R0 + lk + 4 * r;
        const int col = S0 + li;
        if (row < n && col <= row) {
          double2 *p = A + (int64_t)row * n + col;
          const double2 v = *p;
          *p = make_double2(v.x - accR[r], v.y - accI[r]);
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < NT; ++i) tr += red[i];
    const int o = out_map ? out_map[blockIdx.x] : (int)blockIdx.x;
    eps[o] = (failcol >= 0) ? __builtin_nan("") : logacc + tr;
    info[o] = failcol;
  }
}

__global__ void quadrature_kernel(const double *eps, const double *zeta_q, const double *weight,
                                  int32_t nq, int32_t nw, double *E) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double inv2pi = 0.15915494309189533577;
  double acc = 0.0;
  for (int q = 0; q < nq; ++q)
    for (int j = 0; j < nw; ++j) acc += zeta_q[q] * weight[j] * eps[(int64_t)q * nw + j] * inv2pi;
  *E = acc;
}

__global__ void widen_kernel(const double *in, double2 *out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = make_double2(in[i], 0.0);
}

__global__ void narrow_kernel(const double2 *in, double *out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = in[i].x;
}

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_trln_f64(hipStream_t s, double2 *pi, int64_t stride, int32_t n, int32_t batch,
                           double *eps, int32_t *info, const int32_t *out_map) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(trln_kernel, dim3((unsigned)batch), dim3(NT), 0, s, pi, stride, n, eps, info,
                     out_map);
  return hipGetLastError();
}

hipError_t launch_quadrature(hipStream_t s, const double *eps, const double *zeta_q,
                             const double *weight, int32_t nq, int32_t nw, double *E) {
  hipLaunchKernelGGL(quadrature_kernel, dim3(1), dim3(64), 0, s, eps, zeta_q, weight, nq, nw, E);
  return hipGetLastError();
}

hipError_t launch_widen(hipStream_t s, const double *in, double2 *out, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(widen_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_narrow(hipStream_t s, const double2 *in, double *out, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(narrow_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace rpa
