// chi0(q, i w) in FP64 on the matrix cores (v_mfma_f64_16x16x4f64).
//
// chi0_PQ = sum_m conj(B_mP) (w_m zeta_k B_mQ), m = (k, i, a) running over the
// N_k*N_occ*N_virt transitions of one q (Sec. 2.2, fit-basis polarizability equation,
// with w_m = -4 Delta_m / (Delta_m^2 + w^2) and Delta_m = eps_a(k) - eps_i(k (+) q)).
// The k-sum of Algorithm 1 (the k1/k2 loop accumulating P_q) is folded into the
// contraction index m, so one launch performs the whole accumulation.
//
// Work decomposition: one workgroup per 64 x 64 complex tile on or below the diagonal
// of one (q, w) point's output; the point index is blockIdx.y so every point of a
// q-group shares one launch.  The contraction runs in K steps of 16 rows: each thread
// loads 4 consecutive complex coefficients of one row for both operand panels, the
// right operand is multiplied by w_m zeta_k in registers (the weight is computed from
// the band energies there, never stored), and both panels go to a double-buffered LDS
// tile.  Four waves each own a 32 x 32 sub-tile (2 x 2 MFMA blocks, Re and Im
// accumulators).  Off-diagonal tiles also store their conjugate transpose, so the full
// Hermitian matrix is produced from the lower-triangle work only.
#include "common.hpp"

namespace rpa {
namespace {

constexpr int TN = 64;        // output tile edge (complex elements)
constexpr int KT = 16;        // contraction rows per pipeline step
constexpr int LDP = TN + 1;   // LDS row pitch in complex elements (one element of padding)

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <bool CPLX_B>
__device__ __forceinline__ double2 load_b(const void *base, int64_t idx) {
  if (CPLX_B) return reinterpret_cast<const double2 *>(base)[idx];
  return make_double2(reinterpret_cast<const double *>(base)[idx], 0.0);
}

__device__ __forceinline__ void tile_of(int t, int &tr, int &tc) {
  int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  tr = r;
  tc = t - r * (r + 1) / 2;
}

template <bool CPLX_B>
__global__ __launch_bounds__(256, 2) void chi0_f64_kernel(Chi0Args a) {
  __shared__ double2 lds[2][2][KT][LDP];

  const PointDesc pd = a.pts[blockIdx.y];
  int tr, tc;
  tile_of((int)blockIdx.x, tr, tc);
  const int N = a.N;
  const int64_t M = a.M;
  const int P0 = tr * TN, Q0 = tc * TN;
  const bool diag = (tr == tc);

  const int tid = threadIdx.x;
  const int lrow = tid >> 4;          // row of the K step this thread loads
  const int lcol = (tid & 15) * 4;    // first of its 4 columns

  const char *bbase = reinterpret_cast<const char *>(a.B) +
                      (int64_t)pd.bslot * a.b_slot_stride * (CPLX_B ? 16 : 8);
  const int nov = a.nocc * a.nvirt;
  const int32_t *kqrow = a.kq + (int64_t)pd.q * a.nk;
  const double om2 = pd.omega * pd.omega;

  double2 ra[4], rb[4];

  auto gload = [&](int64_t m0) {
    const int64_t m = m0 + lrow;
    double w = 0.0;
    if (m < M) {
      const int k = (int)(m / nov);
      const int rem = (int)(m - (int64_t)k * nov);
      const int i = rem / a.nvirt;
      const int av = rem - i * a.nvirt;
      const double d = a.eps_virt[(int64_t)k * a.nvirt + av] - a.eps_occ[(int64_t)kqrow[k] * a.nocc + i];
      w = -4.0 * a.zeta_k[k] * d / (d * d + om2);
    }
    const int64_t rowoff = m * N;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int P = P0 + lcol + c;
      const int Q = Q0 + lcol + c;
      ra[c] = (m < M && P < N) ? load_b<CPLX_B>(bbase, rowoff + P) : make_double2(0.0, 0.0);
      double2 v;
      if (diag) v = ra[c];
      else v = (m < M && Q < N) ? load_b<CPLX_B>(bbase, rowoff + Q) : make_double2(0.0, 0.0);
      rb[c] = make_double2(w * v.x, w * v.y);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      lds[buf][0][lrow][lcol + c] = ra[c];
      lds[buf][1][lrow][lcol + c] = rb[c];
    }
  };

  const int wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;

  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      accR[x][y] = d4{0.0, 0.0, 0.0, 0.0};
      accI[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    }

  const int64_t nsteps = (M + KT - 1) / KT;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t s = 0; s < nsteps; ++s) {
    const int cur = (int)(s & 1);
    if (s + 1 < nsteps) gload((s + 1) * KT);
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks) {
      double2 av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = lds[cur][0][ks * 4 + lk][wr * 32 + x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = lds[cur][1][ks * 4 + lk][wc * 32 + y * 16 + li];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          // conj(a) * b = (ar br + ai bi) + i (ar bi - ai br)
          accR[x][y] = mfma(av[x].x, bv[y].x, accR[x][y]);
          accR[x][y] = mfma(av[x].y, bv[y].y, accR[x][y]);
          accI[x][y] = mfma(av[x].x, bv[y].y, accI[x][y]);
          accI[x][y] = mfma(-av[x].y, bv[y].x, accI[x][y]);
        }
    }
    if (s + 1 < nsteps) sstore(cur ^ 1);
    __syncthreads();
  }

  double2 *out = a.out + (int64_t)blockIdx.y * a.out_stride;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // f64 16x16x4 accumulator layout: register r of lane l holds row l/16 + 4 r, column l%16
        const int P = P0 + wr * 32 + x * 16 + lk + 4 * r;
        const int Q = Q0 + wc * 32 + y * 16 + li;
        if (P >= N || Q >= N) continue;
        const double re = accR[x][y][r];
        const double im = accI[x][y][r];
        if (diag) {
          if (P < Q) continue;
          if (P == Q) {
            out[(int64_t)P * N + Q] = make_double2(re, 0.0);
            continue;
          }
        }
        out[(int64_t)P * N + Q] = make_double2(re, im);
        out[(int64_t)Q * N + P] = make_double2(re, -im);
      }
}

}  // namespace

hipError_t launch_chi0_f64(hipStream_t s, const Chi0Args &a, int32_t npts, bool cplx_b) {
  if (npts <= 0) return hipSuccess;
  const int T = (a.N + TN - 1) / TN;
  const dim3 grid((unsigned)(T * (T + 1) / 2), (unsigned)npts);
  if (cplx_b)
    hipLaunchKernelGGL(chi0_f64_kernel<true>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(chi0_f64_kernel<false>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace rpa
