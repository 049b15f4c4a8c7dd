// Batched complex FP64 GEMM on the matrix cores for Pi = V^(1/2) chi0 V^(1/2)
// (Algorithm 1, "Z = V^0.5 P V^0.5"): two launches, T = chi0 V^(1/2) and
// Pi = V^(1/2) T, the second restricted to tiles on or below the diagonal because
// only the lower triangle of the Hermitian Pi feeds the Cholesky factorisation and
// the trace.
//
// Tiles are 64 x 64 complex per workgroup with K steps of 16; the left operand is
// transposed into LDS so that both MFMA operand fragments read 16 consecutive
// elements per K row.  Four waves own 32 x 32 sub-tiles (2 x 2 MFMA blocks).
#include "common.hpp"

namespace rpa {
namespace {

constexpr int TN = 64;
constexpr int KT = 16;
constexpr int LDP = TN + 1;

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

__global__ __launch_bounds__(256, 2) void zgemm_f64_kernel(GemmArgs g) {
  __shared__ double2 lA[2][KT][LDP];   // [k][i]
  __shared__ double2 lB[2][KT][LDP];   // [k][j]

  const int b = blockIdx.y;
  const int N = g.N;
  int tr, tc;
  if (g.lower_only) {
    tile_of((int)blockIdx.x, tr, tc);
  } else {
    const int T = (N + TN - 1) / TN;
    tr = (int)blockIdx.x / T;
    tc = (int)blockIdx.x - tr * T;
  }
  const int I0 = tr * TN, J0 = tc * TN;
  const int ai = g.a_map ? g.a_map[b] : b / g.a_div;
  const int bi = g.b_map ? g.b_map[b] : b / g.b_div;
  const double2 *A = g.A + (int64_t)ai * g.a_stride;
  const double2 *B = g.B + (int64_t)bi * g.b_stride;
  double2 *C = g.C + (int64_t)b * g.c_stride;

  const int tid = threadIdx.x;
  // A tile: 64 rows x 16 k; thread -> row tid/4, k (tid%4)*4 .. +3
  const int arow = tid >> 2, akc = (tid & 3) * 4;
  // B tile: 16 k x 64 cols; thread -> k tid/16, cols (tid%16)*4 .. +3
  const int brow = tid >> 4, bcol = (tid & 15) * 4;

  double2 ra[4], rb[4];
  auto gload = [&](int k0) {
    const int i = I0 + arow;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = k0 + akc + c;
      ra[c] = (i < N && k < N) ? A[(int64_t)i * N + k] : make_double2(0.0, 0.0);
    }
    const int kb = k0 + brow;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = J0 + bcol + c;
      rb[c] = (kb < N && j < N) ? B[(int64_t)kb * N + j] : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      lA[buf][akc + c][arow] = ra[c];
      lB[buf][brow][bcol + c] = rb[c];
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

  const int nsteps = (N + KT - 1) / KT;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    const int cur = s & 1;
    if (s + 1 < nsteps) gload((s + 1) * KT);
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks) {
      double2 av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = lA[cur][ks * 4 + lk][wr * 32 + x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = lB[cur][ks * 4 + lk][wc * 32 + y * 16 + li];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          // a * b = (ar br - ai bi) + i (ar bi + ai br)
          accR[x][y] = mfma(av[x].x, bv[y].x, accR[x][y]);
          accR[x][y] = mfma(-av[x].y, bv[y].y, accR[x][y]);
          accI[x][y] = mfma(av[x].x, bv[y].y, accI[x][y]);
          accI[x][y] = mfma(av[x].y, bv[y].x, accI[x][y]);
        }
    }
    if (s + 1 < nsteps) sstore(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I0 + wr * 32 + x * 16 + lk + 4 * r;
        const int j = J0 + wc * 32 + y * 16 + li;
        if (i < N && j < N) C[(int64_t)i * N + j] = make_double2(accR[x][y][r], accI[x][y][r]);
      }
}

}  // namespace

hipError_t launch_zgemm_f64(hipStream_t s, const GemmArgs &g, int32_t batch) {
  if (batch <= 0) return hipSuccess;
  const int T = (g.N + TN - 1) / TN;
  const unsigned tiles = g.lower_only ? (unsigned)(T * (T + 1) / 2) : (unsigned)(T * T);
  hipLaunchKernelGGL(zgemm_f64_kernel, dim3(tiles, (unsigned)batch), dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace rpa
