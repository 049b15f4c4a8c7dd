// Batched complex FP64 GEMM on the matrix cores for Pi = V^(1/2) chi0 V^(1/2)
// (Algorithm 1, the sandwich step): two launches, T = chi0 V^(1/2) and
// Pi = V^(1/2) T, the second restricted to tiles on or below the diagonal because
// only the lower triangle of the Hermitian Pi feeds the Cholesky factorisation and
// the trace.
//
// Tiles are 64 x 64 complex per workgroup with double-buffered K steps of 16; the next
// step's loads are issued ahead of the MFMA block.  Four waves own 32 x 32 sub-tiles
// (2 x 2 MFMA blocks, four real products per complex block).
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

struct GStage {
  double2 a[4], b[4];
};

// A tile [64 rows][16 k] and B tile [16 k][64 columns], both stored as read from memory:
// with the padded pitches, the MFMA fragment reads of 16 lanes on consecutive rows (A)
// or columns (B) hit distinct banks, so no transpose is needed.  Loads use clamped
// (always valid) addresses and are masked at the LDS store.
__device__ __forceinline__ void gemm_load(GStage &st, const double2 *A, const double2 *B, int N, int k0,
                                          int ai_row, int ak, int bk, const int (&bcol)[4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int k = k0 + ak + c;
    st.a[c] = A[(int64_t)ai_row * N + (k < N ? k : 0)];
  }
  const int kb = k0 + bk;
  const int64_t ro = (int64_t)(kb < N ? kb : 0) * N;
#pragma unroll
  for (int c = 0; c < 4; ++c) st.b[c] = B[ro + bcol[c]];
}

// component-wise select: a select of whole double2 values can become a pointer select
// through scratch memory
__device__ __forceinline__ double2 keep_if(bool ok, const double2 &v) {
  return make_double2(ok ? v.x : 0.0, ok ? v.y : 0.0);
}

__device__ __forceinline__ void gemm_store(const GStage &st, double2 (*la)[KT + 1], double2 (*lb)[LDP], int N,
                                           int k0, int arow, bool arow_ok, int ak, int bk, const bool (&bok)[4],
                                           int bc) {
#pragma unroll
  for (int c = 0; c < 4; ++c) la[arow][ak + c] = keep_if(arow_ok && k0 + ak + c < N, st.a[c]);
  const bool kv = k0 + bk < N;
#pragma unroll
  for (int c = 0; c < 4; ++c) lb[bk][bc + 16 * c] = keep_if(kv && bok[c], st.b[c]);
}

__device__ __forceinline__ void gemm_contract(const double2 (*la)[KT + 1], const double2 (*lb)[LDP], int wr, int wc,
                                              int li, int lk, d4 (&accR)[2][2], d4 (&accI)[2][2]) {
#pragma unroll
  for (int ks = 0; ks < KT / 4; ++ks) {
    double2 av[2], bv[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) av[x] = la[wr * 32 + x * 16 + li][ks * 4 + lk];
#pragma unroll
    for (int y = 0; y < 2; ++y) bv[y] = lb[ks * 4 + lk][wc * 32 + y * 16 + li];
    // a * b = (ar br - ai bi) + i (ar bi + ai br)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) accR[x][y] = mfma(av[x].x, bv[y].x, accR[x][y]);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) accI[x][y] = mfma(av[x].x, bv[y].y, accI[x][y]);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) accR[x][y] = mfma(-av[x].y, bv[y].y, accR[x][y]);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) accI[x][y] = mfma(av[x].y, bv[y].x, accI[x][y]);
  }
}

__global__ __launch_bounds__(256) void zgemm_f64_kernel(GemmArgs g) {
  __shared__ double2 lA[2][TN][KT + 1];   // [i][k]
  __shared__ double2 lB[2][KT][LDP];      // [k][j]

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
  const int arow = tid >> 2, ak = (tid & 3) * 4;       // A: row, 4 consecutive k
  const bool arow_ok = I0 + arow < N;
  const int ai_row = arow_ok ? I0 + arow : 0;
  const int bk = tid >> 4, bc = tid & 15;               // B: k row, columns bc + 16 c
  int bcol[4];
  bool bok[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = J0 + bc + 16 * c;
    bok[c] = j < N;
    bcol[c] = bok[c] ? j : 0;
  }

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

  GStage st;
  const int nsteps = (N + KT - 1) / KT;
  gemm_load(st, A, B, N, 0, ai_row, ak, bk, bcol);
  gemm_store(st, lA[0], lB[0], N, 0, arow, arow_ok, ak, bk, bok, bc);
  __syncthreads();
  for (int s = 0; s + 1 < nsteps; ++s) {
    const int cur = s & 1;
    gemm_load(st, A, B, N, (s + 1) * KT, ai_row, ak, bk, bcol);
    __builtin_amdgcn_sched_barrier(0);
    gemm_contract(lA[cur], lB[cur], wr, wc, li, lk, accR, accI);
    __builtin_amdgcn_sched_barrier(0);
    gemm_store(st, lA[cur ^ 1], lB[cur ^ 1], N, (s + 1) * KT, arow, arow_ok, ak, bk, bok, bc);
    __syncthreads();
  }
  gemm_contract(lA[(nsteps - 1) & 1], lB[(nsteps - 1) & 1], wr, wc, li, lk, accR, accI);

  const double sg = g.negate ? -1.0 : 1.0;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I0 + wr * 32 + x * 16 + lk + 4 * r;
        const int j = J0 + wc * 32 + y * 16 + li;
        if (i < N && j < N) C[(int64_t)i * N + j] = make_double2(sg * accR[x][y][r], sg * accI[x][y][r]);
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
