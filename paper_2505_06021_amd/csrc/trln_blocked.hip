// eps = ln det(1 - Pi) + Re Tr Pi for a batch of Hermitian Pi: blocked right-looking
// Cholesky spread over the whole GPU (the paper's log-det step of Algorithm 1, taken
// through a Cholesky factor of the Hermitian positive definite 1 - Pi).
//
// The batch is stored as W = -Pi (lower triangles, complex FP64, factored in place) and
// the identity is kept implicit: with d_c the updated diagonal entry of W, the pivot is
// 1 + d_c and 2 ln L_cc = log1p(d_c), exact to the last bit even when Pi is tiny.
//
// Per 64-column panel j0 of every matrix:
//   diagonal    factor the 64 x 64 diagonal block in LDS, accumulate log1p of its
//               pivots, and form the triangular inverse L11^-1 (one workgroup per
//               matrix; a launch of its own for the first block, else inside the
//               previous panel's update);
//   chol_panel  one workgroup per 64 rows below the block: L21 = W21 L11^-H as a
//               64 x 64 x 64 complex MFMA product;
//   chol_update one workgroup per 64 x 64 lower-triangle tile of the trailing matrix:
//               W22 -= L21 L21^H with v_mfma_f64_16x16x4f64; the workgroups of the
//               first trailing tile then factor it as the next diagonal block.
// A matrix whose pivot fails records the column in info[] and is skipped afterwards.
#include "common.hpp"

namespace rpa {
namespace {

constexpr int NB = 64;
constexpr int LP = NB + 1;   // LDS pitch: 16-byte reads of 16 consecutive rows hit distinct banks

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

// Load rows [r0, r0+64) x columns [c0, c0+kw) of an n x n matrix into lds[row][k]
// (zero outside the matrix or beyond kw).  Four lanes per row, 16 consecutive columns
// each, so a row's 1 KB is read contiguously.
__device__ __forceinline__ void load_block(double2 (*lds)[LP], const double2 *A, int n, int r0, int c0,
                                           int kw) {
  const int t = threadIdx.x;
  const int r = t >> 2, kq = (t & 3) * 16;
  const bool rv = r0 + r < n;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int k = kq + e;
    lds[r][k] = (rv && k < kw) ? A[(int64_t)(r0 + r) * n + c0 + k] : make_double2(0.0, 0.0);
  }
}

// acc[i][j] += sum_k A[i][k] conj(B[j][k]) over k < 64, for the 32 x 32 sub-tile of wave
// (wr, wc): 2 x 2 blocks of 16 x 16, lane (li, lk) of a block supplies row li, k = lk.
__device__ __forceinline__ void cgemm_nt(const double2 (*A)[LP], const double2 (*B)[LP], int wr, int wc,
                                         int li, int lk, d4 (&accR)[2][2], d4 (&accI)[2][2]) {
#pragma unroll 4
  for (int ks = 0; ks < NB / 4; ++ks) {
    double2 a[2], b[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) a[x] = A[wr * 32 + x * 16 + li][ks * 4 + lk];
#pragma unroll
    for (int y = 0; y < 2; ++y) b[y] = B[wc * 32 + y * 16 + li][ks * 4 + lk];
    // a conj(b) = (ar br + ai bi) + i (ai br - ar bi)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) accR[x][y] = mfma(a[x].x, b[y].x, accR[x][y]);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) accI[x][y] = mfma(a[x].y, b[y].x, accI[x][y]);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) accR[x][y] = mfma(a[x].y, b[y].y, accR[x][y]);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) accI[x][y] = mfma(-a[x].x, b[y].y, accI[x][y]);
  }
}

__global__ __launch_bounds__(256) void chol_init_kernel(const double2 *W, int64_t stride, int n, double *trace,
                                                        double *logacc, int32_t *info) {
  __shared__ double part[256];
  const double2 *A = W + (int64_t)blockIdx.x * stride;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += A[(int64_t)i * n + i].x;
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 256; ++i) t += part[i];
    trace[blockIdx.x] = t;       // Tr W = -Tr Pi
    logacc[blockIdx.x] = 0.0;
    info[blockIdx.x] = -1;
  }
}

// Factor the diagonal block at column j0 of matrix b (pivots 1 + d, log1p of them into
// logacc[b], the factor's inverse L11^-1 into linv); D and X are two NB x LP LDS arrays
// of the calling kernel.  A failing pivot records its column in info[b].  Called by the
// whole workgroup (every branch on the pivot is uniform).
__device__ __forceinline__ void diag_block(double2 *W, int64_t stride, int n, int j0, int b, double *logacc,
                                           int32_t *info, double2 *linv, double2 (*D)[LP], double2 (*X)[LP]) {
  __shared__ double2 colbuf[2][NB];
  __shared__ double ld[NB];
  double2 *A = W + (int64_t)b * stride;
  const int jb = min(NB, n - j0);
  const int tid = threadIdx.x;
  // Thread tid owns column s = tid % 64 and rows r = tid / 64 + 4 j (j < 16) of the block,
  // kept in registers; only the current pivot column passes through LDS.
  const int s = tid & 63, r0 = tid >> 6;
  double2 v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int r = r0 + 4 * j;
    v[j] = (r < jb && s <= r) ? A[(int64_t)(j0 + r) * n + j0 + s] : make_double2(0.0, 0.0);
  }
  for (int e = tid; e < NB * NB; e += 256) X[e / NB][e % NB] = make_double2(0.0, 0.0);
  // the pivots' d_c are kept in LDS; their square roots and log1p terms are taken after
  // the loop, in parallel, so no transcendental sits between two barriers
  __shared__ double dpiv[NB];
  for (int c = 0; c < jb; ++c) {
    double2 *cb = colbuf[c & 1];
    if (s == c) {
#pragma unroll
      for (int j = 0; j < 16; ++j) cb[r0 + 4 * j] = v[j];   // column c is final
    }
    __syncthreads();
    const double d = cb[c].x;
    const double piv = 1.0 + d;
    if (!(piv > 0.0) || !(piv < INFINITY)) {
      if (tid == 0) info[b] = j0 + c;
      return;   // uniform: every thread read the same pivot
    }
    if (tid == 0) dpiv[c] = d;
    if (s > c && s < jb) {
      // W[r][s] -= W[r][c] conj(W[s][c]) / piv for r >= s
      const double2 ys = cb[s];
      const double ip = 1.0 / piv;
      const double yr = ys.x * ip, yi = ys.y * ip;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int r = r0 + 4 * j;
        if (r >= s && r < jb) {
          const double2 x = cb[r];
          v[j].x -= x.x * yr + x.y * yi;
          v[j].y -= x.y * yr - x.x * yi;
        }
      }
    }
  }
  __syncthreads();
  if (tid < jb) {
    ld[tid] = sqrt(1.0 + dpiv[tid]);
    dpiv[tid] = log1p(dpiv[tid]);
  }
  __syncthreads();
  if (tid == 0) {
    // summed in column order, once per block: a global read-modify-write per column would
    // make every barrier wait for memory
    double lsum = 0.0;
    for (int c = 0; c < jb; ++c) lsum += dpiv[c];
    logacc[b] += lsum;
  }
  // the factor L11 into D: L[r][s] = W[r][s] / l_s below the diagonal, l_s on it
  {
    const double ls = s < jb ? ld[s] : 1.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int r = r0 + 4 * j;
      D[r][s] = (r < jb && s < r) ? make_double2(v[j].x / ls, v[j].y / ls)
                                  : (r == s && r < jb ? make_double2(ls, 0.0) : make_double2(0.0, 0.0));
    }
  }
  __syncthreads();
  // X = L11^{-1}, row by row: X[i][j] = -(sum_{k<i} L[i][k] X[k][j]) / l_i for j < i,
  // X[i][i] = 1 / l_i.  X is zero above its diagonal, so every lane can run over all
  // k < i: L[i][k] is a broadcast read, X[k][j] a conflict-free row read.  The 256
  // threads split k into four interleaved partitions summed in a fixed order; row i is
  // finished by the thread of partition i % 4, the only one that reads X[i][j] later, so
  // one barrier per row suffices (the partial sums alternate between two buffers).
  {
    __shared__ double2 part[2][4][NB];
    const int j = tid & 63, g = tid >> 6;
    if (tid < jb) X[tid][tid] = make_double2(1.0 / ld[tid], 0.0);
    __syncthreads();
    for (int i = 1; i < jb; ++i) {
      double sr = 0.0, si = 0.0;
      for (int k = g; k < i; k += 4) {
        const double2 lv = D[i][k], xv = X[k][j];
        sr += lv.x * xv.x - lv.y * xv.y;
        si += lv.x * xv.y + lv.y * xv.x;
      }
      double2 (*pp)[NB] = part[i & 1];
      pp[g][j] = make_double2(sr, si);
      __syncthreads();
      if (g == (i & 3) && j < i) {
        const double il = X[i][i].x;   // 1 / l_i
        const double r = (pp[0][j].x + pp[1][j].x) + (pp[2][j].x + pp[3][j].x);
        const double m = (pp[0][j].y + pp[1][j].y) + (pp[2][j].y + pp[3][j].y);
        X[i][j] = make_double2(-r * il, -m * il);
      }
    }
    __syncthreads();
  }
  double2 *out = linv + (int64_t)b * NB * NB;
  for (int e = tid; e < NB * NB; e += 256) out[e] = X[e / NB][e % NB];
}

__global__ __launch_bounds__(256) void chol_diag_kernel(double2 *W, int64_t stride, int n, int j0, double *logacc,
                                                        int32_t *info, double2 *linv) {
  __shared__ double2 D[NB][LP];
  __shared__ double2 X[NB][LP];
  const int b = blockIdx.x;
  if (info[b] >= 0) return;
  diag_block(W, stride, n, j0, b, logacc, info, linv, D, X);
}

__global__ __launch_bounds__(256) void chol_panel_kernel(double2 *W, int64_t stride, int n, int j0,
                                                         const int32_t *info, const double2 *linv) {
  __shared__ double2 Ab[NB][LP];
  __shared__ double2 Bb[NB][LP];
  const int b = blockIdx.y;
  if (info[b] >= 0) return;
  const int jb = min(NB, n - j0);
  const int r0 = j0 + jb + (int)blockIdx.x * NB;
  if (r0 >= n) return;
  double2 *A = W + (int64_t)b * stride;
  load_block(Ab, A, n, r0, j0, jb);
  {
    const double2 *L = linv + (int64_t)b * NB * NB;
    const int t = threadIdx.x;
    const int r = t >> 2, kq = (t & 3) * 16;
#pragma unroll
    for (int e = 0; e < 16; ++e) Bb[r][kq + e] = L[r * NB + kq + e];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) accR[x][y] = accI[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  cgemm_nt(Ab, Bb, wr, wc, li, lk, accR, accI);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wr * 32 + x * 16 + lk + 4 * r;
        const int col = wc * 32 + y * 16 + li;
        if (row < n && col < jb) A[(int64_t)row * n + j0 + col] = make_double2(accR[x][y][r], accI[x][y][r]);
      }
}

// Trailing update of panel j0 with a look-ahead: grid (matrix, tile), tile 0 (the next
// diagonal block) first for every matrix; the workgroups of tile 0 then factor that block
// for the next panel (what chol_diag would do in a launch of its own), so the latency-bound
// factorisation runs beside the other tiles' updates instead of after them.
__global__ __launch_bounds__(256) void chol_update_kernel(double2 *W, int64_t stride, int n, int j0,
                                                          int32_t *info, double *logacc, double2 *linv) {
  __shared__ double2 Ab[NB][LP];
  __shared__ double2 Bb[NB][LP];
  const int b = blockIdx.x;
  if (info[b] >= 0) return;
  const int jb = min(NB, n - j0);
  int tr, tc;
  tile_of((int)blockIdx.y, tr, tc);
  const int R0 = j0 + jb + tr * NB, S0 = j0 + jb + tc * NB;
  if (R0 >= n) return;
  double2 *A = W + (int64_t)b * stride;
  load_block(Ab, A, n, R0, j0, jb);
  if (tr != tc) load_block(Bb, A, n, S0, j0, jb);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) accR[x][y] = accI[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  cgemm_nt(Ab, tr != tc ? Bb : Ab, wr, wc, li, lk, accR, accI);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = R0 + wr * 32 + x * 16 + lk + 4 * r;
        const int col = S0 + wc * 32 + y * 16 + li;
        if (row < n && col <= row) {
          double2 *p = A + (int64_t)row * n + col;
          const double2 v = *p;
          *p = make_double2(v.x - accR[x][y][r], v.y - accI[x][y][r]);
        }
      }
  if (blockIdx.y == 0) {
    // the updated next diagonal block is in global memory, written by this workgroup:
    // the barrier orders those stores before the factorisation's loads
    __syncthreads();
    diag_block(W, stride, n, j0 + jb, b, logacc, info, linv, Ab, Bb);
  }
}

__global__ void chol_finish_kernel(const double *trace, const double *logacc, const int32_t *info, int batch,
                                   double *eps, int32_t *info_out, const int32_t *out_map) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int o = out_map ? out_map[b] : b;
  // eps = sum log1p(d_i) + Re Tr Pi, and Tr Pi = -Tr W
  eps[o] = info[b] >= 0 ? __builtin_nan("") : logacc[b] - trace[b];
  info_out[o] = info[b];
}

__global__ void negate_lower_kernel(double2 *P, int64_t stride, int n, int64_t total) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = g / ((int64_t)n * n);
    const int64_t e = g - b * (int64_t)n * n;
    const double2 v = P[b * stride + e];
    P[b * stride + e] = make_double2(-v.x, -v.y);
  }
}

}  // namespace

int64_t trln_blocked_scratch_bytes(int32_t batch) {
  return (int64_t)batch * (NB * NB * 16 + 3 * 8 + 8);
}

hipError_t launch_negate(hipStream_t s, double2 *p, int64_t stride, int32_t n, int32_t batch) {
  const int64_t total = (int64_t)batch * n * n;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(negate_lower_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, stride, n, total);
  return hipGetLastError();
}

hipError_t launch_trln_blocked(hipStream_t s, double2 *w, int64_t stride, int32_t n, int32_t batch, double *eps,
                               int32_t *info_out, const int32_t *out_map, void *scratch) {
  if (batch <= 0) return hipSuccess;
  char *p = (char *)scratch;
  double2 *linv = (double2 *)p;
  p += (int64_t)batch * NB * NB * 16;
  double *trace = (double *)p;
  p += (int64_t)batch * 8;
  double *logacc = (double *)p;
  p += (int64_t)batch * 8;
  int32_t *info = (int32_t *)p;
  hipLaunchKernelGGL(chol_init_kernel, dim3((unsigned)batch), dim3(256), 0, s, w, stride, n, trace, logacc, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the first diagonal block alone; every later one is factored inside the previous
  // panel's trailing update (look-ahead)
  hipLaunchKernelGGL(chol_diag_kernel, dim3((unsigned)batch), dim3(256), 0, s, w, stride, n, 0, logacc, info, linv);
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = n - j0 < NB ? n - j0 : NB;
    const int rest = n - j0 - jb;
    if (rest > 0) {
      const int nt = (rest + NB - 1) / NB;
      if (nt * (nt + 1) / 2 > 65535) return hipErrorInvalidValue;
      hipLaunchKernelGGL(chol_panel_kernel, dim3((unsigned)nt, (unsigned)batch), dim3(256), 0, s, w, stride, n, j0,
                         info, linv);
      hipLaunchKernelGGL(chol_update_kernel, dim3((unsigned)batch, (unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s,
                         w, stride, n, j0, info, logacc, linv);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(chol_finish_kernel, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, trace, logacc, info,
                     batch, eps, info_out, out_map);
  return hipGetLastError();
}

}  // namespace rpa
