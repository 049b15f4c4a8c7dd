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

// acc[i][j] += sum_k A[i][k] conj(B[j][k]) over k < K, for the 32 x 32 sub-tile of wave
// (wr, wc): 2 x 2 blocks of 16 x 16, lane (li, lk) of a block supplies row li, k = lk.
template <int K, int P>
__device__ __forceinline__ void cgemm_nt(const double2 (*A)[P], const double2 (*B)[P], int wr, int wc, int li,
                                         int lk, d4 (&accR)[2][2], d4 (&accI)[2][2]) {
#pragma unroll 4
  for (int ks = 0; ks < K / 4; ++ks) {
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

// Order this wave's LDS writes before its later LDS reads of other lanes' data (one wave
// issues its LDS instructions in order; the fences keep the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave: acc += A[ra + i][ca + k] conj(B[rb + j][cb + k]) over k < K (nt) or
// acc += A[ra + i][ca + k] B[rb + k][cb + j] (nn) for a 16 x 16 block; lane (li, lk)
// holds output rows lk + 4 r of column li.
template <bool NT>
__device__ __forceinline__ void mm16(const double2 (*A)[LP], int ra, int ca, const double2 (*B)[LP], int rb, int cb,
                                     int K, int li, int lk, d4 &accR, d4 &accI) {
  for (int k0 = 0; k0 < K; k0 += 4) {
    const double2 a = A[ra + li][ca + k0 + lk];
    const double2 b = NT ? B[rb + li][cb + k0 + lk] : B[rb + k0 + lk][cb + li];
    if (NT) {
      // a conj(b) = (ar br + ai bi) + i (ai br - ar bi)
      accR = mfma(a.x, b.x, accR);
      accR = mfma(a.y, b.y, accR);
      accI = mfma(a.y, b.x, accI);
      accI = mfma(-a.x, b.y, accI);
    } else {
      // a b = (ar br - ai bi) + i (ar bi + ai br)
      accR = mfma(a.x, b.x, accR);
      accR = mfma(-a.y, b.y, accR);
      accI = mfma(a.x, b.y, accI);
      accI = mfma(a.y, b.x, accI);
    }
  }
}

// Factor the 16 x 16 diagonal sub-block at (c0, c0) of D (already updated by the earlier
// sub-panels) and invert it, by one wave with no workgroup barrier.  Lane (j, g) keeps
// column j, rows g + 4 t (t < 4), of the block in v and of M in m, in registers; column c
// of W and row c of M go through LDS at step c.  The inverse is built alongside the
// factor (Gauss-Jordan): the elimination's row operations, applied to the identity, give
// M = U^-1 for the unit lower factor U of I + W = U diag(piv) U^H, and L^-1 =
// diag(piv)^-1/2 M.  On return D holds L there (l_c on the diagonal, zero above it), X
// the inverse, dpiv the pivots' d_c and lpiv their l_c; *fail the first failing column.
__device__ __forceinline__ void factor16(double2 (*D)[LP], double2 (*X)[LP], int c0, int lane, double *dpiv,
                                         double *lpiv, double2 (*colbuf)[16], double2 (*rowbuf)[16], int *fail) {
  const int j = lane & 15, g = lane >> 4;
  double2 v[4], m[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i = g + 4 * t;
    v[t] = i >= j ? D[c0 + i][c0 + j] : make_double2(0.0, 0.0);
    m[t] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    double2 *cb = colbuf[c & 1], *rb = rowbuf[c & 1];
    if (j == c) {
#pragma unroll
      for (int t = 0; t < 4; ++t) cb[g + 4 * t] = v[t];   // column c of W is final
    }
    if (g == (c & 3)) rb[j] = m[c >> 2];                  // so is row c of M
    wave_lds_sync();
    const double d = cb[c].x;
    const double piv = 1.0 + d;
    if (!(piv > 0.0) || !(piv < INFINITY)) {
      if (lane == 0) *fail = c0 + c;
      return;   // uniform: every lane read the same pivot
    }
    if (lane == 0) dpiv[c0 + c] = d;
    const double ip = 1.0 / piv;
    const double2 mc = rb[j];
    const double2 ys = cb[j];
    const double yr = ys.x * ip, yi = ys.y * ip;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = g + 4 * t;
      if (i > c) {
        const double2 x = cb[i];
        // M[i][j] -= (W[i][c] / piv) M[c][j]
        const double ur = x.x * ip, ui = x.y * ip;
        m[t].x -= ur * mc.x - ui * mc.y;
        m[t].y -= ur * mc.y + ui * mc.x;
        // W[i][j] -= W[i][c] conj(W[j][c]) / piv for i >= j > c
        if (j > c && i >= j) {
          v[t].x -= x.x * yr + x.y * yi;
          v[t].y -= x.y * yr - x.x * yi;
        }
      }
    }
  }
  if (lane < 16) lpiv[c0 + lane] = sqrt(1.0 + dpiv[c0 + lane]);
  wave_lds_sync();
  // L[i][j] = W[i][j] / l_j below the diagonal, l_j on it; X[i][j] = M[i][j] / l_i
  const double lj = lpiv[c0 + j];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i = g + 4 * t;
    const double li = lpiv[c0 + i];
    D[c0 + i][c0 + j] = i > j ? make_double2(v[t].x / lj, v[t].y / lj)
                              : (i == j ? make_double2(lj, 0.0) : make_double2(0.0, 0.0));
    X[c0 + i][c0 + j] = i >= j ? make_double2(m[t].x / li, m[t].y / li) : make_double2(0.0, 0.0);
  }
}

// Factor the diagonal block at column j0 of matrix b (pivots 1 + d, log1p of them into
// logacc[b], the factor's inverse L11^-1 into linv); D and X are two NB x LP LDS arrays
// of the calling kernel.  A failing pivot records its column in info[b].  Called by the
// whole workgroup.
//
// The block is factored in four 16-column sub-panels p (right-looking, with its inverse
// built alongside):  (a) one wave factors and inverts the 16 x 16 diagonal sub-block;
// (b) the sub-panel below it, L_qp = W_qp X_pp^H, and T_pj = sum_{j<=k<p} L_pk X_kj for
// the inverse's row p, as 16 x 16 complex MFMA products spread over the waves; (c) the
// trailing update W_ab -= L_ap L_bp^H of the sub-blocks to the right, and the inverse's
// row p, X_pj = -X_pp T_pj.  Three workgroup barriers per sub-panel.  Rows and columns at
// and beyond jb hold zeros: their pivots are 1 and add log1p(0) = 0.
__device__ __forceinline__ void diag_block(double2 *W, int64_t stride, int n, int j0, int b, double *logacc,
                                           int32_t *info, double2 *linv, double2 (*D)[LP], double2 (*X)[LP]) {
  __shared__ double2 colbuf[2][16], rowbuf[2][16];
  __shared__ double dpiv[NB], lpiv[NB];
  __shared__ int fail;
  double2 *A = W + (int64_t)b * stride;
  const int jb = min(NB, n - j0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e / NB, s = e % NB;
    D[r][s] = (r < jb && s <= r) ? A[(int64_t)(j0 + r) * n + j0 + s] : make_double2(0.0, 0.0);
    X[r][s] = make_double2(0.0, 0.0);
  }
  if (tid < NB) dpiv[tid] = 0.0;
  if (tid == 0) fail = -1;
  __syncthreads();
  const int np = (jb + 15) / 16;
  for (int p = 0; p < np; ++p) {
    const int c0 = 16 * p;
    // (a)
    if (wave == 0) factor16(D, X, c0, lane, dpiv, lpiv, colbuf, rowbuf, &fail);
    __syncthreads();
    if (fail >= 0) {
      if (tid == 0) info[b] = j0 + fail;
      return;   // uniform
    }
    // (b) tasks: sub-panel blocks q = p+1..3, then T_pj for j = 0..p-1
    {
      const int npanel = 3 - p;
      for (int task = wave; task < npanel + p; task += 4) {
        d4 accR = {0.0, 0.0, 0.0, 0.0}, accI = {0.0, 0.0, 0.0, 0.0};
        int r0, cc;
        if (task < npanel) {
          r0 = 16 * (p + 1 + task);
          cc = c0;
          mm16<true>(D, r0, c0, X, c0, c0, 16, li, lk, accR, accI);
        } else {
          const int jj = task - npanel;
          r0 = c0;
          cc = 16 * jj;
          mm16<false>(D, c0, 16 * jj, X, 16 * jj, 16 * jj, 16 * (p - jj), li, lk, accR, accI);
        }
        double2 (*O)[LP] = task < npanel ? D : X;
#pragma unroll
        for (int r = 0; r < 4; ++r) O[r0 + lk + 4 * r][cc + li] = make_double2(accR[r], accI[r]);
      }
    }
    __syncthreads();
    // (c) tasks: trailing blocks (a, b) with p < b <= a <= 3, then X_pj = -X_pp T_pj
    {
      const int m = 3 - p, ntrail = m * (m + 1) / 2;
      for (int task = wave; task < ntrail + p; task += 4) {
        d4 accR = {0.0, 0.0, 0.0, 0.0}, accI = {0.0, 0.0, 0.0, 0.0};
        if (task < ntrail) {
          int ta, tb;
          tile_of(task, ta, tb);
          const int ra = 16 * (p + 1 + ta), rb = 16 * (p + 1 + tb);
          mm16<true>(D, ra, c0, D, rb, c0, 16, li, lk, accR, accI);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double2 &w = D[ra + lk + 4 * r][rb + li];
            w = make_double2(w.x - accR[r], w.y - accI[r]);
          }
        } else {
          const int jj = task - ntrail;
          mm16<false>(X, c0, c0, X, c0, 16 * jj, 16, li, lk, accR, accI);
#pragma unroll
          for (int r = 0; r < 4; ++r) X[c0 + lk + 4 * r][16 * jj + li] = make_double2(-accR[r], -accI[r]);
        }
      }
    }
    __syncthreads();
  }
  if (tid < jb) dpiv[tid] = log1p(dpiv[tid]);
  __syncthreads();
  if (tid == 0) {
    // summed in column order, once per block
    double lsum = 0.0;
    for (int c = 0; c < jb; ++c) lsum += dpiv[c];
    logacc[b] += lsum;
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

// The 64 x 64 tile products of the panel and update kernels stream their K = 64 columns
// in chunks of KC = 16: each chunk of both operands goes HBM -> registers -> LDS one chunk
// ahead of the MFMAs that use it (double-buffered), so the loads of a chunk overlap the
// products of the previous one.  Thread t stages row t / 4 and four consecutive columns.
constexpr int KC = 16;
constexpr int LPC = KC + 1;
typedef double2 Chunk[NB][LPC];

struct ChunkStage {
  double2 ra[4], rb[4];
  // rows [ra0, ra0 + 64) of A and [rb0, rb0 + 64) of B (pitches lda, ldb), columns
  // [ca0 + KC kc, ...) and [cb0 + KC kc, ...); zero outside rows < nra (A), < nrb (B) and
  // columns < kw
  __device__ __forceinline__ void fetch(const double2 *A, int64_t lda, int ra0, int ca0, int nra, const double2 *B,
                                        int64_t ldb, int rb0, int cb0, int nrb, bool has_b, int kw, int kc) {
    const int t = threadIdx.x, r = t >> 2, q = (t & 3) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = kc * KC + q + e;
      ra[e] = (ra0 + r < nra && k < kw) ? A[(int64_t)(ra0 + r) * lda + ca0 + k] : make_double2(0.0, 0.0);
      if (has_b) rb[e] = (rb0 + r < nrb && k < kw) ? B[(int64_t)(rb0 + r) * ldb + cb0 + k] : make_double2(0.0, 0.0);
    }
  }
  __device__ __forceinline__ void put(Chunk &ca, Chunk &cb, bool has_b) {
    const int t = threadIdx.x, r = t >> 2, q = (t & 3) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ca[r][q + e] = ra[e];
      if (has_b) cb[r][q + e] = rb[e];
    }
  }
};

// acc += A B^H over k < kw for a 64 x 64 tile, A and B as above (B = A when !has_b); the
// chunk buffers ca[2], cb[2] are LDS of the caller.  Ends with a barrier.
__device__ __forceinline__ void tile_product(const double2 *A, int64_t lda, int ra0, int ca0, int nra,
                                             const double2 *B, int64_t ldb, int rb0, int cb0, int nrb, bool has_b,
                                             int kw, Chunk *ca, Chunk *cb, d4 (&accR)[2][2], d4 (&accI)[2][2]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
  const int nk = (kw + KC - 1) / KC;
  ChunkStage st;
  st.fetch(A, lda, ra0, ca0, nra, B, ldb, rb0, cb0, nrb, has_b, kw, 0);
  st.put(ca[0], cb[0], has_b);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int cur = kc & 1;
    if (kc + 1 < nk) st.fetch(A, lda, ra0, ca0, nra, B, ldb, rb0, cb0, nrb, has_b, kw, kc + 1);
    __builtin_amdgcn_sched_barrier(0);
    cgemm_nt<KC, LPC>(ca[cur], has_b ? cb[cur] : ca[cur], wr, wc, li, lk, accR, accI);
    __builtin_amdgcn_sched_barrier(0);
    if (kc + 1 < nk) st.put(ca[cur ^ 1], cb[cur ^ 1], has_b);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void chol_panel_kernel(double2 *W, int64_t stride, int n, int j0,
                                                         const int32_t *info, const double2 *linv) {
  __shared__ Chunk ca[2], cb[2];   // 70 KB: two workgroups per CU
  const int b = blockIdx.y;
  if (info[b] >= 0) return;
  const int jb = min(NB, n - j0);
  const int r0 = j0 + jb + (int)blockIdx.x * NB;
  if (r0 >= n) return;
  double2 *A = W + (int64_t)b * stride;
  const double2 *L = linv + (int64_t)b * NB * NB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) accR[x][y] = accI[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  // L21 = W21 (L11^-1)^H: rows of W21 against the 64 rows of L11^-1 (columns < jb; the
  // inverse is zero beyond)
  tile_product(A, n, r0, j0, n, L, NB, 0, 0, NB, true, jb, ca, cb, accR, accI);
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
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
  // the tile's current values, fetched now so that their latency hides behind the product
  double2 old[2][2][4];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = R0 + wr * 32 + x * 16 + lk + 4 * r;
        const int col = S0 + wc * 32 + y * 16 + li;
        old[x][y][r] = (row < n && col <= row) ? A[(int64_t)row * n + col] : make_double2(0.0, 0.0);
      }
  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) accR[x][y] = accI[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  // W22 -= L21 L21^H: the chunk buffers live in the diagonal factor's LDS arrays
  Chunk *ca = reinterpret_cast<Chunk *>(&Ab[0][0]);
  Chunk *cb = reinterpret_cast<Chunk *>(&Bb[0][0]);
  tile_product(A, n, R0, j0, n, A, n, S0, j0, n, tr != tc, jb, ca, cb, accR, accI);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = R0 + wr * 32 + x * 16 + lk + 4 * r;
        const int col = S0 + wc * 32 + y * 16 + li;
        if (row < n && col <= row)
          A[(int64_t)row * n + col] = make_double2(old[x][y][r].x - accR[x][y][r], old[x][y][r].y - accI[x][y][r]);
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
