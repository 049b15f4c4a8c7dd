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
// q-group shares one launch.  The contraction runs in K steps of KT rows (8, 16 or 32):
// sixteen lanes load one row of both operand panels, the right operand is multiplied by
// w_m zeta_k in registers (from a per-point table of the transition weights), and both
// panels go to a double-buffered LDS tile.  Four waves each own a 32 x 32 sub-tile (2 x 2 MFMA blocks, Re and Im
// accumulators).  Off-diagonal tiles also store their conjugate transpose, so the full
// Hermitian matrix is produced from the lower-triangle work only.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace rpa {
namespace {

constexpr int TN = 64;        // output tile edge (complex elements)
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

// w_m zeta_k for every contraction row m of every point of a launch (Delta and the
// frequency weight of the polarizability equation), one table row per point.
__global__ __launch_bounds__(256) void weight_table_kernel(Chi0Args a, int32_t npts) {
  const int nov = a.nocc * a.nvirt;
  const int64_t total = (int64_t)npts * a.M;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(g / a.M);
    const int m = (int)(g - (int64_t)p * a.M);
    const PointDesc pd = a.pts[p];
    const int kr = m / nov;   // k-point of the row, relative to the rows' first one
    const int rem = m - kr * nov;
    const int k = a.k0 + kr;
    const int i = rem / a.nvirt;
    const int av = rem - i * a.nvirt;
    const int kq = a.kq[(int64_t)pd.q * a.nk + k];
    const double d = a.eps_virt[(int64_t)k * a.nvirt + av] - a.eps_occ[(int64_t)kq * a.nocc + i];
    a.wtab[g] = -4.0 * a.zeta_k[k] * d / (d * d + pd.omega * pd.omega);
  }
}

// Per-thread loader state: 16 lanes per row, lane lc loads columns lc, lc+16, lc+32,
// lc+48 of both operand panels, so each load instruction of 16 lanes reads 256
// contiguous bytes and the LDS stores are conflict-free.
template <int NPASS>
struct Stage {
  double2 a[NPASS][4], b[NPASS][4];
  double w[NPASS];
  bool mv[NPASS];
};

// Raw loads only: nothing consumes them until store_stage() after the MFMA block, so
// they stay in flight while the current tile is contracted.  Out-of-range rows and
// columns read a clamped (valid) address and are zeroed at the store.
template <bool CPLX_B, int NPASS, int RPI>
__device__ __forceinline__ void load_stage(Stage<NPASS> &st, const char *bbase, const double *wrow,
                                           int m0, int lrow, bool row_active, int M, int N,
                                           const int (&pcol)[4], const int (&qcol)[4]) {
#pragma unroll
  for (int ps = 0; ps < NPASS; ++ps) {
    const int m = m0 + ps * RPI + lrow;
    st.mv[ps] = row_active && m < M;
    const int mc = st.mv[ps] ? m : 0;
    st.w[ps] = wrow[mc];
    const int64_t rowoff = (int64_t)mc * N;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      st.a[ps][c] = load_b<CPLX_B>(bbase, rowoff + pcol[c]);
      st.b[ps][c] = load_b<CPLX_B>(bbase, rowoff + qcol[c]);
    }
  }
}

template <int KT, int NPASS, int RPI>
__device__ __forceinline__ void store_stage(const Stage<NPASS> &st, double2 (*la)[LDP],
                                            double2 (*lb)[LDP], int lrow, int lc, bool row_active,
                                            const bool (&pok)[4], const bool (&qok)[4]) {
  if (!row_active) return;
#pragma unroll
  for (int ps = 0; ps < NPASS; ++ps) {
    const double w = st.mv[ps] ? st.w[ps] : 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double2 z = make_double2(0.0, 0.0);
      const double2 a = (st.mv[ps] && pok[c]) ? st.a[ps][c] : z;
      const double2 b = qok[c] ? st.b[ps][c] : z;
      la[ps * RPI + lrow][lc + 16 * c] = a;
      lb[ps * RPI + lrow][lc + 16 * c] = make_double2(w * b.x, w * b.y);
    }
  }
}

// One K step of the 2 x 2 block of 16 x 16 complex products owned by a wave:
// acc += conj(A)^T (w B) over the KT rows held in LDS.
template <int KT>
__device__ __forceinline__ void contract(const double2 (*la)[LDP], const double2 (*lb)[LDP], int wr,
                                         int wc, int li, int lk, d4 (&accR)[2][2], d4 (&accI)[2][2]) {
#pragma unroll
  for (int ks = 0; ks < KT / 4; ++ks) {
    double2 av[2], bv[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) av[x] = la[ks * 4 + lk][wr * 32 + x * 16 + li];
#pragma unroll
    for (int y = 0; y < 2; ++y) bv[y] = lb[ks * 4 + lk][wc * 32 + y * 16 + li];
    // conj(a) * b = (ar br + ai bi) + i (ar bi - ai br); the four products of a block are
    // issued with the other blocks' products in between, so no MFMA waits on its
    // predecessor's accumulator.
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
      for (int y = 0; y < 2; ++y) accR[x][y] = mfma(av[x].y, bv[y].y, accR[x][y]);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) accI[x][y] = mfma(-av[x].y, bv[y].x, accI[x][y]);
  }
}

// The same K step for the waves of a diagonal tile, where only the blocks in the 4-bit
// mask `on` (bit 2x + y) are computed.  The mask is uniform over the wave.
template <int KT>
__device__ __forceinline__ void contract_masked(const double2 (*la)[LDP], const double2 (*lb)[LDP], int wr,
                                                int wc, int li, int lk, int on, d4 (&accR)[2][2],
                                                d4 (&accI)[2][2]) {
#pragma unroll
  for (int ks = 0; ks < KT / 4; ++ks) {
    double2 av[2], bv[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) av[x] = la[ks * 4 + lk][wr * 32 + x * 16 + li];
#pragma unroll
    for (int y = 0; y < 2; ++y) bv[y] = lb[ks * 4 + lk][wc * 32 + y * 16 + li];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        if (on & (1 << (2 * x + y))) accR[x][y] = mfma(av[x].x, bv[y].x, accR[x][y]);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        if (on & (1 << (2 * x + y))) accI[x][y] = mfma(av[x].x, bv[y].y, accI[x][y]);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        if (on & (1 << (2 * x + y))) accR[x][y] = mfma(av[x].y, bv[y].y, accR[x][y]);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        if (on & (1 << (2 * x + y))) accI[x][y] = mfma(-av[x].y, bv[y].x, accI[x][y]);
  }
}

template <bool CPLX_B, int KT>
__global__ __launch_bounds__(256) void chi0_f64_kernel(Chi0Args a) {
  __shared__ double2 lds[2][2][KT][LDP];
  constexpr int RPI = 256 / 16;               // rows covered by one pass of the workgroup
  constexpr int NPASS = KT / RPI > 0 ? KT / RPI : 1;

  const PointDesc pd = a.pts[blockIdx.y];
  int tr, tc;
  tile_of((int)blockIdx.x, tr, tc);
  const int N = a.N;
  // rows [mlo, mhi) of the contraction belong to split blockIdx.z
  const int ms = (int)((((a.M + a.ksplit - 1) / a.ksplit) + KT - 1) / KT) * KT;
  const int mlo = (int)blockIdx.z * ms;
  const int mhi = mlo + ms < (int)a.M ? mlo + ms : (int)a.M;
  const int M = mhi;
  const int P0 = tr * TN, Q0 = tc * TN;
  const bool diag = (tr == tc);

  const int tid = threadIdx.x;
  const int lrow = tid >> 4;
  const int lc = tid & 15;
  const bool row_active = lrow < KT;

  const char *bbase = reinterpret_cast<const char *>(a.B) +
                      (int64_t)pd.bslot * a.b_slot_stride * (CPLX_B ? 16 : 8);
  const double *wrow = a.wtab + (int64_t)blockIdx.y * a.M;

  // column validity and clamped column indices are fixed for the whole contraction
  int pcol[4], qcol[4];
  bool pok[4], qok[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int P = P0 + lc + 16 * c, Q = Q0 + lc + 16 * c;
    pok[c] = P < N;
    qok[c] = Q < N;
    pcol[c] = pok[c] ? P : 0;
    qcol[c] = qok[c] ? Q : 0;
  }

  const int wave = tid >> 6, lane = tid & 63;
  int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  // Diagonal tiles: the upper 32 x 32 quadrant mirrors the lower one, so its wave (0, 1)
  // takes the second 16-column half of the lower quadrant from wave (1, 0), and the two
  // diagonal quadrants skip their strictly upper 16 x 16 block.  The busiest wave then
  // issues 3 of 4 blocks' products (each block summed exactly as before).
  int on = 0xf;   // blocks (x, y) of the wave's quadrant it computes: bit 2x + y
  if (diag) {
    if (wr == 0 && wc == 1) {
      wr = 1;
      wc = 0;
      on = 0xa;   // y = 1 of the lower quadrant
    } else if (wr == 1 && wc == 0) {
      on = 0x5;   // y = 0 of the lower quadrant
    } else {
      on = 0xd;   // diagonal quadrant without block (0, 1)
    }
  }

  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      accR[x][y] = d4{0.0, 0.0, 0.0, 0.0};
      accI[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    }

  Stage<NPASS> st;
  const int nsteps = mhi > mlo ? (mhi - mlo + KT - 1) / KT : 1;
  load_stage<CPLX_B, NPASS, RPI>(st, bbase, wrow, mlo, lrow, row_active, M, N, pcol, qcol);
  store_stage<KT, NPASS, RPI>(st, lds[0][0], lds[0][1], lrow, lc, row_active, pok, qok);
  __syncthreads();
  if (!diag) {
    for (int s = 0; s + 1 < nsteps; ++s) {
      const int cur = s & 1;
      load_stage<CPLX_B, NPASS, RPI>(st, bbase, wrow, mlo + (s + 1) * KT, lrow, row_active, M, N, pcol, qcol);
      // keep the next tile's loads issued ahead of the MFMA block (their latency hides under it)
      __builtin_amdgcn_sched_barrier(0);
      contract<KT>(lds[cur][0], lds[cur][1], wr, wc, li, lk, accR, accI);
      __builtin_amdgcn_sched_barrier(0);
      store_stage<KT, NPASS, RPI>(st, lds[cur ^ 1][0], lds[cur ^ 1][1], lrow, lc, row_active, pok, qok);
      __syncthreads();
    }
    contract<KT>(lds[(nsteps - 1) & 1][0], lds[(nsteps - 1) & 1][1], wr, wc, li, lk, accR, accI);
  } else {
    for (int s = 0; s + 1 < nsteps; ++s) {
      const int cur = s & 1;
      load_stage<CPLX_B, NPASS, RPI>(st, bbase, wrow, mlo + (s + 1) * KT, lrow, row_active, M, N, pcol, qcol);
      __builtin_amdgcn_sched_barrier(0);
      contract_masked<KT>(lds[cur][0], lds[cur][1], wr, wc, li, lk, on, accR, accI);
      __builtin_amdgcn_sched_barrier(0);
      store_stage<KT, NPASS, RPI>(st, lds[cur ^ 1][0], lds[cur ^ 1][1], lrow, lc, row_active, pok, qok);
      __syncthreads();
    }
    contract_masked<KT>(lds[(nsteps - 1) & 1][0], lds[(nsteps - 1) & 1][1], wr, wc, li, lk, on, accR, accI);
  }

  double2 *out = (blockIdx.z == 0 ? a.out : a.partial + (int64_t)(blockIdx.z - 1) * a.split_stride) +
                 (int64_t)blockIdx.y * a.out_stride;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // f64 16x16x4 accumulator layout: register r of lane l holds row l/16 + 4 r, column l%16
        const int P = P0 + wr * 32 + x * 16 + lk + 4 * r;
        const int Q = Q0 + wc * 32 + y * 16 + li;
        if (P >= N || Q >= N || !(on & (1 << (2 * x + y)))) continue;
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

// Diagonal tiles of the paired kernel: the ten 16 x 16 blocks on or below the diagonal
// of a 64 x 64 tile, split five and five between two waves per point ("roles"); block u
// of role R is (DIAG_BX[R][u], DIAG_BY[R][u]) in 16-row/column units.  Each block takes
// the single-point kernel's four products per 4-row sub-step in the same order.
__device__ constexpr int DIAG_BX[2][5] = {{0, 1, 1, 2, 3}, {2, 2, 3, 3, 3}};
__device__ constexpr int DIAG_BY[2][5] = {{0, 0, 1, 0, 0}, {1, 2, 1, 2, 3}};

template <int ROLE>
__device__ __forceinline__ void contract_diag5(const double2 (*la)[LDP], const double2 (*lb)[LDP], const double *lwp,
                                               int li, int lk, d4 (&dR)[5], d4 (&dI)[5]) {
  constexpr bool needA[4] = {ROLE == 0, ROLE == 0, true, true};
  constexpr bool needB[4] = {ROLE == 0, true, ROLE == 1, ROLE == 1};
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int r = ks * 4 + lk;
    double2 av[4], bw[4];
    const double w = lwp[r];
#pragma unroll
    for (int x = 0; x < 4; ++x)
      if (needA[x]) av[x] = la[r][x * 16 + li];
#pragma unroll
    for (int y = 0; y < 4; ++y)
      if (needB[y]) {
        const double2 b = lb[r][y * 16 + li];
        bw[y] = make_double2(w * b.x, w * b.y);
      }
#pragma unroll
    for (int u = 0; u < 5; ++u) dR[u] = mfma(av[DIAG_BX[ROLE][u]].x, bw[DIAG_BY[ROLE][u]].x, dR[u]);
#pragma unroll
    for (int u = 0; u < 5; ++u) dI[u] = mfma(av[DIAG_BX[ROLE][u]].x, bw[DIAG_BY[ROLE][u]].y, dI[u]);
#pragma unroll
    for (int u = 0; u < 5; ++u) dR[u] = mfma(av[DIAG_BX[ROLE][u]].y, bw[DIAG_BY[ROLE][u]].y, dR[u]);
#pragma unroll
    for (int u = 0; u < 5; ++u) dI[u] = mfma(-av[DIAG_BX[ROLE][u]].y, bw[DIAG_BY[ROLE][u]].x, dI[u]);
  }
}

// Two frequencies of one q per workgroup.  The points of a q read the same coefficient
// slab and differ only in the weights w_m zeta_k, so a workgroup stages the unweighted
// panels of a 64 x 64 tile once and contracts them for both points: each lane scales its
// right-operand fragments by the two points' weights of its row (the same double product
// w * b the single-point kernel forms before its LDS store, so the sums are bit for bit
// those of that kernel) and the wave issues the MFMAs of both points.  Per loaded byte and
// per barrier this does twice the MFMA work of the single-point kernel at the same LDS
// footprint (two workgroups per CU).  A workgroup serves pair j of the launch's pair
// table (points a.pairs[2 j] and a.pairs[2 j + 1], on the same slab; a second index of
// -1 leaves the pair single).
// In diagonal tiles waves 0 and 1 take point 0's ten lower blocks, five each, and waves
// 2 and 3 point 1's, so the busiest wave issues 5/8 of an off-diagonal tile's products.
// A launch of the paired kernel holds up to CHI0_MAX_GROUPS groups (the point batches of
// one job, or of several jobs of the serving loop launched together); group i owns the
// workgroups [begin[i], begin[i + 1]) of the one-dimensional grid and is contracted
// exactly as it would be alone.
struct Chi0Launch {
  int32_t ngroups;
  int32_t begin[CHI0_MAX_GROUPS + 1];
  Chi0Args g[CHI0_MAX_GROUPS];
};

template <bool CPLX_B>
__global__ __launch_bounds__(256) void chi0_f64_w2_kernel(Chi0Launch L) {
  constexpr int KT = 16;
  __shared__ double2 lds[2][2][KT][LDP];
  __shared__ double lw[2][2][KT];   // [buffer][point of the pair][row]

  // the group (uniform over the workgroup), selected with constant indices only so that
  // its arguments stay in scalar registers
  int gi = 0;
#pragma unroll
  for (int k = 1; k < CHI0_MAX_GROUPS; ++k)
    if (k < L.ngroups && (int32_t)blockIdx.x >= L.begin[k]) gi = k;
  Chi0Args a = L.g[0];
  int32_t gbase = L.begin[0];
#pragma unroll
  for (int k = 1; k < CHI0_MAX_GROUPS; ++k)
    if (k == gi) {
      a = L.g[k];
      gbase = L.begin[k];
    }

  // One-dimensional grid per group.  Work items run cluster by cluster, a cluster being
  // one (tile, row split) and its members the launch's pairs, which all stage the same
  // panel rows; the off-diagonal clusters of every split come first and the shorter
  // diagonal ones last, so the last round of workgroups is made of short ones.  The
  // hardware hands workgroup g to XCD g mod 8 (up to the group's base offset, the same for
  // every workgroup of the group), so the items are dealt out in chunks of 8 consecutive
  // ones: workgroups g = 64 j + x + 8 o (o = 0..7) take items 8 (8 j + x) + o, and the 8
  // workgroups of a chunk run side by side on one XCD, where its L2 serves the panels
  // they share; each XCD still gets every 8th chunk, hence the same mix of long and short
  // tiles.  The last nw mod 64 items keep their own order.
  const int T = (a.N + TN - 1) / TN;
  const int noff = T * (T - 1) / 2;
  const int64_t np = a.npairs;
  const int64_t ncl_off = (int64_t)noff * a.ksplit;   // off-diagonal clusters
  const int64_t nw = (ncl_off + (int64_t)T * a.ksplit) * np;
  const int64_t g = (int64_t)blockIdx.x - gbase;
  const int64_t w = g < nw / 64 * 64 ? ((g >> 6) * 8 + (g & 7)) * 8 + ((g >> 3) & 7) : g;
  const int64_t c = w / np;
  const int pair = (int)(w % np);
  int tr, tc, split;
  if (c < ncl_off) {
    const int k = (int)(c % noff);   // strictly lower tile k: row r > column c
    int r = (int)((1.0 + sqrt(1.0 + 8.0 * (double)k)) * 0.5);
    while (r * (r - 1) / 2 > k) --r;
    while ((r + 1) * r / 2 <= k) ++r;
    tr = r;
    tc = k - r * (r - 1) / 2;
    split = (int)(c / noff);
  } else {
    const int64_t h = c - ncl_off;
    tr = tc = (int)(h % T);
    split = (int)(h / T);
  }
  const int p0 = a.pairs[2 * pair];
  const int p1s = a.pairs[2 * pair + 1];
  const bool two = p1s >= 0;
  const int p1 = two ? p1s : p0;
  const PointDesc pd = a.pts[p0];
  const int N = a.N;
  const int ms = (int)((((a.M + a.ksplit - 1) / a.ksplit) + KT - 1) / KT) * KT;
  const int mlo = split * ms;
  const int M = mlo + ms < (int)a.M ? mlo + ms : (int)a.M;
  const int P0 = tr * TN, Q0 = tc * TN;
  const bool diag = (tr == tc);
  // an off-diagonal tile of the last tile row with at most 32 valid rows (N not a multiple
  // of 64): its waves split by point instead of by row half, wave (wr, wc) contracting
  // rows P0 .. P0 + 31 of its column half for point wr, so the tile takes half the MFMA
  // time of a full one.  Every output element sees the same products in the same order.
  const bool half = !diag && P0 + TN / 2 >= N;

  const int tid = threadIdx.x;
  const int lrow = tid >> 4;   // 0..15: one row of the K step per 16 lanes
  const int lc = tid & 15;

  const char *bbase = reinterpret_cast<const char *>(a.B) +
                      (int64_t)pd.bslot * a.b_slot_stride * (CPLX_B ? 16 : 8);
  const double *wrow0 = a.wtab + (int64_t)p0 * a.M;
  const double *wrow1 = a.wtab + (int64_t)p1 * a.M;

  int pcol[4], qcol[4];
  bool pok[4], qok[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int P = P0 + lc + 16 * c, Q = Q0 + lc + 16 * c;
    pok[c] = P < N;
    qok[c] = Q < N;
    pcol[c] = pok[c] ? P : 0;
    qcol[c] = qok[c] ? Q : 0;
  }

  const int wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;

  d4 accR[2][2][2], accI[2][2][2];   // [point][x][y]
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        accR[p][x][y] = d4{0.0, 0.0, 0.0, 0.0};
        accI[p][x][y] = d4{0.0, 0.0, 0.0, 0.0};
      }

  double2 sa[4], sb[4];
  double sw0, sw1;
  bool mv;
  auto load = [&](int m0) __attribute__((always_inline)) {
    const int m = m0 + lrow;
    mv = m < M;
    const int mc = mv ? m : 0;
    sw0 = wrow0[mc];
    sw1 = wrow1[mc];
    const int64_t rowoff = (int64_t)mc * N;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sa[c] = load_b<CPLX_B>(bbase, rowoff + pcol[c]);
      sb[c] = load_b<CPLX_B>(bbase, rowoff + qcol[c]);
    }
  };
  auto store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double2 av = sa[c], bv = sb[c];
      const bool aok = mv && pok[c];
      lds[buf][0][lrow][lc + 16 * c] = make_double2(aok ? av.x : 0.0, aok ? av.y : 0.0);
      lds[buf][1][lrow][lc + 16 * c] = make_double2(qok[c] ? bv.x : 0.0, qok[c] ? bv.y : 0.0);
    }
    if (lc == 0) {
      lw[buf][0][lrow] = mv ? sw0 : 0.0;
      lw[buf][1][lrow] = mv ? sw1 : 0.0;
    }
  };
  // one K step of an off-diagonal tile for both points; with LOADS, the next step's
  // global loads are spread over the four sub-steps (column group ks before sub-step ks)
  // instead of issued together, so that no wave waits long for the address unit while
  // its MFMA pipe idles
  auto contract = [&](int buf, auto loads_tag, int m0next) __attribute__((always_inline)) {
    constexpr bool LOADS = decltype(loads_tag)::value;
    int64_t rowoff = 0;
    if (LOADS) {
      const int m = m0next + lrow;
      mv = m < M;
      const int mc = mv ? m : 0;
      sw0 = wrow0[mc];
      sw1 = wrow1[mc];
      rowoff = (int64_t)mc * N;
    }
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks) {
      if (LOADS) {
        sa[ks] = load_b<CPLX_B>(bbase, rowoff + pcol[ks]);
        sb[ks] = load_b<CPLX_B>(bbase, rowoff + qcol[ks]);
      }
      const int r = ks * 4 + lk;
      double2 av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = lds[buf][0][r][wr * 32 + x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = lds[buf][1][r][wc * 32 + y * 16 + li];
      const double wp[2] = {lw[buf][0][r], lw[buf][1][r]};
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        double2 bw[2];
#pragma unroll
        for (int y = 0; y < 2; ++y) bw[y] = make_double2(wp[p] * bv[y].x, wp[p] * bv[y].y);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            accR[p][x][y] = mfma(av[x].x, bw[y].x, accR[p][x][y]);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            accI[p][x][y] = mfma(av[x].x, bw[y].y, accI[p][x][y]);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            accR[p][x][y] = mfma(av[x].y, bw[y].y, accR[p][x][y]);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            accI[p][x][y] = mfma(-av[x].y, bw[y].x, accI[p][x][y]);
      }
    }
  };

  // one K step of a half tile: point wr only, rows 0 .. 31 of the tile
  auto contract_half = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks) {
      const int r = ks * 4 + lk;
      double2 av[2], bv[2], bw[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = lds[buf][0][r][x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = lds[buf][1][r][wc * 32 + y * 16 + li];
      const double w = lw[buf][wr][r];
#pragma unroll
      for (int y = 0; y < 2; ++y) bw[y] = make_double2(w * bv[y].x, w * bv[y].y);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          accR[0][x][y] = mfma(av[x].x, bw[y].x, accR[0][x][y]);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          accI[0][x][y] = mfma(av[x].x, bw[y].y, accI[0][x][y]);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          accR[0][x][y] = mfma(av[x].y, bw[y].y, accR[0][x][y]);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          accI[0][x][y] = mfma(-av[x].y, bw[y].x, accI[0][x][y]);
    }
  };

  const int nsteps = M > mlo ? (M - mlo + KT - 1) / KT : 1;
  double2 *base = split == 0 ? a.out : a.partial + (int64_t)(split - 1) * a.split_stride;
  load(mlo);
  store(0);
  __syncthreads();
  if (half) {
    // a single point's second pair of waves only keeps the loads and barriers going
    const bool act = wr == 0 || two;
    for (int s = 0; s + 1 < nsteps; ++s) {
      const int cur = s & 1;
      load(mlo + (s + 1) * KT);
      __builtin_amdgcn_sched_barrier(0);
      if (act) contract_half(cur);
      __builtin_amdgcn_sched_barrier(0);
      store(cur ^ 1);
      __syncthreads();
    }
    if (act) {
      contract_half((nsteps - 1) & 1);
      double2 *out = base + (int64_t)(wr == 0 ? p0 : p1) * a.out_stride;
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int P = P0 + x * 16 + lk + 4 * r;
            const int Q = Q0 + wc * 32 + y * 16 + li;
            if (P >= N || Q >= N) continue;
            const double re = accR[0][x][y][r];
            const double im = accI[0][x][y][r];
            out[(int64_t)P * N + Q] = make_double2(re, im);
            out[(int64_t)Q * N + P] = make_double2(re, -im);
          }
    }
  } else if (!diag) {
    for (int s = 0; s + 1 < nsteps; ++s) {
      const int cur = s & 1;
      contract(cur, std::integral_constant<bool, true>{}, mlo + (s + 1) * KT);
      __builtin_amdgcn_sched_barrier(0);
      store(cur ^ 1);
      __syncthreads();
    }
    contract((nsteps - 1) & 1, std::integral_constant<bool, false>{}, 0);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (p == 1 && !two) break;
      double2 *out = base + (int64_t)(p == 0 ? p0 : p1) * a.out_stride;
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int P = P0 + wr * 32 + x * 16 + lk + 4 * r;
            const int Q = Q0 + wc * 32 + y * 16 + li;
            if (P >= N || Q >= N) continue;
            const double re = accR[p][x][y][r];
            const double im = accI[p][x][y][r];
            out[(int64_t)P * N + Q] = make_double2(re, im);
            out[(int64_t)Q * N + P] = make_double2(re, -im);
          }
    }
  } else {
    // wave (point pp, role): five of the point's ten lower blocks; a single point's
    // second pair of waves only keeps the loads and barriers going
    const int pp = wave >> 1, role = wave & 1;
    const bool act = pp == 0 || two;
    d4 dR[5], dI[5];
#pragma unroll
    for (int u = 0; u < 5; ++u) dR[u] = dI[u] = d4{0.0, 0.0, 0.0, 0.0};
    auto cdiag = [&](int buf) __attribute__((always_inline)) {
      if (!act) return;
      if (role == 0)
        contract_diag5<0>(lds[buf][0], lds[buf][1], lw[buf][pp], li, lk, dR, dI);
      else
        contract_diag5<1>(lds[buf][0], lds[buf][1], lw[buf][pp], li, lk, dR, dI);
    };
    for (int s = 0; s + 1 < nsteps; ++s) {
      const int cur = s & 1;
      load(mlo + (s + 1) * KT);
      __builtin_amdgcn_sched_barrier(0);
      cdiag(cur);
      __builtin_amdgcn_sched_barrier(0);
      store(cur ^ 1);
      __syncthreads();
    }
    cdiag((nsteps - 1) & 1);
    if (act) {
      double2 *out = base + (int64_t)(pp == 0 ? p0 : p1) * a.out_stride;
#pragma unroll
      for (int u = 0; u < 5; ++u) {
        const int bx = role == 0 ? DIAG_BX[0][u] : DIAG_BX[1][u];
        const int by = role == 0 ? DIAG_BY[0][u] : DIAG_BY[1][u];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int P = P0 + bx * 16 + lk + 4 * r;
          const int Q = Q0 + by * 16 + li;
          if (P >= N || Q >= N || P < Q) continue;
          const double re = dR[u][r];
          const double im = dI[u][r];
          if (P == Q) {
            out[(int64_t)P * N + Q] = make_double2(re, 0.0);
            continue;
          }
          out[(int64_t)P * N + Q] = make_double2(re, im);
          out[(int64_t)Q * N + P] = make_double2(re, -im);
        }
      }
    }
  }
}

// The same contraction on 128 x 128 tiles: eight waves, each a 64 x 32 sub-tile (4 x 2
// MFMA blocks), 16-row K steps (64 KB of LDS per stage, double-buffered, one workgroup
// per CU).  Twice the MFMA work per loaded byte of the 64-wide tile.  A thread stages one
// row and four columns (32 apart) of both panels, so every load instruction of a wave
// reads two 512-byte row segments.  Workgroups are numbered so that each of the 8 XCDs
// (which take workgroups round-robin) gets a contiguous range of the (tile, point,
// split) order and its L2 serves the panels those tiles share.
constexpr int TW = 128;
constexpr int LDPW = TW + 1;
constexpr int KTW = 16;

template <bool CPLX_B>
__global__ __launch_bounds__(512) void chi0_f64_t128_kernel(Chi0Args a, int32_t ntiles, int32_t npts) {
  __shared__ double2 lds[2][2][KTW][LDPW];
  const int G = gridDim.x, hw = blockIdx.x;
  const int per = (G + 7) / 8, tall = G % 8 == 0 ? 8 : G % 8;
  const int xcd = hw % 8, loc = hw / 8;
  const int lg = xcd < tall ? xcd * per + loc : tall * per + (xcd - tall) * (per - 1) + loc;
  const int tile = lg % ntiles, p = (lg / ntiles) % npts, split = lg / (ntiles * npts);

  const PointDesc pd = a.pts[p];
  int tr, tc;
  tile_of(tile, tr, tc);
  const int N = a.N;
  const int ms = (int)((((a.M + a.ksplit - 1) / a.ksplit) + KTW - 1) / KTW) * KTW;
  const int mlo = split * ms;
  const int M = mlo + ms < (int)a.M ? mlo + ms : (int)a.M;
  const int P0 = tr * TW, Q0 = tc * TW;
  const bool diag = (tr == tc);

  const int tid = threadIdx.x;
  const int lrow = tid >> 5, lc = tid & 31;
  const char *bbase = reinterpret_cast<const char *>(a.B) + (int64_t)pd.bslot * a.b_slot_stride * (CPLX_B ? 16 : 8);
  const double *wrow = a.wtab + (int64_t)p * a.M;
  int pcol[4], qcol[4];
  bool pok[4], qok[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int P = P0 + lc + 32 * c, Q = Q0 + lc + 32 * c;
    pok[c] = P < N;
    qok[c] = Q < N;
    pcol[c] = pok[c] ? P : 0;
    qcol[c] = qok[c] ? Q : 0;
  }
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 2, wc = wave & 3;
  const int li = lane & 15, lk = lane >> 4;

  d4 accR[4][2], accI[4][2];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      accR[x][y] = d4{0.0, 0.0, 0.0, 0.0};
      accI[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    }

  double2 sa[4], sb[4];
  double sw;
  bool mv;
  auto load = [&](int m0) {
    const int m = m0 + lrow;
    mv = m < M;
    const int mc = mv ? m : 0;
    sw = wrow[mc];
    const int64_t rowoff = (int64_t)mc * N;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sa[c] = load_b<CPLX_B>(bbase, rowoff + pcol[c]);
      sb[c] = load_b<CPLX_B>(bbase, rowoff + qcol[c]);
    }
  };
  auto store = [&](int buf) {
    const double w = mv ? sw : 0.0;
    const double2 z = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double2 av = (mv && pok[c]) ? sa[c] : z;
      const double2 bv = qok[c] ? sb[c] : z;
      lds[buf][0][lrow][lc + 32 * c] = av;
      lds[buf][1][lrow][lc + 32 * c] = make_double2(w * bv.x, w * bv.y);
    }
  };
  auto contract = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < KTW / 4; ++ks) {
      double2 av[4], bv[2];
#pragma unroll
      for (int x = 0; x < 4; ++x) av[x] = lds[buf][0][ks * 4 + lk][wr * 64 + x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = lds[buf][1][ks * 4 + lk][wc * 32 + y * 16 + li];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accR[x][y] = mfma(av[x].x, bv[y].x, accR[x][y]);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[x][y] = mfma(av[x].x, bv[y].y, accI[x][y]);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accR[x][y] = mfma(av[x].y, bv[y].y, accR[x][y]);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[x][y] = mfma(-av[x].y, bv[y].x, accI[x][y]);
    }
  };

  const int nsteps = M > mlo ? (M - mlo + KTW - 1) / KTW : 1;
  load(mlo);
  store(0);
  __syncthreads();
  for (int s = 0; s + 1 < nsteps; ++s) {
    const int cur = s & 1;
    load(mlo + (s + 1) * KTW);
    __builtin_amdgcn_sched_barrier(0);
    contract(cur);
    __builtin_amdgcn_sched_barrier(0);
    store(cur ^ 1);
    __syncthreads();
  }
  contract((nsteps - 1) & 1);

  double2 *out = (split == 0 ? a.out : a.partial + (int64_t)(split - 1) * a.split_stride) + (int64_t)p * a.out_stride;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int P = P0 + wr * 64 + x * 16 + lk + 4 * r;
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

// out += partial_1 + ... (the row splits after the first, planes n apart), added one
// plane after another in split order, so repeatable
__global__ __launch_bounds__(256) void split_reduce_kernel(const double2 *partial, int32_t nparts, int64_t n,
                                                           double2 *out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double2 a = out[i];
    for (int z = 0; z < nparts; ++z) {
      const double2 b = partial[(int64_t)z * n + i];
      a = make_double2(a.x + b.x, a.y + b.y);
    }
    out[i] = a;
  }
}

}  // namespace

int32_t chi0_pick_ksplit(int64_t work, int64_t slots, int64_t M, int32_t max_split) {
  // fraction of the last round of workgroups that is busy, for 1..max_split splits; a
  // split must keep at least 512 rows.  Each further split costs its partial planes'
  // traffic and their reduction: about 2% of the contraction at M = 16128 rows (the
  // 3x3x1 slab at N_aux 384), a share that falls as 1/M since the contraction grows with
  // M and the planes do not
  const double pen = std::min(0.02, 0.02 * 16128.0 / (double)std::max<int64_t>(M, 1));
  int best = 1;
  double best_eff = 0.0;
  for (int s = 1; s <= max_split; ++s) {
    if (s > 1 && M / s < 512) break;
    const double rounds = (double)(work * s) / (double)slots;
    const double eff = rounds / std::ceil(rounds) * (1.0 - pen * (s - 1));
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = s;
    }
  }
  return best;
}

hipError_t launch_chi0_weights(hipStream_t s, const Chi0Args &a, int32_t npts) {
  const int64_t total = (int64_t)npts * a.M;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(weight_table_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, npts);
  return hipGetLastError();
}

int chi0_cfg_count() { return 5; }
int chi0_cfg_tile(int cfg) { return cfg == 3 ? TW : TN; }
int chi0_cfg_slots_per_cu(int cfg) { return cfg == 3 ? 1 : 2; }
int chi0_cfg_points_per_wg(int cfg) { return cfg == 4 ? 2 : 1; }
const char *chi0_cfg_name(int cfg) {
  static const char *names[5] = {"t64k8", "t64k16", "t64k32", "t128k16", "t64k16w2"};
  return (cfg >= 0 && cfg < 5) ? names[cfg] : "?";
}

hipError_t launch_chi0_f64(hipStream_t s, const Chi0Args &args, int32_t npts, bool cplx_b, int cfg) {
  if (npts <= 0) return hipSuccess;
  if (args.ksplit > kMaxSplit) return hipErrorInvalidValue;
  // split 0 writes a.out, split z >= 1 the z-th plane of a.partial (planes npts points apart)
  const int ks = args.ksplit > 1 ? args.ksplit : 1;
  Chi0Args a = args;
  a.ksplit = ks;
  a.split_stride = (int64_t)npts * a.out_stride;
  // the paired kernel needs the launch's pair table; without one the single-point kernel
  // of the same tile and K step computes the same sums
  if (cfg == 4 && (a.pairs == nullptr || a.npairs <= 0)) cfg = 1;
  if (cfg == 4) {
    Chi0Group one{a, npts};
    return launch_chi0_f64_paired_groups(s, &one, 1, cplx_b);
  }
  if (cfg == 3) {
    const int T = (a.N + TW - 1) / TW;
    const int64_t nwg = (int64_t)T * (T + 1) / 2 * npts * ks;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    if (cplx_b)
      hipLaunchKernelGGL((chi0_f64_t128_kernel<true>), dim3((unsigned)nwg), dim3(512), 0, s, a, T * (T + 1) / 2, npts);
    else
      hipLaunchKernelGGL((chi0_f64_t128_kernel<false>), dim3((unsigned)nwg), dim3(512), 0, s, a, T * (T + 1) / 2, npts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ks == 1) return e;
    return launch_split_add(s, a.partial, ks - 1, (int64_t)npts * a.out_stride, a.out);
  }
  const int kt = cfg == 0 ? 8 : cfg == 2 ? 32 : 16;
  const int T = (a.N + TN - 1) / TN;
  const dim3 grid((unsigned)(T * (T + 1) / 2), (unsigned)npts, (unsigned)ks);
#define RPA_CHI0_LAUNCH(C, K) hipLaunchKernelGGL((chi0_f64_kernel<C, K>), grid, dim3(256), 0, s, a)
  if (kt == 8) {
    if (cplx_b) RPA_CHI0_LAUNCH(true, 8); else RPA_CHI0_LAUNCH(false, 8);
  } else if (kt == 32) {
    if (cplx_b) RPA_CHI0_LAUNCH(true, 32); else RPA_CHI0_LAUNCH(false, 32);
  } else {
    if (cplx_b) RPA_CHI0_LAUNCH(true, 16); else RPA_CHI0_LAUNCH(false, 16);
  }
#undef RPA_CHI0_LAUNCH
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1) return e;
  return launch_split_add(s, a.partial, ks - 1, (int64_t)npts * a.out_stride, a.out);
}

int64_t chi0_paired_workgroups(const Chi0Args &a) {
  const int T = (a.N + TN - 1) / TN;
  return (int64_t)T * (T + 1) / 2 * a.npairs * (a.ksplit > 1 ? a.ksplit : 1);
}

hipError_t launch_chi0_f64_paired_groups(hipStream_t s, const Chi0Group *groups, int ngroups, bool cplx_b) {
  if (ngroups <= 0) return hipSuccess;
  if (ngroups > CHI0_MAX_GROUPS) return hipErrorInvalidValue;
  Chi0Launch L{};
  int64_t total = 0;
  int n = 0;
  for (int i = 0; i < ngroups; ++i) {
    const Chi0Group &gr = groups[i];
    if (gr.npts <= 0) continue;
    if (gr.a.ksplit > kMaxSplit || gr.a.pairs == nullptr || gr.a.npairs <= 0) return hipErrorInvalidValue;
    Chi0Args a = gr.a;
    a.ksplit = a.ksplit > 1 ? a.ksplit : 1;
    a.split_stride = (int64_t)gr.npts * a.out_stride;
    L.g[n] = a;
    L.begin[n] = (int32_t)total;
    total += chi0_paired_workgroups(a);
    if (total > 0x7fffffff) return hipErrorInvalidValue;
    ++n;
  }
  if (n == 0) return hipSuccess;
  L.ngroups = n;
  for (int i = n; i <= CHI0_MAX_GROUPS; ++i) L.begin[i] = (int32_t)total;
  const dim3 grid((unsigned)total);
  if (cplx_b)
    hipLaunchKernelGGL((chi0_f64_w2_kernel<true>), grid, dim3(256), 0, s, L);
  else
    hipLaunchKernelGGL((chi0_f64_w2_kernel<false>), grid, dim3(256), 0, s, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // each group's later row splits added into its output, in split order
  for (int i = 0; i < n; ++i) {
    const Chi0Args &a = L.g[i];
    if (a.ksplit <= 1) continue;
    e = launch_split_add(s, a.partial, a.ksplit - 1, a.split_stride, a.out);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_split_add(hipStream_t s, const double2 *partial, int32_t nparts, int64_t n, double2 *out) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1 || nparts < 1) return hipSuccess;
  hipLaunchKernelGGL(split_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, partial, nparts, n, out);
  return hipGetLastError();
}

}  // namespace rpa
