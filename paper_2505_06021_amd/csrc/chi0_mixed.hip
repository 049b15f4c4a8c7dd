// chi0(q, i w) with the FP32 matrix cores (v_mfma_f32_16x16x4f32), keeping in FP64
// what the FP64 path keeps in FP64:
//  - partial sums are flushed from FP32 into FP64 accumulators every FLUSH_ROWS rows, so
//    FP32 rounding never runs over long chains;
//  - the diagonal chi0_PP = sum_m w_m |B_mP|^2, a sum of same-signed terms whose rounding
//    errors do not cancel, is taken from an exact FP64 pass (diag_partial/diag_reduce)
//    instead of the MFMA result.
// The contraction reads B in FP32 (the device converts the FP64 coefficients once per
// q), the right operand is scaled by w_m zeta_k in FP32 (at the LDS store, or per lane
// after the LDS read in the kernel that contracts two frequencies per workgroup), and the
// output is FP64 complex like the FP64 path's.  (The split-BF16 contraction is
// chi0_bf16.hip.)
#include <type_traits>

#include "common.hpp"

namespace rpa {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TN = 64;
constexpr int FLUSH_ROWS = 256;

__device__ __forceinline__ void tile_of(int t, int &tr, int &tc) {
  int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  tr = r;
  tc = t - r * (r + 1) / 2;
}

// ------------------------------------------------------------------ conversion

__global__ __launch_bounds__(256) void to_f32_kernel(const void *in, float2 *out, int64_t n, int cplx) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (cplx) {
      const double2 v = reinterpret_cast<const double2 *>(in)[i];
      out[i] = make_float2((float)v.x, (float)v.y);
    } else {
      out[i] = make_float2((float)reinterpret_cast<const double *>(in)[i], 0.f);
    }
  }
}

// ------------------------------------------------------------------ exact diagonal
// partial[c][p][P] = sum over the rows m of chunk c of w_p(m) |B_mP|^2 in FP64, for all
// the points p of a launch that share one B slab; a second pass sums the chunks in
// order.  A workgroup covers 64 columns x spw * DIAG_ROWS rows (spw sub-chunks, chosen
// from the shape so that the launch has about 2048 workgroups): four row groups of 64
// lanes (lanes on consecutive columns, so every load instruction reads 1 KB contiguous)
// whose partial sums are combined in LDS in a fixed order.  A thread issues all the row
// loads of a sub-chunk before it accumulates them: the kernel is bound by HBM reads.
constexpr int DIAG_ROWS = 64;      // rows per sub-chunk
constexpr int DIAG_MAXP = 16;      // points per pass

__global__ __launch_bounds__(256) void diag_partial_kernel(const void *B, int cplx, int64_t M, int N,
                                                           const double *wtab, int npts, int spw,
                                                           double *partial) {
  __shared__ double wl[DIAG_MAXP][DIAG_ROWS];   // the sub-chunk's weights, read once
  __shared__ double red[4][DIAG_MAXP][64];
  constexpr int RPG = DIAG_ROWS / 4;            // rows per row group
  const int col = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int P = blockIdx.x * 64 + col;
  const int c = blockIdx.y;
  const int Pc = P < N ? P : 0;
  double acc[DIAG_MAXP];
#pragma unroll
  for (int p = 0; p < DIAG_MAXP; ++p) acc[p] = 0.0;
  for (int sc = 0; sc < spw; ++sc) {
    const int64_t m0 = ((int64_t)c * spw + sc) * DIAG_ROWS;
    if (m0 >= M) break;   // uniform over the workgroup
    const int rows = (int)(M - m0 < DIAG_ROWS ? M - m0 : DIAG_ROWS);
    double b2[RPG];
#pragma unroll
    for (int j = 0; j < RPG; ++j) {
      const int r = grp + 4 * j;
      const int64_t m = m0 + (r < rows ? r : 0);
      if (cplx) {
        const double2 v = reinterpret_cast<const double2 *>(B)[m * N + Pc];
        b2[j] = v.x * v.x + v.y * v.y;
      } else {
        const double v = reinterpret_cast<const double *>(B)[m * N + Pc];
        b2[j] = v * v;
      }
    }
    __syncthreads();   // the previous sub-chunk's weights are no longer read
    for (int e = threadIdx.x; e < DIAG_MAXP * DIAG_ROWS; e += 256) {
      const int p = e / DIAG_ROWS, r = e % DIAG_ROWS;
      wl[p][r] = (p < npts && r < rows) ? wtab[(int64_t)p * M + m0 + r] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RPG; ++j) {
      const int r = grp + 4 * j;
      if (r < rows) {
#pragma unroll
        for (int p = 0; p < DIAG_MAXP; ++p) acc[p] += wl[p][r] * b2[j];
      }
    }
  }
#pragma unroll
  for (int p = 0; p < DIAG_MAXP; ++p) red[grp][p][col] = acc[p];
  __syncthreads();
  if (grp == 0 && P < N) {
    for (int p = 0; p < npts; ++p)
      partial[((int64_t)c * npts + p) * N + P] = ((red[0][p][col] + red[1][p][col]) + red[2][p][col]) +
                                                 red[3][p][col];
  }
}

// sub-chunks per workgroup of the exact-diagonal pass, and the chunk count it gives
inline int diag_spw(int64_t M, int N) {
  const int64_t nsub = (M + DIAG_ROWS - 1) / DIAG_ROWS, ncb = (N + 63) / 64;
  int64_t want = 2048 / ncb;   // chunks for about 2048 workgroups
  if (want < 1) want = 1;
  int64_t spw = (nsub + want - 1) / want;
  if (spw < 1) spw = 1;
  while ((nsub + spw - 1) / spw > 65535) ++spw;
  return (int)spw;
}

inline int64_t diag_nchunks(int64_t M, int N) {
  const int64_t nsub = (M + DIAG_ROWS - 1) / DIAG_ROWS;
  const int spw = diag_spw(M, N);
  return (nsub + spw - 1) / spw;
}

__global__ __launch_bounds__(256) void diag_reduce_kernel(const double *partial, int nchunks, int npts,
                                                          int N, double *diag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)npts * N) return;
  // the chunks are added in order; their loads go out 16 at a time (few workgroups: the
  // loads' latency, not bandwidth, sets the time)
  const int64_t st = (int64_t)npts * N;
  double s = 0.0;
  int c = 0;
  for (; c + 16 <= nchunks; c += 16) {
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = partial[(int64_t)(c + u) * st + i];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += t[u];
  }
  for (; c < nchunks; ++c) s += partial[(int64_t)c * st + i];
  diag[i] = s;
}

// ------------------------------------------------------------------ FP32 MFMA

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int LDP32 = TN + 1;

// Diagonal tiles of the paired kernel: the ten 16 x 16 blocks on or below the diagonal
// of a 64 x 64 tile, split five and five between two waves per point ("roles"); block u
// of role R is (DIAG_BX[R][u], DIAG_BY[R][u]) in 16-row/column units.  Each block takes
// the single-point kernel's four products per 4-row sub-step in the same order.
__device__ constexpr int DIAG_BX[2][5] = {{0, 1, 1, 2, 3}, {2, 2, 3, 3, 3}};
__device__ constexpr int DIAG_BY[2][5] = {{0, 0, 1, 0, 0}, {1, 2, 1, 2, 3}};

template <int KT, int ROLE>
__device__ __forceinline__ void contract_diag5_f32(const float2 (*la)[LDP32], const float2 (*lb)[LDP32],
                                                   const float *lwp, int li, int lk, f4 (&dR)[5], f4 (&dI)[5]) {
  constexpr bool needA[4] = {ROLE == 0, ROLE == 0, true, true};
  constexpr bool needB[4] = {ROLE == 0, true, ROLE == 1, ROLE == 1};
#pragma unroll
  for (int ks = 0; ks < KT / 4; ++ks) {
    const int r = ks * 4 + lk;
    float2 av[4], bw[4];
    const float w = lwp[r];
#pragma unroll
    for (int x = 0; x < 4; ++x)
      if (needA[x]) av[x] = la[r][x * 16 + li];
#pragma unroll
    for (int y = 0; y < 4; ++y)
      if (needB[y]) {
        const float2 b = lb[r][y * 16 + li];
        bw[y] = make_float2(w * b.x, w * b.y);
      }
#pragma unroll
    for (int u = 0; u < 5; ++u) dR[u] = mfma32(av[DIAG_BX[ROLE][u]].x, bw[DIAG_BY[ROLE][u]].x, dR[u]);
#pragma unroll
    for (int u = 0; u < 5; ++u) dI[u] = mfma32(av[DIAG_BX[ROLE][u]].x, bw[DIAG_BY[ROLE][u]].y, dI[u]);
#pragma unroll
    for (int u = 0; u < 5; ++u) dR[u] = mfma32(av[DIAG_BX[ROLE][u]].y, bw[DIAG_BY[ROLE][u]].y, dR[u]);
#pragma unroll
    for (int u = 0; u < 5; ++u) dI[u] = mfma32(-av[DIAG_BX[ROLE][u]].y, bw[DIAG_BY[ROLE][u]].x, dI[u]);
  }
}

// NP = 2: a workgroup contracts two frequencies of one q (pair j of the launch's pair
// table: a.pairs[2 j] and a.pairs[2 j + 1], the second -1 when single): the unweighted FP32 panels are staged once and each lane
// scales its right-operand fragments by the two points' weights of its row (the same
// float product w * b the single-point kernel forms at its LDS store, so the sums are bit
// for bit the same); half the loads, LDS stores and barriers per MFMA.  In diagonal tiles
// waves 0 and 1 take point 0's ten lower blocks, five each, and waves 2 and 3 point 1's.
// A launch holds up to CHI0_MAX_GROUPS groups (NP = 2 only: the point batches of several
// serving jobs launched together); group i owns the workgroups [begin[i], begin[i + 1])
// of the one-dimensional grid and is contracted exactly as it would be alone.
struct Chi0F32Launch {
  int32_t ngroups;
  int32_t begin[CHI0_MAX_GROUPS + 1];
  Chi0Args g[CHI0_MAX_GROUPS];
  const float2 *B32[CHI0_MAX_GROUPS];
  const double *diag[CHI0_MAX_GROUPS];
};

template <int KT, int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void chi0_f32_kernel(Chi0F32Launch L) {
  // the group (uniform over the workgroup), selected with constant indices only so that
  // its arguments stay in scalar registers
  int gi = 0;
  if constexpr (NP == 2) {
#pragma unroll
    for (int k = 1; k < CHI0_MAX_GROUPS; ++k)
      if (k < L.ngroups && (int32_t)blockIdx.x >= L.begin[k]) gi = k;
  }
  Chi0Args a = L.g[0];
  const float2 *B32 = L.B32[0];
  const double *diag = L.diag[0];
  int32_t gbase = L.begin[0];
  if constexpr (NP == 2) {
#pragma unroll
    for (int k = 1; k < CHI0_MAX_GROUPS; ++k)
      if (k == gi) {
        a = L.g[k];
        B32 = L.B32[k];
        diag = L.diag[k];
        gbase = L.begin[k];
      }
  }
  __shared__ float2 lds[2][2][KT][LDP32];
  __shared__ float lw[2][NP][KT];   // per-row weights of the pair (NP = 2 only)
  constexpr int RPI = 16;
  constexpr int NPASS = KT / RPI;

  // NP = 1: grid (tile, point, split).  NP = 2: the one-dimensional grid of the paired
  // FP64 kernel (clusters of the pairs of one (tile, split), off-diagonal ones first, dealt
  // out to the XCDs in chunks of 8 items).
  int tr, tc, unit, split, nsplit;
  if constexpr (NP == 1) {
    tile_of((int)blockIdx.x, tr, tc);
    unit = (int)blockIdx.y;
    split = (int)blockIdx.z;
    nsplit = (int)gridDim.z;
  } else {
    const int T = (a.N + TN - 1) / TN;
    const int noff = T * (T - 1) / 2;
    const int64_t np = a.npairs;
    const int64_t ncl_off = (int64_t)noff * a.ksplit;   // off-diagonal (tile, split) clusters
    const int64_t nw = (ncl_off + (int64_t)T * a.ksplit) * np;
    const int64_t g = (int64_t)blockIdx.x - gbase;
    const int64_t w = g < nw / 64 * 64 ? ((g >> 6) * 8 + (g & 7)) * 8 + ((g >> 3) & 7) : g;
    const int64_t c = w / np;
    unit = (int)(w % np);
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
    nsplit = a.ksplit;
  }
  int pidx[NP];
  bool pon[NP];
  if constexpr (NP == 1) {
    pidx[0] = unit;
    pon[0] = true;
  } else {
    pidx[0] = a.pairs[2 * unit];
    const int p1 = a.pairs[2 * unit + 1];
    pon[0] = true;
    pon[1] = p1 >= 0;
    pidx[1] = p1 >= 0 ? p1 : pidx[0];
  }
  const PointDesc pd = a.pts[pidx[0]];
  const int N = a.N;
  // rows [mlo, mhi) of the contraction belong to split `split`
  const int ms = (int)((((a.M + nsplit - 1) / nsplit) + KT - 1) / KT) * KT;
  const int mlo = split * ms;
  const int M = mlo + ms < (int)a.M ? mlo + ms : (int)a.M;
  const int P0 = tr * TN, Q0 = tc * TN;
  const bool is_diag = (tr == tc);
  const int tid = threadIdx.x;
  const int lrow = tid >> 4, lc = tid & 15;
  const float2 *bb = B32 + (int64_t)pd.bslot * a.b_slot_stride;
  const double *wrow[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) wrow[p] = a.wtab + (int64_t)pidx[p] * a.M;

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
  // diagonal quadrants skip their strictly upper 16 x 16 block (each block summed
  // exactly as before); bit 2x + y of `on` marks the blocks a wave computes.
  int on = 0xf;
  // paired kernel, an off-diagonal tile of the last tile row with at most 32 valid rows:
  // the waves split by point instead of by row half (wave (wr, wc) contracts rows
  // P0 .. P0 + 31 of its column half for point hp = wr into accumulator set 0), so the tile
  // takes half the MFMA time; every output element sees the same products, flushes and
  // order as in a full tile
  const bool half = NP == 2 && !is_diag && P0 + TN / 2 >= N;
  const int hp = wr;
  if (half) wr = 0;
  if (is_diag) {
    if (wr == 0 && wc == 1) {
      wr = 1;
      wc = 0;
      on = 0xa;
    } else if (wr == 1 && wc == 0) {
      on = 0x5;
    } else {
      on = 0xd;
    }
  }

  f4 accR[NP][2][2], accI[NP][2][2];
  double hR[NP][2][2][4], hI[NP][2][2][4];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        accR[p][x][y] = f4{0.f, 0.f, 0.f, 0.f};
        accI[p][x][y] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < 4; ++r) hR[p][x][y][r] = hI[p][x][y][r] = 0.0;
      }

  float2 sa[NPASS][4], sb[NPASS][4];
  double sw[NPASS][NP];
  bool smv[NPASS];
  auto load = [&](int m0) __attribute__((always_inline)) {
#pragma unroll
    for (int ps = 0; ps < NPASS; ++ps) {
      const int m = m0 + ps * RPI + lrow;
      smv[ps] = m < M;
      const int mc = smv[ps] ? m : 0;
#pragma unroll
      for (int p = 0; p < NP; ++p) sw[ps][p] = wrow[p][mc];
      const int64_t ro = (int64_t)mc * N;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sa[ps][c] = bb[ro + pcol[c]];
        sb[ps][c] = bb[ro + qcol[c]];
      }
    }
  };
  auto store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int ps = 0; ps < NPASS; ++ps) {
      if constexpr (NP == 1) {
        const float w = smv[ps] ? (float)sw[ps][0] : 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float2 z = make_float2(0.f, 0.f);
          const float2 x = (smv[ps] && pok[c]) ? sa[ps][c] : z;
          const float2 y = qok[c] ? sb[ps][c] : z;
          lds[buf][0][ps * RPI + lrow][lc + 16 * c] = x;
          lds[buf][1][ps * RPI + lrow][lc + 16 * c] = make_float2(w * y.x, w * y.y);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float2 x = sa[ps][c], y = sb[ps][c];
          const bool aok = smv[ps] && pok[c];
          lds[buf][0][ps * RPI + lrow][lc + 16 * c] = make_float2(aok ? x.x : 0.f, aok ? x.y : 0.f);
          lds[buf][1][ps * RPI + lrow][lc + 16 * c] = make_float2(qok[c] ? y.x : 0.f, qok[c] ? y.y : 0.f);
        }
        if (lc == 0) {
#pragma unroll
          for (int p = 0; p < NP; ++p) lw[buf][p][ps * RPI + lrow] = smv[ps] ? (float)sw[ps][p] : 0.f;
        }
      }
    }
  };
  // MASKED: only the blocks marked in `on` (diagonal tiles)
  auto contract = [&](int buf, auto masked) __attribute__((always_inline)) {
    constexpr bool MASKED = decltype(masked)::value;
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks) {
      const int r = ks * 4 + lk;
      float2 av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = lds[buf][0][r][wr * 32 + x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = lds[buf][1][r][wc * 32 + y * 16 + li];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        float2 bw[2];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          if constexpr (NP == 1) {
            bw[y] = bv[y];
          } else {
            const float wp = lw[buf][p][r];
            bw[y] = make_float2(wp * bv[y].x, wp * bv[y].y);
          }
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            if (!MASKED || (on & (1 << (2 * x + y)))) accR[p][x][y] = mfma32(av[x].x, bw[y].x, accR[p][x][y]);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            if (!MASKED || (on & (1 << (2 * x + y)))) accI[p][x][y] = mfma32(av[x].x, bw[y].y, accI[p][x][y]);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            if (!MASKED || (on & (1 << (2 * x + y)))) accR[p][x][y] = mfma32(av[x].y, bw[y].y, accR[p][x][y]);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            if (!MASKED || (on & (1 << (2 * x + y)))) accI[p][x][y] = mfma32(-av[x].y, bw[y].x, accI[p][x][y]);
      }
    }
  };
  // one K step of a half tile (NP = 2 only): point hp, rows 0 .. 31
  auto contract_half = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks) {
      const int r = ks * 4 + lk;
      float2 av[2], bv[2], bw[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = lds[buf][0][r][x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = lds[buf][1][r][wc * 32 + y * 16 + li];
      const float wp = lw[buf][NP == 2 ? hp : 0][r];
#pragma unroll
      for (int y = 0; y < 2; ++y) bw[y] = make_float2(wp * bv[y].x, wp * bv[y].y);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accR[0][x][y] = mfma32(av[x].x, bw[y].x, accR[0][x][y]);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[0][x][y] = mfma32(av[x].x, bw[y].y, accI[0][x][y]);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accR[0][x][y] = mfma32(av[x].y, bw[y].y, accR[0][x][y]);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[0][x][y] = mfma32(-av[x].y, bw[y].x, accI[0][x][y]);
    }
  };
  auto flush = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            hR[p][x][y][r] += (double)accR[p][x][y][r];
            hI[p][x][y][r] += (double)accI[p][x][y][r];
          }
          accR[p][x][y] = f4{0.f, 0.f, 0.f, 0.f};
          accI[p][x][y] = f4{0.f, 0.f, 0.f, 0.f};
        }
  };

  constexpr int FLUSH_STEPS = FLUSH_ROWS / KT;
  const int nsteps = M > mlo ? (M - mlo + KT - 1) / KT : 1;
  if constexpr (NP == 2) {
    if (is_diag) {
      // wave (point pp, role): five of the point's ten lower blocks, flushed to FP64 at
      // the same rows as the single-point kernel; a single point's second pair of waves
      // only keeps the loads and barriers going
      const int pp = wave >> 1, role = wave & 1;
      const bool act = pon[pp];
      f4 dR[5], dI[5];
      double gR[5][4], gI[5][4];
#pragma unroll
      for (int u = 0; u < 5; ++u) {
        dR[u] = dI[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < 4; ++r) gR[u][r] = gI[u][r] = 0.0;
      }
      auto cdiag = [&](int buf) __attribute__((always_inline)) {
        if (!act) return;
        if (role == 0)
          contract_diag5_f32<KT, 0>(lds[buf][0], lds[buf][1], lw[buf][pp], li, lk, dR, dI);
        else
          contract_diag5_f32<KT, 1>(lds[buf][0], lds[buf][1], lw[buf][pp], li, lk, dR, dI);
      };
      auto dflush = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < 5; ++u) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            gR[u][r] += (double)dR[u][r];
            gI[u][r] += (double)dI[u][r];
          }
          dR[u] = dI[u] = f4{0.f, 0.f, 0.f, 0.f};
        }
      };
      load(mlo);
      store(0);
      __syncthreads();
      for (int s = 0; s + 1 < nsteps; ++s) {
        const int cur = s & 1;
        load(mlo + (s + 1) * KT);
        __builtin_amdgcn_sched_barrier(0);
        cdiag(cur);
        __builtin_amdgcn_sched_barrier(0);
        if ((s + 1) % FLUSH_STEPS == 0) dflush();
        store(cur ^ 1);
        __syncthreads();
      }
      cdiag((nsteps - 1) & 1);
      dflush();
      if (!act) return;
      double2 *out = (split == 0 ? a.out : a.partial + (int64_t)(split - 1) * a.split_stride) +
                     (int64_t)pidx[pp] * a.out_stride;
      const double *dg = diag + (int64_t)pidx[pp] * N;
      const bool first = split == 0;   // the exact diagonal enters once
#pragma unroll
      for (int u = 0; u < 5; ++u) {
        const int bx = role == 0 ? DIAG_BX[0][u] : DIAG_BX[1][u];
        const int by = role == 0 ? DIAG_BY[0][u] : DIAG_BY[1][u];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int P = P0 + bx * 16 + 4 * lk + r;
          const int Q = Q0 + by * 16 + li;
          if (P >= N || Q >= N || P < Q) continue;
          if (P == Q) {
            out[(int64_t)P * N + Q] = make_double2(first ? dg[P] : 0.0, 0.0);
            continue;
          }
          out[(int64_t)P * N + Q] = make_double2(gR[u][r], gI[u][r]);
          out[(int64_t)Q * N + P] = make_double2(gR[u][r], -gI[u][r]);
        }
      }
      return;
    }
  }
  // a single point's second pair of waves in a half tile only keeps the loads and
  // barriers going
  const bool hact = !half || hp == 0 || (NP == 2 && pon[NP - 1]);
  auto run = [&](auto masked, auto halfc) __attribute__((always_inline)) {
    constexpr bool HALF = decltype(halfc)::value;
    load(mlo);
    store(0);
    __syncthreads();
    for (int s = 0; s + 1 < nsteps; ++s) {
      const int cur = s & 1;
      load(mlo + (s + 1) * KT);
      __builtin_amdgcn_sched_barrier(0);
      if (HALF) {
        if (hact) contract_half(cur);
      } else {
        contract(cur, masked);
      }
      __builtin_amdgcn_sched_barrier(0);
      if ((s + 1) % FLUSH_STEPS == 0) flush();
      store(cur ^ 1);
      __syncthreads();
    }
    if (HALF) {
      if (hact) contract_half((nsteps - 1) & 1);
    } else {
      contract((nsteps - 1) & 1, masked);
    }
    flush();
  };
  if (is_diag) run(std::integral_constant<bool, true>{}, std::integral_constant<bool, false>{});
  else if (NP == 2 && half) run(std::integral_constant<bool, false>{}, std::integral_constant<bool, true>{});
  else run(std::integral_constant<bool, false>{}, std::integral_constant<bool, false>{});

  double2 *base = split == 0 ? a.out : a.partial + (int64_t)(split - 1) * a.split_stride;
  const bool first = split == 0;   // the exact diagonal enters once
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    // a half tile keeps its one point's sums in set 0
    if (half && p > 0) break;
    const int pt = half ? hp : p;
    if (!(pt == 0 ? pon[0] : pon[NP - 1])) continue;
    const int pid = pt == 0 ? pidx[0] : pidx[NP - 1];
    double2 *out = base + (int64_t)pid * a.out_stride;
    const double *dg = diag + (int64_t)pid * N;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // f32 16x16 accumulator layout: register r of lane l holds row 4 (l/16) + r, column l%16
          const int P = P0 + wr * 32 + x * 16 + 4 * lk + r;
          const int Q = Q0 + wc * 32 + y * 16 + li;
          if (P >= N || Q >= N || !(on & (1 << (2 * x + y)))) continue;
          const double re = hR[p][x][y][r], im = hI[p][x][y][r];
          if (is_diag) {
            if (P < Q) continue;
            if (P == Q) {
              out[(int64_t)P * N + Q] = make_double2(first ? dg[P] : 0.0, 0.0);
              continue;
            }
          }
          out[(int64_t)P * N + Q] = make_double2(re, im);
          out[(int64_t)Q * N + P] = make_double2(re, -im);
        }
  }
}

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// The FP32 contraction on 128 x 128 tiles: eight waves of 64 x 32 (4 x 2 blocks), 16-row
// K steps (32 KB of LDS per stage, double-buffered), one workgroup per CU, FP64 flush
// every FLUSH_ROWS rows as in the 64-wide kernel, XCD-contiguous (tile, point, split)
// order (the 8 XCDs take workgroups round-robin).  Twice the MFMA work per loaded byte.
constexpr int TW32 = 128;
constexpr int LDPW32 = TW32 + 1;
constexpr int KTW32 = 16;

__global__ __launch_bounds__(512) void chi0_f32_t128_kernel(Chi0Args a, const float2 *B32, const double *diag,
                                                            int32_t ntiles, int32_t npts) {
  __shared__ float2 lds[2][2][KTW32][LDPW32];
  const int G = gridDim.x, hw = blockIdx.x;
  const int per = (G + 7) / 8, tall = G % 8 == 0 ? 8 : G % 8;
  const int xcd = hw % 8, loc = hw / 8;
  const int lg = xcd < tall ? xcd * per + loc : tall * per + (xcd - tall) * (per - 1) + loc;
  const int tile = lg % ntiles, p = (lg / ntiles) % npts, split = lg / (ntiles * npts);

  const PointDesc pd = a.pts[p];
  int tr, tc;
  tile_of(tile, tr, tc);
  const int N = a.N;
  const int ms = (int)((((a.M + a.ksplit - 1) / a.ksplit) + KTW32 - 1) / KTW32) * KTW32;
  const int mlo = split * ms;
  const int M = mlo + ms < (int)a.M ? mlo + ms : (int)a.M;
  const int P0 = tr * TW32, Q0 = tc * TW32;
  const bool is_diag = (tr == tc);
  const int tid = threadIdx.x;
  const int lrow = tid >> 5, lc = tid & 31;
  const float2 *bb = B32 + (int64_t)pd.bslot * a.b_slot_stride;
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

  f4 accR[4][2], accI[4][2];
  double hR[4][2][4], hI[4][2][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      accR[x][y] = f4{0.f, 0.f, 0.f, 0.f};
      accI[x][y] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) hR[x][y][r] = hI[x][y][r] = 0.0;
    }

  float2 sa[4], sb[4];
  double sw;
  bool mv;
  auto load = [&](int m0) {
    const int m = m0 + lrow;
    mv = m < M;
    const int mc = mv ? m : 0;
    sw = wrow[mc];
    const int64_t ro = (int64_t)mc * N;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sa[c] = bb[ro + pcol[c]];
      sb[c] = bb[ro + qcol[c]];
    }
  };
  auto store = [&](int buf) {
    const float w = mv ? (float)sw : 0.f;
    const float2 z = make_float2(0.f, 0.f);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float2 x = (mv && pok[c]) ? sa[c] : z;
      const float2 y = qok[c] ? sb[c] : z;
      lds[buf][0][lrow][lc + 32 * c] = x;
      lds[buf][1][lrow][lc + 32 * c] = make_float2(w * y.x, w * y.y);
    }
  };
  auto contract = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < KTW32 / 4; ++ks) {
      float2 av[4], bv[2];
#pragma unroll
      for (int x = 0; x < 4; ++x) av[x] = lds[buf][0][ks * 4 + lk][wr * 64 + x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = lds[buf][1][ks * 4 + lk][wc * 32 + y * 16 + li];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accR[x][y] = mfma32(av[x].x, bv[y].x, accR[x][y]);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[x][y] = mfma32(av[x].x, bv[y].y, accI[x][y]);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accR[x][y] = mfma32(av[x].y, bv[y].y, accR[x][y]);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[x][y] = mfma32(-av[x].y, bv[y].x, accI[x][y]);
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          hR[x][y][r] += (double)accR[x][y][r];
          hI[x][y][r] += (double)accI[x][y][r];
        }
        accR[x][y] = f4{0.f, 0.f, 0.f, 0.f};
        accI[x][y] = f4{0.f, 0.f, 0.f, 0.f};
      }
  };

  constexpr int FLUSH_STEPS = FLUSH_ROWS / KTW32;
  const int nsteps = M > mlo ? (M - mlo + KTW32 - 1) / KTW32 : 1;
  load(mlo);
  store(0);
  __syncthreads();
  for (int s = 0; s + 1 < nsteps; ++s) {
    const int cur = s & 1;
    load(mlo + (s + 1) * KTW32);
    __builtin_amdgcn_sched_barrier(0);
    contract(cur);
    __builtin_amdgcn_sched_barrier(0);
    if ((s + 1) % FLUSH_STEPS == 0) flush();
    store(cur ^ 1);
    __syncthreads();
  }
  contract((nsteps - 1) & 1);
  flush();

  double2 *out = (split == 0 ? a.out : a.partial + (int64_t)(split - 1) * a.split_stride) + (int64_t)p * a.out_stride;
  const double *dg = diag + (int64_t)p * N;
  const bool first = split == 0;   // the exact diagonal enters once
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int P = P0 + wr * 64 + x * 16 + 4 * lk + r;
        const int Q = Q0 + wc * 32 + y * 16 + li;
        if (P >= N || Q >= N) continue;
        const double re = hR[x][y][r], im = hI[x][y][r];
        if (is_diag) {
          if (P < Q) continue;
          if (P == Q) {
            out[(int64_t)P * N + Q] = make_double2(first ? dg[P] : 0.0, 0.0);
            continue;
          }
        }
        out[(int64_t)P * N + Q] = make_double2(re, im);
        out[(int64_t)Q * N + P] = make_double2(re, -im);
      }
}

}  // namespace

hipError_t launch_to_f32(hipStream_t s, const void *in, float2 *out, int64_t n, bool cplx) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(to_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n, cplx ? 1 : 0);
  return hipGetLastError();
}

int64_t diag_exact_scratch_doubles(int64_t M, int N, int npts) {
  const int64_t nchunks = diag_nchunks(M, N);
  const int per = npts < DIAG_MAXP ? npts : DIAG_MAXP;
  return nchunks * per * (int64_t)N;
}

hipError_t launch_diag_exact(hipStream_t s, const void *B, bool cplx, int64_t M, int N, const double *wtab,
                             int npts, double *scratch, double *diag) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int nchunks = (int)diag_nchunks(M, N);
  const int spw = diag_spw(M, N);
  for (int p0 = 0; p0 < npts; p0 += DIAG_MAXP) {
    const int np = npts - p0 < DIAG_MAXP ? npts - p0 : DIAG_MAXP;
    hipLaunchKernelGGL(diag_partial_kernel, dim3((unsigned)((N + 63) / 64), (unsigned)nchunks), dim3(256), 0,
                       s, B, cplx ? 1 : 0, M, N, wtab + (int64_t)p0 * M, np, spw, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t tot = (int64_t)np * N;
    hipLaunchKernelGGL(diag_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, scratch, nchunks,
                       np, N, diag + (int64_t)p0 * N);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int f32_cfg_edge(int cfg) { return cfg == kF32T128 ? 128 : 64; }
int f32_cfg_points_per_wg(int cfg) { return cfg == kF32T64W2 ? 2 : 1; }
const char *f32_cfg_name(int cfg) { return cfg == kF32T128 ? "t128" : cfg == kF32T64W2 ? "t64w2" : "t64"; }

hipError_t launch_chi0_mixed(hipStream_t s, const Chi0Args &args, int32_t npts, const float2 *B32,
                             const double *diag, int prec, int tile) {
  if (npts <= 0) return hipSuccess;
  if (prec != 1) return hipErrorInvalidValue;   // FP32 only; split-BF16 is chi0_bf16.hip
  if (args.ksplit > kMaxSplit) return hipErrorInvalidValue;
  // split 0 writes a.out, split z >= 1 the z-th plane of a.partial (planes npts points apart)
  const int ks = args.ksplit > 1 ? args.ksplit : 1;
  Chi0Args a = args;
  a.ksplit = ks;
  a.split_stride = (int64_t)npts * a.out_stride;
  // the paired kernel needs the launch's pair table; without one the single-point kernel
  // of the same tile computes the same sums
  if (tile == kF32T64W2 && (a.pairs == nullptr || a.npairs <= 0)) tile = kF32T64;
  if (tile == kF32T64W2) {
    Chi0F32Group one{a, npts, B32, diag};
    return launch_chi0_f32_paired_groups(s, &one, 1);
  } else if (tile == kF32T128) {
    const int T = (a.N + TW32 - 1) / TW32;
    const int64_t nwg = (int64_t)T * (T + 1) / 2 * npts * ks;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chi0_f32_t128_kernel, dim3((unsigned)nwg), dim3(512), 0, s, a, B32, diag, T * (T + 1) / 2,
                       npts);
  } else {
    const int T = (a.N + TN - 1) / TN;
    const dim3 grid((unsigned)(T * (T + 1) / 2), (unsigned)npts, (unsigned)ks);
    Chi0F32Launch L{};
    L.ngroups = 1;
    L.g[0] = a;
    L.B32[0] = B32;
    L.diag[0] = diag;
    hipLaunchKernelGGL((chi0_f32_kernel<16, 1>), grid, dim3(256), 0, s, L);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1) return e;
  return launch_split_add(s, a.partial, ks - 1, (int64_t)npts * a.out_stride, a.out);
}

hipError_t launch_chi0_f32_paired_groups(hipStream_t s, const Chi0F32Group *groups, int ngroups) {
  if (ngroups <= 0) return hipSuccess;
  if (ngroups > CHI0_MAX_GROUPS) return hipErrorInvalidValue;
  Chi0F32Launch L{};
  int64_t total = 0;
  int n = 0;
  for (int i = 0; i < ngroups; ++i) {
    const Chi0F32Group &gr = groups[i];
    if (gr.npts <= 0) continue;
    if (gr.a.ksplit > kMaxSplit || gr.a.pairs == nullptr || gr.a.npairs <= 0) return hipErrorInvalidValue;
    Chi0Args a = gr.a;
    a.ksplit = a.ksplit > 1 ? a.ksplit : 1;
    a.split_stride = (int64_t)gr.npts * a.out_stride;
    L.g[n] = a;
    L.B32[n] = gr.B32;
    L.diag[n] = gr.diag;
    L.begin[n] = (int32_t)total;
    total += chi0_paired_workgroups(a);
    if (total > 0x7fffffff) return hipErrorInvalidValue;
    ++n;
  }
  if (n == 0) return hipSuccess;
  L.ngroups = n;
  for (int i = n; i <= CHI0_MAX_GROUPS; ++i) L.begin[i] = (int32_t)total;
  hipLaunchKernelGGL((chi0_f32_kernel<16, 2>), dim3((unsigned)total), dim3(256), 0, s, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int i = 0; i < n; ++i) {   // each group's later row splits, added in split order
    const Chi0Args &a = L.g[i];
    if (a.ksplit <= 1) continue;
    e = launch_split_add(s, a.partial, a.ksplit - 1, a.split_stride, a.out);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rpa
