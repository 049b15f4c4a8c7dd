// Fit coefficients of atomic-orbital systems, built on the device: the MO transform of
// the pair-fit coefficients (Sec. 2.2, the expansion of psi*_a(k) psi_i(k+q) from that of
// the basis-function products),
//
//   C^{ai}_gamma(k+q,k) = sum_{mu nu} conj(c~_{mu a}(k)) C^{mu nu}_gamma(k,q) c~_{nu i}(k (+) q),
//
// with c~ the KS coefficients after the periodic projector (Sec. 2.3; applied by the
// caller).  The library's B is the complex conjugate, B^gamma_ia = conj(C^{ai}_gamma), so
// that chi0_PQ = sum conj(B^P) w B^Q is the fit-basis polarizability of Sec. 2.2 with its
// C_gamma C*_gamma' index order.  Per (q, k) block: C from the Philox generator (stream 1),
// then two batched complex FP64 MFMA products, the occupied index first (the cheaper order):
//   T1[mu][i][gamma] = sum_nu c~_{nu i} C[mu][nu][gamma]                 (batch over mu)
//   B[i][a][gamma]   = conj(sum_mu conj(c~_{mu a}) T1[mu][i][gamma])     (batch over i;
//                      the conjugate taken at the store)
// Both are O[b][m][n] = sum_k op(X[b][k][m]) Y[b][k][n] with the contraction index k
// slowest in both operands, so an output tile streams 16-row panels of X and Y through
// LDS exactly as the chi0 contraction does (64 x 64 tiles; 16 x 128 for the thin
// occupied-index output of the first product).
#include "common.hpp"

namespace rpa {
namespace {

constexpr int TT = 64;         // output tile edge
constexpr int TLP = TT + 1;    // LDS row pitch (complex elements)
constexpr int TK = 16;         // contraction rows per LDS step

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct TnArgs {
  const double2 *X;   // X[b][k][m] at X + b * sxb + k * ldx + m
  int64_t ldx, sxb;
  const double2 *Y;   // Y[b][k][n] at Y + b * syb + k * ldy + n
  int64_t ldy, syb;
  double2 *O;         // O[b][m][n] at O + b * sob + m * ldo + n
  int64_t ldo, sob;
  int32_t M, N, K;
  int32_t conj_out;   // store conj(O) instead of O
};

// O[b][m][n] = sum_k op(X[b][k][m]) Y[b][k][n], op = complex conjugation when CONJ.
// Four waves, each a 32 x 32 sub-tile (2 x 2 blocks of 16 x 16, real and imaginary
// accumulators); out-of-range rows and columns read a clamped address and are zeroed at
// the LDS store.
template <bool CONJ>
__global__ __launch_bounds__(256) void zgemm_tn_kernel(TnArgs g) {
  __shared__ double2 lds[2][2][TK][TLP];
  const int b = blockIdx.z;
  const int m0 = blockIdx.y * TT, n0 = blockIdx.x * TT;
  const double2 *X = g.X + (int64_t)b * g.sxb;
  const double2 *Y = g.Y + (int64_t)b * g.syb;
  const int tid = threadIdx.x, lrow = tid >> 4, lc = tid & 15;
  int mcol[4], ncol[4];
  bool mok[4], nok[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int m = m0 + lc + 16 * c, n = n0 + lc + 16 * c;
    mok[c] = m < g.M;
    nok[c] = n < g.N;
    mcol[c] = mok[c] ? m : 0;
    ncol[c] = nok[c] ? n : 0;
  }
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;

  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      accR[x][y] = d4{0.0, 0.0, 0.0, 0.0};
      accI[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    }

  double2 sa[4], sb[4];
  bool kv;
  auto load = [&](int k0) {
    const int k = k0 + lrow;
    kv = k < g.K;
    const int64_t kc = kv ? k : 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sa[c] = X[kc * g.ldx + mcol[c]];
      sb[c] = Y[kc * g.ldy + ncol[c]];
    }
  };
  auto store = [&](int buf) {
    const double2 z = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      lds[buf][0][lrow][lc + 16 * c] = (kv && mok[c]) ? sa[c] : z;
      lds[buf][1][lrow][lc + 16 * c] = (kv && nok[c]) ? sb[c] : z;
    }
  };
  auto contract = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      double2 av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = lds[buf][0][ks * 4 + lk][wr * 32 + x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = lds[buf][1][ks * 4 + lk][wc * 32 + y * 16 + li];
      // a b = (ar br - ai bi) + i (ar bi + ai br); conj(a) b flips the sign of ai
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
        for (int y = 0; y < 2; ++y) accR[x][y] = mfma(CONJ ? av[x].y : -av[x].y, bv[y].y, accR[x][y]);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[x][y] = mfma(CONJ ? -av[x].y : av[x].y, bv[y].x, accI[x][y]);
    }
  };

  const int nsteps = g.K > 0 ? (g.K + TK - 1) / TK : 1;
  load(0);
  store(0);
  __syncthreads();
  for (int s = 0; s + 1 < nsteps; ++s) {
    const int cur = s & 1;
    load((s + 1) * TK);
    __builtin_amdgcn_sched_barrier(0);
    contract(cur);
    __builtin_amdgcn_sched_barrier(0);
    store(cur ^ 1);
    __syncthreads();
  }
  contract((nsteps - 1) & 1);

  double2 *O = g.O + (int64_t)b * g.sob;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // f64 16x16x4 accumulator layout: register r of lane l holds row l/16 + 4 r, column l%16
        const int m = m0 + wr * 32 + x * 16 + lk + 4 * r;
        const int n = n0 + wc * 32 + y * 16 + li;
        if (m < g.M && n < g.N)
          O[(int64_t)m * g.ldo + n] = make_double2(accR[x][y][r], g.conj_out ? -accI[x][y][r] : accI[x][y][r]);
      }
}

// The same product for thin outputs (M a few tens, the occupied count): 16 x 128 tiles,
// each wave a 16 x 32 strip (two 16 x 16 blocks), so no MFMA work is spent on padding rows.
constexpr int TNW = 128;
template <bool CONJ>
__global__ __launch_bounds__(256) void zgemm_tn16_kernel(TnArgs g) {
  __shared__ double2 la[2][TK][17];
  __shared__ double2 lb[2][TK][TNW + 1];
  const int b = blockIdx.z;
  const int m0 = blockIdx.y * 16, n0 = blockIdx.x * TNW;
  const double2 *X = g.X + (int64_t)b * g.sxb;
  const double2 *Y = g.Y + (int64_t)b * g.syb;
  const int tid = threadIdx.x, lrow = tid >> 4, lc = tid & 15;
  const bool mok = m0 + lc < g.M;
  const int mcol = mok ? m0 + lc : 0;
  int ncol[8];
  bool nok[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int n = n0 + lc + 16 * c;
    nok[c] = n < g.N;
    ncol[c] = nok[c] ? n : 0;
  }
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  d4 accR[2], accI[2];
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    accR[y] = d4{0.0, 0.0, 0.0, 0.0};
    accI[y] = d4{0.0, 0.0, 0.0, 0.0};
  }
  double2 sa, sb[8];
  bool kv;
  auto load = [&](int k0) {
    const int k = k0 + lrow;
    kv = k < g.K;
    const int64_t kc = kv ? k : 0;
    sa = X[kc * g.ldx + mcol];
#pragma unroll
    for (int c = 0; c < 8; ++c) sb[c] = Y[kc * g.ldy + ncol[c]];
  };
  auto store = [&](int buf) {
    const double2 z = make_double2(0.0, 0.0);
    la[buf][lrow][lc] = (kv && mok) ? sa : z;
#pragma unroll
    for (int c = 0; c < 8; ++c) lb[buf][lrow][lc + 16 * c] = (kv && nok[c]) ? sb[c] : z;
  };
  auto contract = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const double2 av = la[buf][ks * 4 + lk][li];
      double2 bv[2];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = lb[buf][ks * 4 + lk][wave * 32 + y * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) accR[y] = mfma(av.x, bv[y].x, accR[y]);
#pragma unroll
      for (int y = 0; y < 2; ++y) accI[y] = mfma(av.x, bv[y].y, accI[y]);
#pragma unroll
      for (int y = 0; y < 2; ++y) accR[y] = mfma(CONJ ? av.y : -av.y, bv[y].y, accR[y]);
#pragma unroll
      for (int y = 0; y < 2; ++y) accI[y] = mfma(CONJ ? -av.y : av.y, bv[y].x, accI[y]);
    }
  };
  const int nsteps = g.K > 0 ? (g.K + TK - 1) / TK : 1;
  load(0);
  store(0);
  __syncthreads();
  for (int s = 0; s + 1 < nsteps; ++s) {
    const int cur = s & 1;
    load((s + 1) * TK);
    __builtin_amdgcn_sched_barrier(0);
    contract(cur);
    __builtin_amdgcn_sched_barrier(0);
    store(cur ^ 1);
    __syncthreads();
  }
  contract((nsteps - 1) & 1);
  double2 *O = g.O + (int64_t)b * g.sob;
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + lk + 4 * r;
      const int n = n0 + wave * 32 + y * 16 + li;
      if (m < g.M && n < g.N)
        O[(int64_t)m * g.ldo + n] = make_double2(accR[y][r], g.conj_out ? -accI[y][r] : accI[y][r]);
    }
}

hipError_t launch_tn(hipStream_t s, bool conj, const TnArgs &g, int batch) {
  if (batch <= 0 || g.M <= 0 || g.N <= 0) return hipSuccess;
  if (batch > 65535) return hipErrorInvalidValue;
  if (g.M <= 32) {   // thin output: 16-row tiles
    const dim3 grid((unsigned)((g.N + TNW - 1) / TNW), (unsigned)((g.M + 15) / 16), (unsigned)batch);
    if (conj) hipLaunchKernelGGL(zgemm_tn16_kernel<true>, grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL(zgemm_tn16_kernel<false>, grid, dim3(256), 0, s, g);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((g.N + TT - 1) / TT), (unsigned)((g.M + TT - 1) / TT), (unsigned)batch);
  if (conj) hipLaunchKernelGGL(zgemm_tn_kernel<true>, grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL(zgemm_tn_kernel<false>, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace

int64_t ao_scratch_bytes(int32_t nbas, int32_t nocc, int32_t naux) {
  return ((int64_t)nbas * nbas * naux + (int64_t)nbas * nocc * naux) * 16;
}

hipError_t launch_ao_B(hipStream_t s, uint64_t seed, double sigma, int32_t nk, int32_t iq, int32_t ik, int32_t nbas,
                       int32_t nocc, int32_t nvirt, int32_t naux, const double2 *c_occ, const double2 *c_virt,
                       void *scratch, double2 *out) {
  double2 *C = reinterpret_cast<double2 *>(scratch);
  double2 *T1 = C + (int64_t)nbas * nbas * naux;
  hipError_t e = launch_philox_C(s, seed, sigma, nk, iq, ik, nbas, naux, C);
  if (e != hipSuccess) return e;
  TnArgs g1{};   // T1[mu][i][gamma] = sum_nu c_occ[nu][i] C[mu][nu][gamma]
  g1.X = c_occ; g1.ldx = nocc; g1.sxb = 0;
  g1.Y = C; g1.ldy = naux; g1.syb = (int64_t)nbas * naux;
  g1.O = T1; g1.ldo = naux; g1.sob = (int64_t)nocc * naux;
  g1.M = nocc; g1.N = naux; g1.K = nbas;
  e = launch_tn(s, false, g1, nbas);
  if (e != hipSuccess) return e;
  TnArgs g2{};   // B[i][a][gamma] = conj(sum_mu conj(c_virt[mu][a]) T1[mu][i][gamma])
  g2.X = c_virt; g2.ldx = nvirt; g2.sxb = 0;
  g2.Y = T1; g2.ldy = (int64_t)nocc * naux; g2.syb = naux;
  g2.O = out; g2.ldo = naux; g2.sob = (int64_t)nvirt * naux;
  g2.M = nvirt; g2.N = naux; g2.K = nbas;
  g2.conj_out = 1;
  return launch_tn(s, true, g2, nocc);
}

}  // namespace rpa
