// Split-BF16 and split-FP16 chi0 from prepared operands (the reduced-precision paths of
// the chi0 build, periodic RPA section: chi0_PQ(q, i w) = sum_k zeta_k sum_ia
// conj(B_iaP) w_ia B_iaQ).
//
// The operands are written once into HBM in the form the 16-bit MFMA consumes:
//   L   = s_L B            per q (shared by every frequency of that q)
//   R_p = s_p w_p zeta B   per point p of a launch
// every element x of both split in FP64 as hi = t(x), lo = t(x - hi), t the rounding to
// the 16-bit format (bf16, or fp16), for its real and imaginary parts: four planes (re hi,
// re lo, im hi, im lo).  The contraction then does nothing but copy panels into LDS and
// issue MFMAs:
//   Re chi0 += Lr Rr + Li Ri,   Im chi0 += Lr Ri - Li Rr,
// each real product as hi*hi + hi*lo + lo*hi with FP32 accumulation (the lo*lo term is
// below the FP32 rounding of the sum).  The two formats differ in what hi + lo keeps:
// bf16's 8-bit significands leave about 2^-17 of each element (enough for a relative
// energy error near 1e-8, not for 1e-6 Ha on every system), fp16's 11-bit significands
// about 2^-22.  fp16 has a narrow exponent range, so the fp16 operands are scaled by
// powers of two (s_L from the largest |Re|, |Im| of the B slab, s_p from that times the
// largest |w_m zeta_k| of the point) that put their largest element just below 2^14:
// hi*hi stays far inside FP32's range and an element below fp16's normal range carries
// an error below 2^-39 of the largest one.  The reduction divides by s_L s_p (exact).
// bf16 keeps s = 1.  The contraction rows are cut into splits of at
// most BF16_SPLIT_ROWS rows; each split's FP32 tile goes to a partial buffer, so no FP32
// sum runs over more rows than that, and a reduction adds the splits in FP64 in a fixed
// order, mirrors the lower triangle into the Hermitian matrix and puts in the diagonal
// from the exact FP64 pass (a sum of same-signed terms whose rounding errors would not
// cancel).
//
// Prepared layout of one operand (bf16 elements, Mp = M rounded up to 32 rows, Np = N
// rounded up to the 128-wide output tile; rows >= M and columns >= N are zero):
//   element (m, n, plane) at ((m / 32 * 4 + plane) * Np + n) * 32 + pos(m % 32, n)
//   pos(r, n) = ((r / 8) ^ ((n / 2) % 4)) * 8 + r % 8
// so the 32 rows of one column are 64 contiguous bytes, a 128-column panel of one plane
// is 8 KB contiguous (copied into LDS as is), and the XOR on the 16-byte segments makes
// the MFMA fragment reads from LDS free of bank conflicts (the eight lanes served
// together read eight columns at one segment index: the XOR spreads them over the
// 128 bytes the LDS delivers per clock).
#include <type_traits>

#include "common.hpp"

namespace rpa {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int HT = 128;          // column padding of the prepared layout (the largest tile)
constexpr int HK = 32;           // contraction rows per step (the K of one BF16 MFMA)
constexpr int PREP_COLS = 64;    // columns per preparation workgroup
constexpr int PREP_MAXP = 16;    // points per preparation launch
// a contraction workgroup owns a TW x TW tile (TW = 64 or 128) with TW / 16 waves of
// (TW / 2) x 32 each: 2 x 2 waves for 64, 2 x 4 for 128

__device__ __forceinline__ void tile_of(int t, int &tr, int &tc) {
  int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  tr = r;
  tc = t - r * (r + 1) / 2;
}

__device__ __forceinline__ int seg_pos(int s, int n) { return s ^ ((n >> 1) & 3); }

// hi = t(x) (round to nearest even through FP32), lo = t(x - hi) with the difference
// taken in FP64 (exact: hi has at most 11 significant bits); two values at once, packed
// as the MFMA reads them.  t = bf16, or fp16 when F16.
template <bool F16>
__device__ __forceinline__ void split_pair(double x0, double x1, unsigned &hi, unsigned &lo) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  typedef __bf16 b2v __attribute__((ext_vector_type(2)));
  typedef _Float16 h2v __attribute__((ext_vector_type(2)));
  const f2v xf = {(float)x0, (float)x1};
  if (F16) {
    const h2v h = __builtin_convertvector(xf, h2v);
    hi = __builtin_bit_cast(unsigned, h);
    const f2v r = {(float)(x0 - (double)h[0]), (float)(x1 - (double)h[1])};
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, h2v));
  } else {
    hi = __builtin_bit_cast(unsigned, __builtin_convertvector(xf, b2v));
    const double h0 = (double)__builtin_bit_cast(float, hi << 16);
    const double h1 = (double)__builtin_bit_cast(float, hi & 0xffff0000u);
    const f2v r = {(float)(x0 - h0), (float)(x1 - h1)};
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, b2v));
  }
}

// Power of two that puts a largest magnitude m just below 2^14 (1 for m = 0 or not finite).
__device__ __forceinline__ double f16_scale_of(double m) {
  if (!(m > 0.0) || !(m < 1e300)) return 1.0;
  int e;
  (void)frexp(m, &e);          // m < 2^e
  return ldexp(1.0, 14 - e);
}

// ------------------------------------------------------------------ preparation
// One workgroup: PREP_STEPS steps of 32 rows x 64 columns.  Each step's B rows are read
// coalesced into LDS, then thread (c, s) splits rows 8 s .. 8 s + 7 of column c for every
// point (or once, unscaled, when wtab is null) and writes one 16-byte segment per plane.
// With dpart set, the workgroup also sums w_m |B_mc|^2 in FP64 over its rows for every
// point (the exact diagonal of chi0, from the unsplit values it holds anyway): rows in
// order within a thread, then the four row groups in a fixed order, one partial per
// (workgroup row chunk, point, column).
constexpr int PREP_STEPS = 4;

template <bool CPLX, bool NTS, bool F16>
__global__ __launch_bounds__(256) void bf16_prepare_kernel(const void *B, int64_t M, int N, int Np,
                                                           const double *wtab, int64_t w_stride, int np,
                                                           unsigned short *out, int64_t out_stride,
                                                           double *dpart, const double *scale) {
  // the row tile and, after the last step, the diagonal's reduction buffer share one LDS
  // array (37 KB a workgroup in all: four workgroups per CU)
  constexpr int TB_BYTES = HK * (PREP_COLS + 1) * 16, RED_BYTES = 4 * PREP_MAXP * PREP_COLS * 8;
  __shared__ __attribute__((aligned(16))) char lds_raw[TB_BYTES > RED_BYTES ? TB_BYTES : RED_BYTES];
  double2 (*tb)[PREP_COLS + 1] = reinterpret_cast<double2 (*)[PREP_COLS + 1]>(lds_raw);
  double (*red)[PREP_MAXP][PREP_COLS] = reinterpret_cast<double (*)[PREP_MAXP][PREP_COLS]>(lds_raw);
  __shared__ double wl[PREP_MAXP][HK];
  const int c0 = blockIdx.y * PREP_COLS;
  const int64_t nkc = (M + HK - 1) / HK;
  const int tid = threadIdx.x;
  const int c = tid >> 2, s = tid & 3;
  const int n = c0 + c;
  const int64_t unit = seg_pos(s, n);   // 16-byte segment within the column's 64 bytes
  const int reps = wtab ? np : 1;
  double dsum[PREP_MAXP];
#pragma unroll
  for (int p = 0; p < PREP_MAXP; ++p) dsum[p] = 0.0;
  for (int t = 0; t < PREP_STEPS; ++t) {
    const int64_t kc = (int64_t)blockIdx.x * PREP_STEPS + t;
    if (kc >= nkc) break;   // uniform over the workgroup
    const int64_t m0 = kc * HK;
    {
      const int col = tid & 63, r0 = tid >> 6;
      const int nn = c0 + col;
#pragma unroll
      for (int j = 0; j < HK / 4; ++j) {
        const int r = r0 + 4 * j;
        const int64_t m = m0 + r;
        double2 v = make_double2(0.0, 0.0);
        if (m < M && nn < N) {
          if (CPLX) v = reinterpret_cast<const double2 *>(B)[m * N + nn];
          else v.x = reinterpret_cast<const double *>(B)[m * N + nn];
        }
        tb[r][col] = v;
      }
      if (wtab) {
        for (int e = tid; e < np * HK; e += 256) {
          const int p = e / HK, r = e % HK;
          wl[p][r] = (m0 + r < M) ? wtab[(int64_t)p * w_stride + m0 + r] : 0.0;
        }
      }
    }
    __syncthreads();
    double2 v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = tb[8 * s + e][c];
    double b2[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) b2[e] = v[e].x * v[e].x + v[e].y * v[e].y;
    for (int p = 0; p < reps; ++p) {
      unsigned hr[4], lr[4], hi_[4], li_[4];
      const double sc = scale ? scale[p] : 1.0;   // a power of two: exact
#pragma unroll
      for (int e2 = 0; e2 < 4; ++e2) {
        const double w0 = (wtab ? wl[p][8 * s + 2 * e2] : 1.0) * sc;
        const double w1 = (wtab ? wl[p][8 * s + 2 * e2 + 1] : 1.0) * sc;
        split_pair<F16>(w0 * v[2 * e2].x, w1 * v[2 * e2 + 1].x, hr[e2], lr[e2]);
        if (CPLX) split_pair<F16>(w0 * v[2 * e2].y, w1 * v[2 * e2 + 1].y, hi_[e2], li_[e2]);
      }
      if (dpart) {
        double d = 0.0;
#pragma unroll
        for (int e = 0; e < 8; ++e) d += wl[p][8 * s + e] * b2[e];
#pragma unroll
        for (int q = 0; q < PREP_MAXP; ++q)
          if (q == p) dsum[q] += d;
      }
      uint4 *o = reinterpret_cast<uint4 *>(out + (int64_t)p * out_stride);
      // 16-byte units: plane base ((kc * 4 + plane) * Np + n) * 4, then the segment.  The
      // right operands (one per point, far more than the caches hold) are written with
      // non-temporal stores; the left operand, read again soon, through the caches.
      typedef unsigned u4v __attribute__((ext_vector_type(4)));
      u4v *o0 = reinterpret_cast<u4v *>(&o[((kc * 4 + 0) * Np + n) * 4 + unit]);
      u4v *o1 = reinterpret_cast<u4v *>(&o[((kc * 4 + 1) * Np + n) * 4 + unit]);
      u4v *o2 = reinterpret_cast<u4v *>(&o[((kc * 4 + 2) * Np + n) * 4 + unit]);
      u4v *o3 = reinterpret_cast<u4v *>(&o[((kc * 4 + 3) * Np + n) * 4 + unit]);
      const u4v vhr = {hr[0], hr[1], hr[2], hr[3]}, vlr = {lr[0], lr[1], lr[2], lr[3]};
      if (NTS) {
        __builtin_nontemporal_store(vhr, o0);
        __builtin_nontemporal_store(vlr, o1);
        if (CPLX) {
          __builtin_nontemporal_store(u4v{hi_[0], hi_[1], hi_[2], hi_[3]}, o2);
          __builtin_nontemporal_store(u4v{li_[0], li_[1], li_[2], li_[3]}, o3);
        }
      } else {
        *o0 = vhr;
        *o1 = vlr;
        if (CPLX) {
          *o2 = u4v{hi_[0], hi_[1], hi_[2], hi_[3]};
          *o3 = u4v{li_[0], li_[1], li_[2], li_[3]};
        }
      }
    }
    __syncthreads();   // tb and wl are refilled by the next step
  }
  if (dpart && wtab) {
    __syncthreads();   // every step's reads of tb are done
#pragma unroll
    for (int p = 0; p < PREP_MAXP; ++p) red[s][p][c] = dsum[p];
    __syncthreads();
    for (int e = tid; e < np * PREP_COLS; e += 256) {
      const int p = e / PREP_COLS, cc = e % PREP_COLS;
      if (c0 + cc < N)
        dpart[((int64_t)blockIdx.x * np + p) * N + c0 + cc] =
            ((red[0][p][cc] + red[1][p][cc]) + red[2][p][cc]) + red[3][p][cc];
    }
  }
}

// diag[p][n] = sum over the row chunks, in order, of the partials
__global__ __launch_bounds__(256) void prepare_diag_reduce_kernel(const double *dpart, int64_t nchunks, int np, int N,
                                                                  double *diag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)np * N) return;
  // chunks added in order, loads issued 16 at a time (latency-bound: few workgroups)
  const int64_t st = (int64_t)np * N;
  double d = 0.0;
  int64_t c = 0;
  for (; c + 16 <= nchunks; c += 16) {
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = dpart[(c + u) * st + i];
#pragma unroll
    for (int u = 0; u < 16; ++u) d += t[u];
  }
  for (; c < nchunks; ++c) d += dpart[c * st + i];
  diag[i] = d;
}

// ------------------------------------------------------------------ contraction
struct HerkArgs {
  const unsigned short *L;   // prepared left operands, one per B slot
  int64_t l_stride;          // elements between slots
  const unsigned short *R;   // prepared right operands, one per point of the launch
  int64_t r_stride;
  const PointDesc *pts;
  float2 *part;              // [npts][nsplit][ntiles][TW * TW]
  int32_t Np, ntiles, nsplit, kc_per_split;
  int64_t nkc;               // steps in the whole contraction (Mp / 32)
};

__device__ __forceinline__ f4 mfma16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(h8 a, h8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// -x of eight packed 16-bit values (the sign is bit 15 in both formats)
template <class V>
__device__ __forceinline__ V negate(V x) {
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  u4v u = __builtin_bit_cast(u4v, x);
  u ^= 0x80008000u;
  return __builtin_bit_cast(V, u);
}

// one 8 KB panel (128 columns x 32 rows of one plane) from HBM straight into LDS: one
// 16-byte load per thread; wave w fills units w * 64 .. w * 64 + 63
__device__ __forceinline__ void copy_panel(const uint4 *src, uint4 *dst, int wave, int lane) {
  const int u = wave * 64;
  __builtin_amdgcn_global_load_lds((const void *)(src + u + lane),
                                   (__attribute__((address_space(3))) void *)(dst + u), 16, 0, 0);
}

// A launch holds up to BF16_MAX_GROUPS groups (sub-batches of one or of several jobs of
// a serving loop); group g owns workgroups [begin[g], begin[g + 1]).
struct HerkLaunch {
  int32_t ngroups;
  int32_t begin[BF16_MAX_GROUPS + 1];
  HerkArgs g[BF16_MAX_GROUPS];
};

template <bool CPLX, int TW, bool F16>
__global__ __launch_bounds__(4 * TW) void herk_bf16x3_kernel(HerkLaunch hl) {
  typedef typename std::conditional<F16, h8, bf8>::type bf8;   // the fragment type
  constexpr int NPL = CPLX ? 4 : 2;
  constexpr int XB = TW / 32;      // 16-row blocks per wave (wave rows: TW / 2)
  constexpr int NWC = TW / 32;     // waves across the tile's columns (32 columns each)
  // [buffer][operand][plane][column * 4 + segment], 16-byte units
  __shared__ __attribute__((aligned(16))) uint4 lds[2][2][NPL][TW * 4];

  // workgroups go to the 8 XCDs round-robin; give each XCD a contiguous range of the
  // (group, then tile fastest, then split, then point) order so that its L2 serves
  // shared panels
  const int G = gridDim.x, hw = blockIdx.x;
  const int per = (G + 7) / 8, tall = G % 8 == 0 ? 8 : G % 8;
  const int xcd = hw % 8, loc = hw / 8;
  const int lgg = xcd < tall ? xcd * per + loc : tall * per + (xcd - tall) * (per - 1) + loc;
  // the group (uniform over the workgroup), selected with constant indices only so the
  // arguments stay in scalar registers
  int gi = 0;
#pragma unroll
  for (int k = 1; k < BF16_MAX_GROUPS; ++k)
    if (k < hl.ngroups && lgg >= hl.begin[k]) gi = k;
  HerkArgs h = hl.g[0];
  int g0 = hl.begin[0];
#pragma unroll
  for (int k = 1; k < BF16_MAX_GROUPS; ++k)
    if (k == gi) {
      h = hl.g[k];
      g0 = hl.begin[k];
    }
  const int lg = lgg - g0;
  const int tile = lg % h.ntiles, split = (lg / h.ntiles) % h.nsplit, p = lg / (h.ntiles * h.nsplit);
  int tr, tc;
  tile_of(tile, tr, tc);
  const PointDesc pd = h.pts[p];
  const int tid = threadIdx.x, lane = tid & 63;
  // wave index as a scalar: the LDS base of a direct-to-LDS load must be wave-uniform
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave / NWC, wc = wave % NWC;   // (TW / 2) rows x 32 columns of the tile
  const int li = lane & 15, lk = lane >> 4;

  const uint4 *Lg = reinterpret_cast<const uint4 *>(h.L + (int64_t)pd.bslot * h.l_stride) + (int64_t)tr * TW * 4;
  const uint4 *Rg = reinterpret_cast<const uint4 *>(h.R + (int64_t)p * h.r_stride) + (int64_t)tc * TW * 4;
  const int64_t plane_units = (int64_t)h.Np * 4;   // 16-byte units of one plane of one step
  const int64_t kc0 = (int64_t)split * h.kc_per_split;
  const int64_t kc1 = kc0 + h.kc_per_split < h.nkc ? kc0 + h.kc_per_split : h.nkc;
  const int nsteps = (int)(kc1 - kc0);

  auto issue = [&](int buf, int64_t kc) {
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl) {
      const int64_t off = (kc * 4 + pl) * plane_units;
      copy_panel(Lg + off, lds[buf][0][pl], wave, lane);
      copy_panel(Rg + off, lds[buf][1][pl], wave, lane);
    }
  };

  f4 accR[XB][2], accI[XB][2];
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      accR[x][y] = f4{0.f, 0.f, 0.f, 0.f};
      accI[x][y] = f4{0.f, 0.f, 0.f, 0.f};
    }

  // fragment of the block at column `col` of a panel: lane (li, lk) reads rows
  // 8 lk .. 8 lk + 7 of column col
  auto frag = [&](const uint4 *panel, int col) -> bf8 {
    return __builtin_bit_cast(bf8, panel[col * 4 + seg_pos(lk, col)]);
  };

  auto contract = [&](int buf) {
    bf8 Bv[2][NPL];
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int pl = 0; pl < NPL; ++pl) Bv[y][pl] = frag(lds[buf][1][pl], wc * 32 + y * 16 + li);
#pragma unroll
    for (int x = 0; x < XB; ++x) {
      bf8 A[NPL];
#pragma unroll
      for (int pl = 0; pl < NPL; ++pl) A[pl] = frag(lds[buf][0][pl], wr * (TW / 2) + x * 16 + li);
      // Re: Lr Rr (+ Li Ri); each as hi hi + hi lo + lo hi
#pragma unroll
      for (int y = 0; y < 2; ++y) accR[x][y] = mfma16(A[0], Bv[y][0], accR[x][y]);
#pragma unroll
      for (int y = 0; y < 2; ++y) accR[x][y] = mfma16(A[0], Bv[y][1], accR[x][y]);
#pragma unroll
      for (int y = 0; y < 2; ++y) accR[x][y] = mfma16(A[1], Bv[y][0], accR[x][y]);
      if (CPLX) {
        const bf8 nh = negate(A[2]), nl = negate(A[3]);
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[x][y] = mfma16(A[0], Bv[y][2], accI[x][y]);
#pragma unroll
        for (int y = 0; y < 2; ++y) accR[x][y] = mfma16(A[2], Bv[y][2], accR[x][y]);
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[x][y] = mfma16(A[0], Bv[y][3], accI[x][y]);
#pragma unroll
        for (int y = 0; y < 2; ++y) accR[x][y] = mfma16(A[2], Bv[y][3], accR[x][y]);
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[x][y] = mfma16(A[1], Bv[y][2], accI[x][y]);
#pragma unroll
        for (int y = 0; y < 2; ++y) accR[x][y] = mfma16(A[3], Bv[y][2], accR[x][y]);
        // Im: - Li Rr
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[x][y] = mfma16(nh, Bv[y][0], accI[x][y]);
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[x][y] = mfma16(nh, Bv[y][1], accI[x][y]);
#pragma unroll
        for (int y = 0; y < 2; ++y) accI[x][y] = mfma16(nl, Bv[y][0], accI[x][y]);
      }
    }
  };

  // Diagonal tiles need only the NLB 16 x 16 blocks on or below the diagonal; they are
  // dealt out in row-major order, a contiguous run of at most MAXB blocks per wave (so a
  // wave's blocks share few block rows), each summed exactly as in an off-diagonal tile.
  constexpr int NB16 = TW / 16, NW = TW / 16;
  constexpr int NLB = NB16 * (NB16 + 1) / 2, MAXB = (NLB + NW - 1) / NW;
  const int kb0 = wave * NLB / NW, kb1 = (wave + 1) * NLB / NW;
  int bxs[MAXB], bys[MAXB];
#pragma unroll
  for (int j = 0; j < MAXB; ++j) {
    const int k = kb0 + j < kb1 ? kb0 + j : kb0;
    int bx = 0;
    while ((bx + 1) * (bx + 2) / 2 <= k) ++bx;
    bxs[j] = bx;
    bys[j] = k - bx * (bx + 1) / 2;
  }
  f4 dR[MAXB], dI[MAXB];
#pragma unroll
  for (int j = 0; j < MAXB; ++j) {
    dR[j] = f4{0.f, 0.f, 0.f, 0.f};
    dI[j] = f4{0.f, 0.f, 0.f, 0.f};
  }
  auto contract_diag = [&](int buf) {
#pragma unroll
    for (int j = 0; j < MAXB; ++j) {
      if (kb0 + j >= kb1) break;   // uniform over the wave
      bf8 A[NPL], Bv[NPL];
#pragma unroll
      for (int pl = 0; pl < NPL; ++pl) {
        A[pl] = frag(lds[buf][0][pl], bxs[j] * 16 + li);
        Bv[pl] = frag(lds[buf][1][pl], bys[j] * 16 + li);
      }
      dR[j] = mfma16(A[0], Bv[0], dR[j]);
      dR[j] = mfma16(A[0], Bv[1], dR[j]);
      dR[j] = mfma16(A[1], Bv[0], dR[j]);
      if (CPLX) {
        const bf8 nh = negate(A[2]), nl = negate(A[3]);
        dI[j] = mfma16(A[0], Bv[2], dI[j]);
        dR[j] = mfma16(A[2], Bv[2], dR[j]);
        dI[j] = mfma16(A[0], Bv[3], dI[j]);
        dR[j] = mfma16(A[2], Bv[3], dR[j]);
        dI[j] = mfma16(A[1], Bv[2], dI[j]);
        dR[j] = mfma16(A[3], Bv[2], dR[j]);
        dI[j] = mfma16(nh, Bv[0], dI[j]);
        dI[j] = mfma16(nh, Bv[1], dI[j]);
        dI[j] = mfma16(nl, Bv[0], dI[j]);
      }
    }
  };
  const bool dtile = tr == tc;

  auto run = [&](auto diag_tag) {
    constexpr bool D = decltype(diag_tag)::value;
    if (nsteps <= 0) return;
    issue(0, kc0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
      const int cur = s & 1;
      if (s + 1 < nsteps) issue(cur ^ 1, kc0 + s + 1);
      if (D) contract_diag(cur);
      else contract(cur);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
  };
  if (dtile) run(std::integral_constant<bool, true>{});
  else run(std::integral_constant<bool, false>{});

  // FP32 tile of this split: row i, column j of the TW x TW tile at i * TW + j;
  // accumulator register r of lane (li, lk) holds row 4 lk + r, column li of a block.
  // Diagonal tiles write only their lower blocks (the reduction reads nothing else).
  float2 *o = h.part + (((int64_t)p * h.nsplit + split) * h.ntiles + tile) * (TW * TW);
  if (dtile) {
#pragma unroll
    for (int j = 0; j < MAXB; ++j) {
      if (kb0 + j >= kb1) break;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = bxs[j] * 16 + 4 * lk + r, jj = bys[j] * 16 + li;
        o[i * TW + jj] = make_float2(dR[j][r], CPLX ? dI[j][r] : 0.f);
      }
    }
    return;
  }
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr * (TW / 2) + x * 16 + 4 * lk + r;
        const int j = wc * 32 + y * 16 + li;
        o[i * TW + j] = make_float2(accR[x][y][r], CPLX ? accI[x][y][r] : 0.f);
      }
}

// ------------------------------------------------------------------ reduction
// chi0[p][P][Q] (lower triangle and mirror, FP64) = sum over the splits, in order, of
// the FP32 tiles; the diagonal from `diag`.  A workgroup covers a 32 x 32 block of one
// tile (tw x tw); the mirrored block goes through LDS so both writes are row-contiguous.
__global__ __launch_bounds__(256) void herk_reduce_kernel(const float2 *part, int nsplit, int ntiles, int tw, int N,
                                                          const double *diag, double2 *out, int64_t out_stride,
                                                          const PointDesc *pts, const double *lscale,
                                                          const double *rscale) {
  __shared__ double2 tb[32][33];
  const int tile = blockIdx.x, blk = blockIdx.y, p = blockIdx.z;
  int tr, tc;
  tile_of(tile, tr, tc);
  const int nb = tw / 32;
  const int bi = blk / nb, bj = blk % nb;   // 32 x 32 block of the tile
  const bool dtile = tr == tc;
  if (dtile && bj > bi) return;           // strictly upper blocks of a diagonal tile
  const int tid = threadIdx.x;
  const int j = tid & 31;
  const int64_t tsz = (int64_t)tw * tw;
  const int64_t tstride = (int64_t)ntiles * tsz;
  const float2 *src = part + ((int64_t)p * nsplit * ntiles + tile) * tsz;
  double2 *dst = out + (int64_t)p * out_stride;
  const double *dg = diag + (int64_t)p * N;
  // undo the operands' power-of-two scales (1 for bf16 operands): exact
  const double inv = lscale ? 1.0 / (lscale[pts[p].bslot] * rscale[p]) : 1.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = (tid >> 5) + 8 * k;
    const int li = bi * 32 + i, lj = bj * 32 + j;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < nsplit; ++s) {
      const float2 v = src[s * tstride + li * tw + lj];
      re += (double)v.x;
      im += (double)v.y;
    }
    re *= inv;
    im *= inv;
    tb[i][j] = make_double2(re, im);
    const int P = tr * tw + li, Q = tc * tw + lj;
    if (P < N && Q < N && (!dtile || P >= Q))
      dst[(int64_t)P * N + Q] = (P == Q) ? make_double2(dg[P], 0.0) : make_double2(re, im);
  }
  __syncthreads();
  // mirror: conj(chi0[P][Q]) into chi0[Q][P] for P > Q
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = (tid >> 5) + 8 * k;   // row of the mirrored block = column of the source
    const int Q = tc * tw + bj * 32 + i, P = tr * tw + bi * 32 + j;
    if (P < N && Q < N && P > Q) {
      const double2 v = tb[j][i];
      dst[(int64_t)Q * N + P] = make_double2(v.x, -v.y);
    }
  }
}

// ------------------------------------------------------------------ fp16 scales
// part[seg][blk] = max |x| over block blk of segment seg (segments of seg_len doubles,
// seg_stride apart); the maximum is exact, so the result does not depend on the order.
constexpr int AMAX_BLOCKS = 256;
__global__ __launch_bounds__(256) void absmax_partial_kernel(const double *x, int64_t seg_len, int64_t seg_stride,
                                                             double *part) {
  __shared__ double red[256];
  const int seg = blockIdx.y;
  const double *xs = x + (int64_t)seg * seg_stride;
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < seg_len; i += (int64_t)gridDim.x * 256)
    m = fmax(m, fabs(xs[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)seg * gridDim.x + blockIdx.x] = red[0];
}

// out[i] = the fp16 scale of bmax[slot_i] * (wmax ? wmax[i] : 1), slot_i = pts[i].bslot
// (or i without pts); bmax and wmax come from absmax_partial_kernel's blocks (nblk per
// segment) and are reduced here.
__global__ __launch_bounds__(64) void f16_scale_kernel(const double *bpart, const double *wpart, int nblk,
                                                       const PointDesc *pts, int n, double *out) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  const int slot = pts ? pts[i].bslot : i;
  double mb = 0.0, mw = 1.0;
  for (int b = 0; b < nblk; ++b) mb = fmax(mb, bpart[(int64_t)slot * nblk + b]);
  if (wpart) {
    mw = 0.0;
    for (int b = 0; b < nblk; ++b) mw = fmax(mw, wpart[(int64_t)i * nblk + b]);
  }
  out[i] = f16_scale_of(mb * mw);
}

}  // namespace

int64_t f16_absmax_scratch_doubles(int nseg) { return (int64_t)nseg * AMAX_BLOCKS; }

hipError_t launch_absmax_blocks(hipStream_t s, const double *x, int64_t seg_len, int64_t seg_stride, int nseg,
                                double *part) {
  if (nseg <= 0) return hipSuccess;
  if (nseg > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(absmax_partial_kernel, dim3(AMAX_BLOCKS, (unsigned)nseg), dim3(256), 0, s, x, seg_len, seg_stride,
                     part);
  return hipGetLastError();
}

hipError_t launch_f16_scales(hipStream_t s, const double *bpart, const double *wpart, const PointDesc *pts, int n,
                             double *out) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(f16_scale_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, bpart, wpart, AMAX_BLOCKS, pts,
                     n, out);
  return hipGetLastError();
}

int64_t bf16_prepared_elems(int64_t M, int N) {
  const int64_t Mp = (M + HK - 1) / HK * HK;
  const int64_t Np = (N + HT - 1) / HT * HT;
  return Mp * Np * 4;
}

void bf16_plan(int64_t M, int N, int npts, int64_t slots, int64_t max_part, int tn, Bf16Plan *pl) {
  pl->tn = tn == 64 ? 64 : HT;
  pl->Np = (N + HT - 1) / HT * HT;
  pl->nkc = (M + HK - 1) / HK;
  const int T = (N + pl->tn - 1) / pl->tn;
  pl->ntiles = T * (T + 1) / 2;
  const int64_t tsz = (int64_t)pl->tn * pl->tn;
  // fewest splits that keep every FP32 sum within BF16_SPLIT_ROWS rows, then more (down
  // to 512 rows a split) while the launch has fewer than two workgroups per slot and the
  // partial tiles stay within max_part elements (0: no limit)
  const int64_t wg_per_slot = pl->tn == 64 ? 4 : 2;   // 64-wide tiles: two workgroups per CU
  int64_t per = BF16_SPLIT_ROWS / HK;
  int64_t ns = (pl->nkc + per - 1) / per;
  while ((int64_t)pl->ntiles * npts * ns < wg_per_slot * slots && per > 512 / HK) {
    const int64_t per2 = per / 2, ns2 = (pl->nkc + per2 - 1) / per2;
    if (max_part > 0 && (int64_t)npts * ns2 * pl->ntiles * tsz > max_part) break;
    per = per2;
    ns = ns2;
  }
  pl->kc_per_split = (int)per;
  pl->nsplit = (int)ns;
}

int64_t bf16_partial_elems(const Bf16Plan &pl, int npts) {
  return (int64_t)npts * pl.nsplit * pl.ntiles * pl.tn * pl.tn;
}

int64_t bf16_diag_scratch_doubles(int64_t M, int N) {
  const int64_t nkc = (M + HK - 1) / HK;
  return (nkc + PREP_STEPS - 1) / PREP_STEPS * PREP_MAXP * (int64_t)N;
}

hipError_t launch_bf16_prepare(hipStream_t s, const void *B, bool cplx, int64_t M, int N, const double *wtab,
                               int npts, unsigned short *out, double *dscratch, double *diag, const double *scale,
                               bool f16) {
  const int64_t nkc = (M + HK - 1) / HK;
  const int Np = (N + HT - 1) / HT * HT;
  const int64_t stride = bf16_prepared_elems(M, N);
  if (nkc <= 0) return hipSuccess;
  const int64_t nchunks = (nkc + PREP_STEPS - 1) / PREP_STEPS;
  const bool want_diag = wtab && dscratch && diag;
  const int reps = wtab ? npts : 1;
  for (int p0 = 0; p0 < reps; p0 += PREP_MAXP) {
    const int np = reps - p0 < PREP_MAXP ? reps - p0 : PREP_MAXP;
    const double *w = wtab ? wtab + (int64_t)p0 * M : nullptr;
    const dim3 grid((unsigned)nchunks, (unsigned)(Np / PREP_COLS));
    double *dp = want_diag ? dscratch : nullptr;
    // right operands (w set) with non-temporal stores, the left operand through the caches
    const double *sc = scale ? scale + p0 : nullptr;
#define RPA_PREP_LAUNCH(C, NT, F)                                                                       \
  hipLaunchKernelGGL((bf16_prepare_kernel<C, NT, F>), grid, dim3(256), 0, s, B, M, N, Np, w, M, np, \
                     out + (int64_t)p0 * stride, stride, dp, sc)
    if (f16) {
      if (cplx) {
        if (w) RPA_PREP_LAUNCH(true, true, true); else RPA_PREP_LAUNCH(true, false, true);
      } else {
        if (w) RPA_PREP_LAUNCH(false, true, true); else RPA_PREP_LAUNCH(false, false, true);
      }
    } else {
      if (cplx) {
        if (w) RPA_PREP_LAUNCH(true, true, false); else RPA_PREP_LAUNCH(true, false, false);
      } else {
        if (w) RPA_PREP_LAUNCH(false, true, false); else RPA_PREP_LAUNCH(false, false, false);
      }
    }
#undef RPA_PREP_LAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (want_diag) {
      const int64_t tot = (int64_t)np * N;
      hipLaunchKernelGGL(prepare_diag_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, dscratch,
                         nchunks, np, N, diag + (int64_t)p0 * N);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_bf16_herk_groups(hipStream_t s, const Bf16Group *groups, int ngroups, bool cplx) {
  if (ngroups <= 0) return hipSuccess;
  if (ngroups > BF16_MAX_GROUPS) return hipErrorInvalidValue;
  const int tn = groups[0].pl.tn;
  const bool f16 = groups[0].f16;
  for (int i = 1; i < ngroups; ++i)   // one tile size and one 16-bit format per launch
    if (groups[i].pl.tn != tn || groups[i].f16 != f16) return hipErrorInvalidValue;
  HerkLaunch hl{};
  int64_t total = 0;
  int n = 0;
  for (int i = 0; i < ngroups; ++i) {
    const Bf16Group &g = groups[i];
    if (g.npts <= 0) continue;
    HerkArgs &h = hl.g[n];
    h.L = g.L;
    h.l_stride = g.l_stride;
    h.R = g.R;
    h.r_stride = g.r_stride;
    h.pts = g.pts;
    h.part = g.part;
    h.Np = g.pl.Np;
    h.ntiles = g.pl.ntiles;
    h.nsplit = g.pl.nsplit;
    h.kc_per_split = g.pl.kc_per_split;
    h.nkc = g.pl.nkc;
    hl.begin[n] = (int32_t)total;
    total += (int64_t)g.pl.ntiles * g.pl.nsplit * g.npts;
    if (total > 0x7fffffff) return hipErrorInvalidValue;
    ++n;
  }
  if (n == 0) return hipSuccess;
  hl.ngroups = n;
  for (int i = n; i <= BF16_MAX_GROUPS; ++i) hl.begin[i] = (int32_t)total;
  const dim3 grid((unsigned)total);
#define RPA_HERK_LAUNCH(C, T, F) hipLaunchKernelGGL((herk_bf16x3_kernel<C, T, F>), grid, dim3(4 * T), 0, s, hl)
  if (f16) {
    if (tn == 64) {
      if (cplx) RPA_HERK_LAUNCH(true, 64, true); else RPA_HERK_LAUNCH(false, 64, true);
    } else {
      if (cplx) RPA_HERK_LAUNCH(true, 128, true); else RPA_HERK_LAUNCH(false, 128, true);
    }
  } else {
    if (tn == 64) {
      if (cplx) RPA_HERK_LAUNCH(true, 64, false); else RPA_HERK_LAUNCH(false, 64, false);
    } else {
      if (cplx) RPA_HERK_LAUNCH(true, 128, false); else RPA_HERK_LAUNCH(false, 128, false);
    }
  }
#undef RPA_HERK_LAUNCH
  return hipGetLastError();
}

hipError_t launch_bf16_reduce(hipStream_t s, const Bf16Plan &pl, const float2 *part, int npts, int N,
                              const double *diag, double2 *out, int64_t out_stride, const PointDesc *pts,
                              const double *lscale, const double *rscale) {
  if (npts <= 0) return hipSuccess;
  if (lscale && (!pts || !rscale)) return hipErrorInvalidValue;
  const int nb = pl.tn / 32;
  hipLaunchKernelGGL(herk_reduce_kernel, dim3((unsigned)pl.ntiles, (unsigned)(nb * nb), (unsigned)npts), dim3(256), 0,
                     s, part, pl.nsplit, pl.ntiles, pl.tn, N, diag, out, out_stride, pts, lscale, rscale);
  return hipGetLastError();
}

}  // namespace rpa
