// Internal declarations shared by the HIP kernels and the host runtime of librpa.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpa {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// One (q, omega) point of a chi0 launch.
struct PointDesc {
  int32_t q;        // q index (selects the kq row and the Delta pairing)
  int32_t bslot;    // which B(q) slab of the launch holds this q's coefficients
  double omega;
};

// Arguments of the chi0 contraction kernels.
constexpr int kMaxSplit = 16;    // row splits of one FP64/FP32 contraction launch
constexpr int kBatchSplits = 4;  // at most this many in the batched point pipeline (its
                                 // partial planes hold a whole batch of points each)

struct Chi0Args {
  const void *B;            // bslot-major slabs of [M][N] coefficients (complex or real)
  int64_t b_slot_stride;    // elements (complex or real) between slabs
  const double *eps_occ;    // [nk][nocc]
  const double *eps_virt;   // [nk][nvirt]
  const int32_t *kq;        // [nq][nk]
  const double *zeta_k;     // [nk]
  const PointDesc *pts;     // [npts]
  double *wtab;             // [npts][M] w_m zeta_k of every contraction row
  double2 *out;             // [npts][N][N] complex
  int64_t out_stride;       // complex elements between outputs
  int32_t ksplit;           // row splits (FP64 and FP32: 1..kMaxSplit): the
                            // first writes out, split z >= 1 plane z - 1 of partial, and
                            // out += the planes in split order follows
  double2 *partial;         // [ksplit - 1][npts][N][N] (used when ksplit >= 2)
  int64_t split_stride;     // complex elements between partial planes (set by the launcher)
  int32_t nk, nocc, nvirt, N;
  int64_t M;                // nk * nocc * nvirt
  const int32_t *pairs;     // [npairs][2] points of one slab contracted together (second
                            // index -1: none), for the paired FP64 kernel; may be null
  int32_t npairs;
  int32_t k0;               // k-point of row 0: the rows are those of k-points k0 .. k0 +
                            // M / (nocc * nvirt) - 1 (a chunk of a streamed q; else 0)
};

// Batched complex GEMM C_b = A_{a(b)} * B_{b(b)}, all N x N row-major.
struct GemmArgs {
  const double2 *A; int64_t a_stride; int32_t a_div;   // A index = b / a_div
  const double2 *B; int64_t b_stride; int32_t b_div;   // B index = b / b_div
  double2 *C; int64_t c_stride;
  const int32_t *a_map;   // optional: A index = a_map[b]   (overrides a_div)
  const int32_t *b_map;   // optional: B index = b_map[b]
  int32_t N;
  int32_t lower_only;     // compute only the tiles on or below the diagonal
  int32_t negate;         // store -C instead of C
};

// ---- launchers (each returns the launch's hipError_t) -----------------------

hipError_t launch_philox_B(hipStream_t s, uint64_t seed, double sigma, int32_t nk, int32_t iq,
                           int32_t k0, int32_t k1, int32_t nocc, int32_t nvirt, int32_t naux,
                           bool cplx, void *out);
// Pair-fit coefficients C^{mu nu}_gamma(k,q) of block (q, k) of an atomic-orbital system,
// complex [nbas][nbas][naux]: Philox stream 1 of the key of B's block (q, k), element
// e = (mu * nbas + nu) * naux + gamma.
hipError_t launch_philox_C(hipStream_t s, uint64_t seed, double sigma, int32_t nk, int32_t iq, int32_t ik,
                           int32_t nbas, int32_t naux, void *out);
// B^gamma_ia(k,q) = conj(sum_{mu nu} conj(cv_{mu a}) C^{mu nu}_gamma co_{nu i}) of one (q, k)
// block into out ([nocc][nvirt][naux]): the conjugate of the pair coefficient C^{ai}_gamma: C from launch_philox_C into `scratch`
// (ao_scratch_bytes), then two batched complex FP64 MFMA products.  c_occ points at the
// projected occupied coefficients of k (+) q ([nbas][nocc]), c_virt at the virtual ones of
// k ([nbas][nvirt]).
int64_t ao_scratch_bytes(int32_t nbas, int32_t nocc, int32_t naux);
hipError_t launch_ao_B(hipStream_t s, uint64_t seed, double sigma, int32_t nk, int32_t iq, int32_t ik, int32_t nbas,
                       int32_t nocc, int32_t nvirt, int32_t naux, const double2 *c_occ, const double2 *c_virt,
                       void *scratch, double2 *out);
// The periodic projector of Sec. 2.3 (projector.hip): T(k) = U(k) R~ U(k)^H from the
// overlaps S [nk][nbas][nbas] (complex, Hermitian; device memory), R~ keeping the
// eigen-directions whose ascending-order eigenvalue is >= eps_d at every k; T written to
// T [nk][nbas][nbas].  scratch holds projector_scratch_bytes(nk, nbas) bytes.  nbas <= 1024.
int64_t projector_scratch_bytes(int32_t nk, int32_t nbas);
hipError_t launch_projector(hipStream_t s, const double2 *S, int32_t nk, int32_t nbas, double eps_d, void *scratch,
                            double2 *T);
// out[k] = T[k] c[k] for c [nk][nbas][nb] (complex), out of place.
hipError_t launch_project_coeff(hipStream_t s, const double2 *T, const double2 *c, int32_t nk, int32_t nbas,
                                int32_t nb, double2 *out);
hipError_t launch_philox_words(hipStream_t s, uint64_t seed, int32_t nk, int32_t iq, int32_t ik,
                               uint64_t e0, int64_t count, uint32_t *out);

// Fill a.wtab for the npts points of a launch (must precede the contraction launch).
hipError_t launch_chi0_weights(hipStream_t s, const Chi0Args &a, int32_t npts);
// cfg selects the tile and K step: 0, 1, 2 = 64-wide tiles with 8, 16, 32-row steps,
// 3 = 128-wide tiles with 16-row steps, 4 = 64-wide tiles with 16-row steps contracting
// the two points of each a.pairs entry per workgroup (without a pair table: cfg 1); all
// give the same sums in the same row order.  With a.ksplit = s > 1 (at most kMaxSplit)
// splits 1..s-1 write planes of a.partial (npts points apart) and the launch then adds
// them into a.out in split order (repeatable).
hipError_t launch_chi0_f64(hipStream_t s, const Chi0Args &a, int32_t npts, bool cplx_b, int cfg);
// Paired FP64 contraction (configuration 4) of several groups of points (each with its
// own Chi0Args and point count, all with pair tables) in one launch: every group's
// results are exactly those of launching it alone, its row splits added in split order.
constexpr int CHI0_MAX_GROUPS = 8;
struct Chi0Group {
  Chi0Args a;
  int32_t npts;
};
hipError_t launch_chi0_f64_paired_groups(hipStream_t s, const Chi0Group *groups, int ngroups, bool cplx_b);
// Workgroups of one group's paired launch (FP64 or FP32: both use 64-wide tiles).
int64_t chi0_paired_workgroups(const Chi0Args &a);
// The same for the paired FP32 contraction (configuration kF32T64W2), each group with its
// own FP32 copy of B and exact FP64 diagonal.
struct Chi0F32Group {
  Chi0Args a;
  int32_t npts;
  const float2 *B32;
  const double *diag;
};
hipError_t launch_chi0_f32_paired_groups(hipStream_t s, const Chi0F32Group *groups, int ngroups);
int chi0_cfg_count();
int chi0_cfg_tile(int cfg);            // output tile edge of a configuration
int chi0_cfg_slots_per_cu(int cfg);    // workgroups of it that fit on one CU
int chi0_cfg_points_per_wg(int cfg);   // points one workgroup contracts (2: paired kernel)
const char *chi0_cfg_name(int cfg);
// Number of row splits (1..max_split) that best fills `slots` concurrent workgroups for
// `work` workgroups of one split.
int32_t chi0_pick_ksplit(int64_t work, int64_t slots, int64_t M, int32_t max_split);
// out += partial[0] + ... + partial[nparts - 1] (planes of n complex elements), in that order
hipError_t launch_split_add(hipStream_t s, const double2 *partial, int32_t nparts, int64_t n, double2 *out);

hipError_t launch_zgemm_f64(hipStream_t s, const GemmArgs &a, int32_t batch);

// eps_b = ln det(1 - Pi_b) + Re Tr Pi_b; Pi is overwritten by its factor.  info[b] = -1 on
// success, else the failing column.  Results of batch entry b go to index out_map[b]
// (or b if out_map is NULL).
hipError_t launch_trln_f64(hipStream_t s, double2 *pi, int64_t stride, int32_t n, int32_t batch,
                           double *eps, int32_t *info, const int32_t *out_map);

// ---- reduced-precision chi0 -----------------------------------------------------
// FP64 (complex or real) [n] -> complex FP32 [n].
hipError_t launch_to_f32(hipStream_t s, const void *in, float2 *out, int64_t n, bool cplx);
// Exact FP64 diagonal diag[p][P] = sum_m wtab[p][m] |B_mP|^2 for npts points sharing one
// FP64 B slab; `scratch` holds diag_exact_scratch_doubles(M, N, npts) doubles.
int64_t diag_exact_scratch_doubles(int64_t M, int N, int npts);
hipError_t launch_diag_exact(hipStream_t s, const void *B, bool cplx, int64_t M, int N, const double *wtab,
                             int npts, double *scratch, double *diag);
// chi0 with FP32 MFMA (prec 1) from the FP32 copy B32 (slab stride a.b_slot_stride), FP64
// flush of partial sums and the exact diagonal `diag` [npts][N], in one of three
// configurations (tile): 64- or 128-wide tiles, or 64-wide tiles contracting the two points
// of each entry of a.pairs per workgroup (without a pair table: the 64-wide kernel); all
// sum the same products in the same order.  a.ksplit: 1..kMaxSplit row splits.
constexpr int kF32T64 = 64, kF32T128 = 128, kF32T64W2 = 65;
int f32_cfg_edge(int cfg);             // output tile edge
int f32_cfg_points_per_wg(int cfg);    // 2 for the paired kernel
const char *f32_cfg_name(int cfg);     // t64, t128, t64w2
hipError_t launch_chi0_mixed(hipStream_t s, const Chi0Args &a, int32_t npts, const float2 *B32,
                             const double *diag, int prec, int tile = kF32T64);

// ---- split-BF16 chi0 from prepared operands (chi0_bf16.hip) ------------------------
// No FP32 sum of the contraction runs over more rows than this.
constexpr int64_t BF16_SPLIT_ROWS = 4096;
struct Bf16Plan {
  int32_t tn;            // output tile edge: 64 or 128
  int32_t Np;            // N rounded up to 128 (the prepared layout's padding)
  int32_t ntiles;        // tiles on and below the diagonal
  int32_t nsplit;        // row splits
  int32_t kc_per_split;  // 32-row steps per split
  int64_t nkc;           // 32-row steps of the whole contraction
};
// bf16 elements of one prepared operand (four planes, rows and columns padded).
int64_t bf16_prepared_elems(int64_t M, int N);
// Tiles (edge tn = 64 or 128) and row splits of a launch of npts points on a device with
// `slots` CUs, with at most max_part partial-tile elements when max_part > 0 (never
// fewer splits than needed to bound the FP32 sums).
void bf16_plan(int64_t M, int N, int npts, int64_t slots, int64_t max_part, int tn, Bf16Plan *pl);
// float2 elements of the partial-tile buffer of such a launch.
int64_t bf16_partial_elems(const Bf16Plan &pl, int npts);
// Prepared operands from an FP64 B slab: wtab == nullptr gives the unscaled left operand
// (one), else one right operand w_p B per point p < npts, at bf16_prepared_elems apart.
// With dscratch (bf16_diag_scratch_doubles) and diag set, also the exact FP64 diagonal
// diag[p][P] = sum_m wtab[p][m] |B_mP|^2 of those points.
// scale (null: 1) is the operand's power-of-two factor (one per point for right operands,
// read at scale[p]); f16 selects the fp16 split instead of bf16.
int64_t bf16_diag_scratch_doubles(int64_t M, int N);
hipError_t launch_bf16_prepare(hipStream_t s, const void *B, bool cplx, int64_t M, int N, const double *wtab,
                               int npts, unsigned short *out, double *dscratch = nullptr, double *diag = nullptr,
                               const double *scale = nullptr, bool f16 = false);
// fp16 operand scales.  launch_absmax_blocks writes, for each of nseg segments of seg_len
// doubles (seg_stride apart), the maxima of |x| over its blocks into part (nseg *
// f16_absmax_scratch_doubles(1) doubles).  launch_f16_scales then sets out[i] to the
// power of two that brings max(B slab of pts[i].bslot) * max|w_i| (wpart null: the slab
// alone, slab i without pts) just below 2^14.
int64_t f16_absmax_scratch_doubles(int nseg);
hipError_t launch_absmax_blocks(hipStream_t s, const double *x, int64_t seg_len, int64_t seg_stride, int nseg,
                                double *part);
hipError_t launch_f16_scales(hipStream_t s, const double *bpart, const double *wpart, const PointDesc *pts, int n,
                             double *out);
// One contraction launch's worth of work (a sub-batch of one job).
constexpr int BF16_MAX_GROUPS = 16;
struct Bf16Group {
  const unsigned short *L;
  int64_t l_stride;
  const unsigned short *R;
  int64_t r_stride;          // bf16_prepared_elems of the group's shape
  const PointDesc *pts;
  float2 *part;
  Bf16Plan pl;
  int32_t npts;
  bool f16 = false;          // fp16 operands (else bf16); one format per launch
};
// FP32 partial tiles of the row splits of every group's points (left operand of point p
// at L + pts[p].bslot * l_stride, right operand p at R + p * r_stride) into its part
// buffer (bf16_partial_elems(pl, npts) float2).  Up to BF16_MAX_GROUPS groups of any
// shapes (all complex or all real, all of one tile edge) in one launch; every group's
// results are exactly those of launching it alone.
hipError_t launch_bf16_herk_groups(hipStream_t s, const Bf16Group *groups, int ngroups, bool cplx);
// chi0 of those points into out (FP64 complex, Hermitian, point p at p * out_stride): the
// splits summed in FP64 in order, divided by lscale[pts[p].bslot] * rscale[p] (fp16
// operands; lscale null: no scaling), the diagonal from diag[p][P].
hipError_t launch_bf16_reduce(hipStream_t s, const Bf16Plan &pl, const float2 *part, int npts, int N,
                              const double *diag, double2 *out, int64_t out_stride,
                              const PointDesc *pts = nullptr, const double *lscale = nullptr,
                              const double *rscale = nullptr);

// Blocked Cholesky log-det over the whole GPU on W = -Pi (see trln_blocked.hip):
// eps[out_map[b]] = ln det(1 - Pi_b) + Re Tr Pi_b, info_out[out_map[b]] = -1 or the failing
// column.  W is overwritten; scratch holds trln_blocked_scratch_bytes(batch) bytes.
int64_t trln_blocked_scratch_bytes(int32_t batch);
hipError_t launch_trln_blocked(hipStream_t s, double2 *w, int64_t stride, int32_t n, int32_t batch, double *eps,
                               int32_t *info_out, const int32_t *out_map, void *scratch);
// P <- -P elementwise for batch matrices of n x n.
hipError_t launch_negate(hipStream_t s, double2 *p, int64_t stride, int32_t n, int32_t batch);

// E = sum_q zeta_q sum_j W_j eps[q][j] / (2 pi) in a fixed order.
hipError_t launch_quadrature(hipStream_t s, const double *eps, const double *zeta_q,
                             const double *weight, int32_t nq, int32_t nw, double *E);

// Real [n] -> complex [n] with zero imaginary parts, and back (real part).
hipError_t launch_widen(hipStream_t s, const double *in, double2 *out, int64_t n);
hipError_t launch_narrow(hipStream_t s, const double2 *in, double *out, int64_t n);

// Fill `bytes` of device memory at p with 0xFF bytes (a NaN in FP64, FP32, FP16 and BF16),
// for the RPA_POISON debugging mode.
hipError_t launch_poison_fill(hipStream_t s, void *p, int64_t bytes);

}  // namespace rpa
