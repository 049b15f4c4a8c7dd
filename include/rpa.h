/*
 * rpa.h -- C-ABI of the MI355X periodic RPA hot path (librpa.so, gfx950).
 *
 * The library evaluates the RPA correlation energy per unit cell of a periodic
 * insulator in a density-fitting (auxiliary) basis, following arXiv:2505.06021
 * (Spadetto, Philipsen, Foerster, Visscher):
 *
 *   chi0_PQ(q, i w) = sum_k zeta_k sum_ia conj(B^P_ia(k,q)) w_ia(w) B^Q_ia(k,q)
 *       with w_ia(w) = -4 Delta / (Delta^2 + w^2), Delta = eps_a(k) - eps_i(k (+) q)
 *       (Sec. 2.2, the fit-basis polarizability equation; the -2 is the closed-shell
 *        occupation factor and the complex-conjugate term doubles the real part).
 *       B is the complex conjugate of the paper's pair coefficient: B^P_ia(k,q) =
 *       conj(C^{ai}_P(k+q,k)), C^{ai}_P being the coefficient of f_P in the expansion of
 *       psi*_a(k) psi_i(k+q), so that conj(B^P) B^Q = C^{ai}_P conj(C^{ai}_Q) keeps the
 *       index order of that equation.
 *   Pi  = V^(1/2) chi0 V^(1/2)                 (working equation; Algorithm 1)
 *   eps(q, w) = ln det(1 - Pi) + Re Tr Pi      (Eq. 1 summed as -ln(1 - Z) - Z)
 *   E   = sum_q zeta_q sum_j W_j eps(q, w_j) / (2 pi)
 *                                               (Eq. 1 with the main-loop quadrature)
 *
 * Conventions for every entry point:
 *  - Return value: RPA_OK (0) on success, RPA_PENDING (1) from rpa_poll while a job runs,
 *    a negative rpa_status otherwise.  Nothing aborts or throws across the ABI;
 *    rpa_last_error() gives a message for the calling thread's last failure.
 *  - Complex arrays are interleaved (re, im) binary64 pairs, row-major.
 *    Real systems (is_complex = 0) use plain binary64 arrays of the same shape.
 *  - memspace says where the caller's array pointers live: RPA_MEM_HOST (pageable or
 *    pinned host memory) or RPA_MEM_DEVICE (device memory of the context's GPU).
 *    Device-side work runs on the context's stream (rpa_set_stream); synchronous
 *    entry points return after that stream has finished the call's work.
 *  - Inputs are borrowed for the duration of a synchronous call; the library keeps
 *    no pointer to them afterwards.  Outputs are written to caller buffers.
 *  - A context is safe to use from several threads; calls are serialised inside.
 */
#ifndef RPA_H
#define RPA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum rpa_status {
  RPA_OK = 0,
  RPA_PENDING = 1,
  RPA_E_ARG = -1,          /* invalid argument, shape or null pointer                  */
  RPA_E_NOMEM = -2,        /* request exceeds the context's HBM limit                  */
  RPA_E_DEVICE = -3,       /* HIP runtime or launch error                              */
  RPA_E_NOTSPD = -4,       /* 1 - Pi is not Hermitian positive definite (Cholesky fails) */
  RPA_E_UNKNOWN_JOB = -5,  /* job id never issued or already consumed                  */
  RPA_E_INTERNAL = -6,
  RPA_E_CANCELLED = -7     /* job cancelled by rpa_finalize                            */
};

/* Arithmetic of the chi0 contraction; Pi, the Cholesky/log-det and the sums are FP64.
 * Energy error per cell against FP64, as tested: FP32 and split-FP16 within 1e-6 Ha on
 * every tested system; split-BF16 within about 1e-8 relative, which exceeds 1e-6 Ha on
 * some systems (its tested bound is 2e-5 Ha): it is the fastest, not the most exact. */
typedef enum {
  RPA_FP64 = 0,      /* FP64 MFMA                                                      */
  RPA_FP32 = 1,      /* FP32 MFMA, FP64 flush of partial sums, exact FP64 diagonal     */
  RPA_BF16X3 = 2,    /* split-BF16 (hi*hi + hi*lo + lo*hi) on MFMA, FP32 accumulate,
                        FP64 sum of the row splits, exact FP64 diagonal                */
  RPA_F16X3 = 3      /* split-FP16 (hi*hi + hi*lo + lo*hi) on MFMA with power-of-two
                        operand scaling, FP32 accumulate, FP64 sum of the row splits,
                        exact FP64 diagonal; as fast as split-BF16                     */
} rpa_precision;

typedef enum { RPA_MEM_HOST = 0, RPA_MEM_DEVICE = 1 } rpa_memspace;

typedef struct rpa_ctx rpa_ctx;

/*
 * One periodic system (the inputs of Algorithm 1: fit coefficients and band energies).
 * The contraction runs over the nk k-points of the regular grid for each of the nq
 * q-points; Delta_kia(q) = eps_a(k) - eps_i(k (+) q).
 *  kq        [nq][nk]  int32: row of eps_occ that holds k (+) q, in [0, nk_occ).
 *  eps_occ   [nk_occ][nocc]: occupied band energies (Hartree) at every point k (+) q can
 *            reach; eps_virt [nk][nvirt]: virtual band energies at the regular k.
 *  nk_occ    rows of eps_occ; 0 means nk (regular grids, Q_G = K_G).  The dual grids of
 *            Sec. 3.2 (Gamma removed from the q-grid, 2/4/8 displaced q-points added around
 *            it) reach (N_add + 1) * nk points, so nk_occ = (N_add + 1) * nk there.
 *  nbas      0, or the size of an atomic-orbital basis: B is then built on the device by
 *            the MO transform of Sec. 2.2, C^{ai}_P(k+q,k) = sum_{mu nu} conj(c_virt[k][mu][a])
 *            C^{mu nu}_P(k,q) c_occ[k (+) q][nu][i] and B^P_ia(k,q) = conj(C^{ai}_P), with
 *            the pair-fit coefficients C^{mu nu}_P drawn from Philox stream 1 of B's key
 *            (philox_seed, sigma; element e = (mu * nbas + nu) * naux + P).  Requires
 *            is_complex = 1 and B = NULL.
 *  c_occ     [nk_occ][nbas][nocc], c_virt [nk][nbas][nvirt]: KS coefficients (complex):
 *            already projected (T(k) c of Sec. 2.3) when S_ao is NULL, else raw.
 *  S_ao      NULL, or [nk][nbas][nbas] (complex, Hermitian): the overlaps S(k) of the basis;
 *            the library then applies the periodic projector of Sec. 2.3 on the device,
 *            c~(k) = T(k) c(k) with T(k) = U(k) R~ U(k)^H from S(k) = U D U^H, keeping the
 *            eigen-directions whose eigenvalue (ascending order) is >= eps_d at every k.
 *            Regular grids only (nk_occ = nk), nbas <= 1024.
 *  eps_d     the projector's threshold (used when S_ao != NULL).
 *  zeta_k    [nk], zeta_q [nq]: integration weights; NULL means 1/nk and 1/nq.
 *  B         [nq][nk][nocc][nvirt][naux]: fit coefficients B^P_ia(k,q), P fastest: the
 *            complex conjugates of the MO-basis PADF coefficients C^{ai}_P(k+q,k) of
 *            Sec. 2.2 (a caller holding C passes conj(C); for real systems B = C).  NULL
 *            means: generate them on the device from Philox4x32-10 with philox_seed and
 *            sigma (the stream definition is that of rpa_philox_B).
 *  vhalf     [nq][naux][naux]: V^(1/2)(q), Hermitian (symmetric if real).
 * All arrays live in `memspace`.
 */
typedef struct {
  int32_t nk, nq, nocc, nvirt, naux, is_complex;
  int32_t memspace;
  const int32_t *kq;
  const double *eps_occ;
  const double *eps_virt;
  const double *zeta_k;
  const double *zeta_q;
  const void *B;
  uint64_t philox_seed;
  double sigma;
  const void *vhalf;
  int32_t nk_occ;
  int32_t nbas;
  const void *c_occ;
  const void *c_virt;
  const void *S_ao;
  double eps_d;
} rpa_system;

/* Imaginary-frequency quadrature (host memory): nodes omega_j and weights W_j that
 * already include d omega / dx of the node map.  The 1/(2 pi) of Eq. 1 is applied
 * by the library. */
typedef struct {
  int32_t nw;
  const double *omega;
  const double *weight;
} rpa_freq;

/* Final record of a submitted job (times in seconds on the library's monotonic clock). */
typedef struct {
  double E;
  int32_t status;
  int32_t npoints;
  double t_submit, t_start, t_done;
  int64_t hbm_bytes;     /* device bytes the job held while running */
} rpa_result;

typedef struct {
  int64_t hbm_limit, hbm_in_use, hbm_high_water;
  int64_t jobs_submitted, jobs_done, jobs_running, jobs_queued;
  /* contractions of served jobs (split 16-bit, paired FP64, paired FP32): fused launches,
   * the job sub-batches they carried, and sub-batches launched alone (large enough to fill
   * the GPU, or of a configuration that is not fused) */
  int64_t fused_launches, fused_groups, solo_groups;
} rpa_stats;

/* Create a context on HIP device `device`.  hbm_limit_bytes caps the device memory the
 * context may hold (0 = 90% of the device memory free at creation).  Debugging modes,
 * read from the environment here, once per context: RPA_POISON=1 fills every new device
 * allocation with 0xFF bytes (NaN in every floating-point format used) before use, so a
 * kernel that reads workspace it has not written shows up as a changed or NaN result;
 * RPA_FAULT=alloc:N[,N2,...] makes the N-th (1-based) device allocation of the context,
 * and each further listed one, fail with RPA_E_NOMEM ("injected" in the message), for
 * tests of the error paths.  Errors: RPA_E_ARG (ctx NULL, bad device, malformed
 * RPA_FAULT), RPA_E_DEVICE. */
int rpa_init(rpa_ctx **ctx, int device, uint64_t hbm_limit_bytes);

/* Cancel queued jobs, wait for running ones, free all device memory, destroy ctx. */
int rpa_finalize(rpa_ctx *ctx);

/* Message of the calling thread's last error ("" if none).  ctx may be NULL. */
const char *rpa_last_error(const rpa_ctx *ctx);

/* Use `hip_stream` (a hipStream_t, NULL = the context's own stream) for the context's
 * synchronous device work, e.g. torch.cuda.current_stream().cuda_stream. */
int rpa_set_stream(rpa_ctx *ctx, void *hip_stream);

/* chi0(q = iq, i omega) of Sec. 2.2 into chi0 [naux][naux] (complex, or real if
 * is_complex = 0), in sys->memspace.  The full Hermitian matrix is written.  The FP64
 * and FP32 contractions split the rows of this one point up to 16 ways so that the
 * launch fills the GPU; the context's workspace then holds up to 15 partial planes of
 * naux x naux complex doubles (summed in split order, so a call is repeatable).
 * Errors: RPA_E_ARG, RPA_E_NOMEM, RPA_E_DEVICE. */
int rpa_chi0(rpa_ctx *ctx, const rpa_system *sys, int32_t iq, double omega,
             rpa_precision prec, void *chi0);

/* rpa_chi0 for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same FP64 chi0 of one
 * (q, omega) point, written in full into chi0 [naux][naux] (complex, device memory), with
 * no device allocation.  Its scratch (the small system arrays, one weight per contraction
 * row and the partial planes of the row splits) is a fixed 64 MiB device array per GPU,
 * held until the process ends; the row split count is capped to the planes that fit
 * beside the weights.  The system must be complex with B given (nbas = 0), and every array
 * in device memory; prec must be RPA_FP64.  The tile configuration is the one the tuner
 * already chose for this shape in the process (by rpa_chi0), else the fixed or default
 * one; nothing is timed.  Calls through one context are serialised; calls through two
 * contexts on the same GPU at the same time race on the shared scratch.  Results equal
 * rpa_chi0's to rounding (bit for bit at the same configuration and split count).
 * Errors: RPA_E_ARG (precision, memspace, real or atomic-orbital system, B NULL, bad
 * sizes), RPA_E_NOMEM if the band energies and nk*nocc*nvirt row weights do not fit in
 * the 64 MiB, RPA_E_DEVICE. */
int rpa_chi0_noalloc(rpa_ctx *ctx, const rpa_system *sys, int32_t iq, double omega,
                     rpa_precision prec, void *chi0);

/* Pi = V^(1/2) chi0 V^(1/2) (Algorithm 1, the sandwich step) for one n x n pair, all
 * arrays [n][n] in `memspace`; Pi is written in full.  Errors: RPA_E_ARG, RPA_E_NOMEM,
 * RPA_E_DEVICE. */
int rpa_pi(rpa_ctx *ctx, int32_t n, int32_t is_complex, int32_t memspace,
           const void *vhalf, const void *chi0, void *pi);

/* eps_b = ln det(1 - Pi_b) + Re Tr Pi_b for `batch` matrices Pi [batch][n][n] (only the
 * lower triangle is read), through a Cholesky factor of 1 - Pi (the log-det step of
 * Algorithm 1 with the sign of Eq. 1).  out [batch] doubles; all in `memspace`.
 * Errors: RPA_E_NOTSPD if some 1 - Pi_b is not positive definite (the message names b
 * and the failing column), RPA_E_ARG, RPA_E_NOMEM, RPA_E_DEVICE. */
int rpa_trln(rpa_ctx *ctx, int32_t n, int32_t batch, int32_t is_complex, int32_t memspace,
             const void *pi, double *out);

/* RPA correlation energy per cell: E (host double) and, if eps_qw != NULL, the integrand
 * eps(q, omega_j) [nq][nw] (host memory).  All steps run on the GPU; the q/omega sum is
 * taken on the device in a fixed order (q outer, omega inner).  Environment: RPA_LANES=2
 * splits the points into two batches on two streams, so one batch's sandwich and
 * Cholesky overlap the other's contraction (a few percent faster; the two batches'
 * contractions then also run side by side); RPA_TRLN_SINGLE=1 takes the
 * one-workgroup-per-matrix Cholesky instead of the blocked one.
 * Errors: RPA_E_ARG, RPA_E_NOMEM, RPA_E_NOTSPD, RPA_E_DEVICE. */
int rpa_energy(rpa_ctx *ctx, const rpa_system *sys, const rpa_freq *freq,
               rpa_precision prec, double *E, double *eps_qw);

/* Same as rpa_energy for a subset of points only: eps[p] = eps(q = iq[p], omega = w[p]).
 * iq, w and eps are host arrays of npts entries.  Errors as rpa_energy. */
int rpa_points(rpa_ctx *ctx, const rpa_system *sys, int32_t npts, const int32_t *iq,
               const double *w, rpa_precision prec, double *eps);

/* The periodic projector of Sec. 2.3: T [nk][nbas][nbas] (complex) from the overlaps
 * S [nk][nbas][nbas] (complex, Hermitian) and the threshold eps_d, both arrays in
 * `memspace`: S(k) = U D U^H (Jacobi eigendecomposition on the device, FP64), the
 * eigen-directions sorted by ascending eigenvalue, an index kept only if its eigenvalue is
 * >= eps_d at every k, T(k) = U R~ U^H.  Errors: RPA_E_ARG (sizes, nbas > 1024),
 * RPA_E_NOMEM, RPA_E_DEVICE. */
int rpa_projector(rpa_ctx *ctx, int32_t nk, int32_t nbas, double eps_d, int32_t memspace, const void *S,
                  void *T);

/* Device Philox generator of the fit coefficients of block (q = iq, k = ik):
 * out [nocc][nvirt][naux] in `memspace`.  Stream: Philox4x32-10 (Salmon et al., SC'11)
 * with key (seed mod 2^32, (seed >> 32) + iq*nk + ik mod 2^32) and counter
 * (e mod 2^32, e >> 32, 0, 0), e = (i*nvirt + a)*naux + P; the words w0..w3 give
 * u = ((w_even >> 6) * 2^26 + (w_odd >> 6) + 1/2) * 2^-52 and Box-Muller in FP64:
 * B = sigma/sqrt(2) * sqrt(-2 ln u1) * (cos 2 pi u2 + i sin 2 pi u2), or
 * sigma * sqrt(-2 ln u1) * cos 2 pi u2 for real systems.  Errors: RPA_E_ARG, RPA_E_DEVICE. */
int rpa_philox_B(rpa_ctx *ctx, uint64_t seed, double sigma, int32_t nk, int32_t iq,
                 int32_t ik, int32_t nocc, int32_t nvirt, int32_t naux, int32_t is_complex,
                 int32_t memspace, void *out);

/* The raw 32-bit Philox words of elements e0 .. e0+count-1 of block (iq, ik):
 * out [count][4] uint32 in `memspace`. */
int rpa_philox_words(rpa_ctx *ctx, uint64_t seed, int32_t nk, int32_t iq, int32_t ik,
                     uint64_t e0, int64_t count, int32_t memspace, uint32_t *out);

/* Serving (continuous batching).  rpa_submit copies every input it needs (B must be
 * NULL, i.e. Philox-generated, or host memory) and returns at once with a job id.
 * A scheduler thread admits queued jobs while their projected device memory fits
 * under the HBM limit, and runs the (q, omega) points of all admitted jobs through
 * shared kernel launches.  A job that can never fit fails at submit with RPA_E_NOMEM.
 * rpa_poll waits up to timeout_ms (0 = do not wait, < 0 = forever) and returns
 * RPA_PENDING, or the job's final status with *out filled and, if eps_qw != NULL,
 * its [nq][nw] integrand; a finished job is consumed by the successful poll.
 * A queued job that does not fit yet is passed by later jobs that fit, until it has waited
 * RPA_SERVE_HOLD_MS (default 60000): then no job is admitted before it.
 * Environment: RPA_SERVE_WORKERS (concurrent jobs, 1..16, default 4), RPA_SERVE_HOLD_MS,
 * and RPA_FUSE_WINDOW_US (how long the fuser waits for other jobs' small contraction
 * launches, default 300).
 * Errors: RPA_E_ARG, RPA_E_NOMEM, RPA_E_UNKNOWN_JOB, or the job's own error. */
int rpa_submit(rpa_ctx *ctx, const rpa_system *sys, const rpa_freq *freq,
               rpa_precision prec, uint64_t *job_id);
int rpa_poll(rpa_ctx *ctx, uint64_t job_id, int32_t timeout_ms, rpa_result *out,
             double *eps_qw);

/* Counters of the context (device memory, jobs). */
int rpa_get_stats(rpa_ctx *ctx, rpa_stats *out);

/* Per-kernel device time of the synchronous entry points, measured with HIP events
 * recorded on the stream each kernel is launched on.  Index by rpa_kernel_kind. */
enum rpa_kernel_kind {
  RPA_K_PHILOX = 0,   /* B generation                                 */
  RPA_K_CHI0 = 1,     /* chi0 contraction (the MFMA kernel alone)     */
  RPA_K_PI = 2,       /* the two GEMMs of V^(1/2) chi0 V^(1/2)         */
  RPA_K_TRLN = 3,     /* Cholesky log-det                             */
  RPA_K_OTHER = 4,    /* quadrature, widening, copies                 */
  RPA_K_CHI0_AUX = 5, /* transition-weight table, FP32 copy of B and the exact FP64
                         diagonal of the reduced-precision paths       */
  RPA_K_COUNT = 8
};
typedef struct {
  int64_t launches[RPA_K_COUNT];
  double ms[RPA_K_COUNT];
} rpa_kernel_times;

/* enable != 0 turns event timing on and clears the totals; 0 turns it off. */
int rpa_profile(rpa_ctx *ctx, int32_t enable);
int rpa_profile_read(rpa_ctx *ctx, rpa_kernel_times *out);

/* Tile configurations of the chi0 contractions chosen so far in this process.
 * FP64 buckets ("f64_...") name the output tile edge and the rows of B staged per LDS
 * step (t64k8, t64k16, t64k32, t128k16, and t64k16w2: two frequencies of a q per
 * workgroup); FP32 buckets ("f32_...") name t64, t128 or t64w2 (the paired 64-wide
 * kernel), split-BF16 buckets ("bf16_...") the tile edge (t64, t128).  A choice changes
 * the speed of the contraction, never its sums at a given row split count (the chi0
 * equation of the periodic RPA section, summed in the same row order by every
 * configuration of a precision); each shape bucket is timed once on its first launch,
 * every candidate at the row split count the launch would give it.  Writes "bucket
 * configuration" lines, NUL-terminated and truncated to len bytes, into buf
 * (caller-owned; may be NULL when len is 0) and the untruncated length into *needed (may
 * be NULL).  Environment: RPA_CHI0_CFG=<name> (or RPA_CHI0_KT=8|16|32) fixes the FP64
 * configuration, RPA_F32_TILE=64|128|64w2 the FP32 one, RPA_BF16_TILE=64|128 the
 * split-BF16 tile edge, RPA_CHI0_KSPLIT=n the row split count of the FP64 and FP32
 * contractions (at most 16 in rpa_chi0, 4 in the batched calls, and 2 where the budget
 * holds no more partial planes), RPA_TUNE=0 keeps the
 * defaults (t64k16, t64, t128), RPA_TUNE_CACHE=<file> keeps the choices across
 * processes.  Never fails. */
int rpa_tuned(char *buf, int32_t len, int32_t *needed);

#ifdef __cplusplus
}
#endif

#endif /* RPA_H */
