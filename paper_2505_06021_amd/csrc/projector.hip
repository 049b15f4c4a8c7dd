// The periodic projector method of Sec. 2.3 on the device, FP64:
//
//   S(k) = U(k) D(k) U(k)^H                        (eigendecomposition of the overlap)
//   R_ii(k) = 1 if D_ii(k) >= eps_d, else 0        (eigenvalues in ascending order)
//   R~_ii = prod_k R_ii(k)                          (an index dropped at any k is dropped at all)
//   T(k) = U(k) R~ U(k)^H,   c~(k) = T(k) c(k)
//
// The eigendecomposition is a cyclic two-sided Jacobi method (one workgroup per k): every
// round applies n/2 rotations on disjoint index pairs (a round-robin schedule, so each pair
// meets once a sweep), first to the rows, then to the columns and to the accumulated
// eigenvectors; sweeps repeat until the off-diagonal part is below 1e-30 of the diagonal
// part in squared Frobenius norm.  Each rotation makes one Hermitian 2 x 2 block real with
// a phase, then diagonal with a real rotation, so the eigenvalues come out on the diagonal
// and U's columns are the eigenvectors.  The sort, the mask across k and the two products
// are small kernels.  The projector is O(N_bas^3) per k once per system, outside the
// (q, omega) loop.
#include "common.hpp"

namespace rpa {
namespace {

constexpr int PJ_MAXN = 1024;   // basis size limit (LDS holds one rotation per index pair)

__device__ __forceinline__ int rr_index(int slot, int r, int m) {
  // round-robin schedule of m (even) indices: slot 0 fixed, the others rotate by one a round
  return slot == 0 ? 0 : 1 + (slot - 1 + r) % (m - 1);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(256) void jacobi_kernel(double2 *A, double2 *V, int n, int64_t stride, double *evals,
                                                     int max_sweeps) {
  __shared__ double2 rot[PJ_MAXN / 2];   // (c, s) of the round's pairs
  __shared__ double2 phs[PJ_MAXN / 2];   // phase e = a_pq / |a_pq|
  __shared__ int ip[PJ_MAXN / 2], iq[PJ_MAXN / 2];
  __shared__ double red[2][256];
  __shared__ int go;
  const int b = blockIdx.x, tid = threadIdx.x;
  double2 *a = A + (int64_t)b * stride;
  double2 *v = V + (int64_t)b * stride;
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = tid; e < nn; e += 256) v[e] = make_double2(e / n == e % n ? 1.0 : 0.0, 0.0);
  const int m = n + (n & 1);   // an odd size gets a dummy index n that never rotates
  const int np = m / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int64_t e = tid; e < nn; e += 256) {
      const double2 x = a[e];
      const double q2 = x.x * x.x + x.y * x.y;
      if (e / n == e % n) dia += q2;
      else off += q2;
    }
    red[0][tid] = off;
    red[1][tid] = dia;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) {
        red[0][tid] += red[0][tid + w];
        red[1][tid] += red[1][tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) go = red[0][0] > 1e-30 * red[1][0];
    __syncthreads();
    if (!go) break;
    for (int r = 0; r + 1 < m; ++r) {
      for (int i = tid; i < np; i += 256) {
        int p = rr_index(i, r, m), q = rr_index(m - 1 - i, r, m);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        ip[i] = p;
        iq[i] = q;
        double c = 1.0, s = 0.0;
        double2 e = make_double2(1.0, 0.0);
        if (q < n) {
          const double2 g = a[(int64_t)p * n + q];
          const double ag = sqrt(g.x * g.x + g.y * g.y);
          const double app = a[(int64_t)p * n + p].x, aqq = a[(int64_t)q * n + q].x;
          if (ag > 1e-300 && ag > 1e-17 * (fabs(app) + fabs(aqq))) {
            e = make_double2(g.x / ag, g.y / ag);
            const double zeta = (aqq - app) / (2.0 * ag);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        rot[i] = make_double2(c, s);
        phs[i] = e;
      }
      __syncthreads();
      // rows: A <- J^H A, row p = c A_p - e s A_q, row q = s A_p + e c A_q
      for (int64_t idx = tid; idx < (int64_t)np * n; idx += 256) {
        const int i = (int)(idx / n), k = (int)(idx % n);
        const int p = ip[i], q = iq[i];
        if (q >= n) continue;
        const double c = rot[i].x, s = rot[i].y;
        const double2 e = phs[i];
        const double2 x = a[(int64_t)p * n + k], y = a[(int64_t)q * n + k];
        const double2 ey = cmul(e, y);
        a[(int64_t)p * n + k] = make_double2(c * x.x - s * ey.x, c * x.y - s * ey.y);
        a[(int64_t)q * n + k] = make_double2(s * x.x + c * ey.x, s * x.y + c * ey.y);
      }
      __syncthreads();
      // columns: A <- A J and V <- V J, column p = c X_p - conj(e) s X_q,
      // column q = s X_p + conj(e) c X_q
      for (int64_t idx = tid; idx < (int64_t)np * n; idx += 256) {
        const int i = (int)(idx / n), k = (int)(idx % n);
        const int p = ip[i], q = iq[i];
        if (q >= n) continue;
        const double c = rot[i].x, s = rot[i].y;
        const double2 ce = make_double2(phs[i].x, -phs[i].y);
        {
          const double2 x = a[(int64_t)k * n + p], y = a[(int64_t)k * n + q];
          const double2 ey = cmul(ce, y);
          a[(int64_t)k * n + p] = make_double2(c * x.x - s * ey.x, c * x.y - s * ey.y);
          a[(int64_t)k * n + q] = make_double2(s * x.x + c * ey.x, s * x.y + c * ey.y);
        }
        {
          const double2 x = v[(int64_t)k * n + p], y = v[(int64_t)k * n + q];
          const double2 ey = cmul(ce, y);
          v[(int64_t)k * n + p] = make_double2(c * x.x - s * ey.x, c * x.y - s * ey.y);
          v[(int64_t)k * n + q] = make_double2(s * x.x + c * ey.x, s * x.y + c * ey.y);
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += 256) evals[(int64_t)b * n + i] = a[(int64_t)i * n + i].x;
}

// Ascending order of every k's eigenvalues: perm[k][r] = the index of the r-th smallest
// (ties by index), sorted[k][r] its value.
__global__ __launch_bounds__(256) void eig_sort_kernel(const double *evals, int n, int nk, double *sorted, int32_t *perm) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)nk * n) return;
  const int k = (int)(g / n), i = (int)(g % n);
  const double *l = evals + (int64_t)k * n;
  const double x = l[i];
  int rank = 0;
  for (int j = 0; j < n; ++j) rank += (l[j] < x || (l[j] == x && j < i)) ? 1 : 0;
  sorted[(int64_t)k * n + rank] = x;
  perm[(int64_t)k * n + rank] = i;
}

// keep[r] = 1 if the r-th smallest eigenvalue is >= eps_d at every k
__global__ __launch_bounds__(256) void keep_kernel(const double *sorted, int n, int nk, double eps_d, int32_t *keep) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  int kp = 1;
  for (int k = 0; k < nk; ++k) kp &= sorted[(int64_t)k * n + r] >= eps_d ? 1 : 0;
  keep[r] = kp;
}

// T(k)[i][j] = sum_r keep[r] U[i][perm[r]] conj(U[j][perm[r]])
__global__ __launch_bounds__(256) void projector_kernel(const double2 *V, const int32_t *perm, const int32_t *keep,
                                                        int n, double2 *T) {
  const int k = blockIdx.y;
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)n * n) return;
  const int i = (int)(g / n), j = (int)(g % n);
  const double2 *u = V + (int64_t)k * n * n;
  const int32_t *pk = perm + (int64_t)k * n;
  double re = 0.0, im = 0.0;
  for (int r = 0; r < n; ++r) {
    if (!keep[r]) continue;
    const int c = pk[r];
    const double2 x = u[(int64_t)i * n + c], y = u[(int64_t)j * n + c];
    re += x.x * y.x + x.y * y.y;   // x conj(y)
    im += x.y * y.x - x.x * y.y;
  }
  T[(int64_t)k * n * n + g] = make_double2(re, im);
}

// c~(k)[i][b] = sum_j T(k)[i][j] c(k)[j][b], c of shape [nk][n][nb], out of place
__global__ __launch_bounds__(256) void project_coeff_kernel(const double2 *T, const double2 *c, int n, int nb,
                                                            double2 *out) {
  const int k = blockIdx.y;
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)n * nb) return;
  const int i = (int)(g / nb), bb = (int)(g % nb);
  const double2 *t = T + (int64_t)k * n * n + (int64_t)i * n;
  const double2 *ck = c + (int64_t)k * n * nb;
  double re = 0.0, im = 0.0;
  for (int j = 0; j < n; ++j) {
    const double2 x = t[j], y = ck[(int64_t)j * nb + bb];
    re += x.x * y.x - x.y * y.y;
    im += x.x * y.y + x.y * y.x;
  }
  out[(int64_t)k * n * nb + g] = make_double2(re, im);
}

}  // namespace

int64_t projector_scratch_bytes(int32_t nk, int32_t nbas) {
  const int64_t nn = (int64_t)nbas * nbas;
  return (int64_t)nk * nn * 16 * 2 + (int64_t)nk * nbas * (8 + 8 + 4) + (int64_t)nbas * 4 + 1024;
}

hipError_t launch_projector(hipStream_t s, const double2 *S, int32_t nk, int32_t nbas, double eps_d, void *scratch,
                            double2 *T) {
  if (nk <= 0 || nbas <= 0) return hipSuccess;
  if (nbas > PJ_MAXN || nk > 65535) return hipErrorInvalidValue;
  const int64_t nn = (int64_t)nbas * nbas;
  char *p = (char *)scratch;
  double2 *A = (double2 *)p;
  p += (int64_t)nk * nn * 16;
  double2 *V = (double2 *)p;
  p += (int64_t)nk * nn * 16;
  double *evals = (double *)p;
  p += (int64_t)nk * nbas * 8;
  double *sorted = (double *)p;
  p += (int64_t)nk * nbas * 8;
  int32_t *perm = (int32_t *)p;
  p += (int64_t)nk * nbas * 4;
  int32_t *keep = (int32_t *)p;
  hipError_t e = hipMemcpyAsync(A, S, (size_t)(nk * nn * 16), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(jacobi_kernel, dim3((unsigned)nk), dim3(256), 0, s, A, V, nbas, nn, evals, 60);
  const int64_t nkn = (int64_t)nk * nbas;
  hipLaunchKernelGGL(eig_sort_kernel, dim3((unsigned)((nkn + 255) / 256)), dim3(256), 0, s, evals, nbas, nk, sorted,
                     perm);
  hipLaunchKernelGGL(keep_kernel, dim3((unsigned)((nbas + 255) / 256)), dim3(256), 0, s, sorted, nbas, nk, eps_d, keep);
  hipLaunchKernelGGL(projector_kernel, dim3((unsigned)((nn + 255) / 256), (unsigned)nk), dim3(256), 0, s, V, perm,
                     keep, nbas, T);
  return hipGetLastError();
}

hipError_t launch_project_coeff(hipStream_t s, const double2 *T, const double2 *c, int32_t nk, int32_t nbas,
                                int32_t nb, double2 *out) {
  if (nk <= 0 || nbas <= 0 || nb <= 0) return hipSuccess;
  if (nk > 65535) return hipErrorInvalidValue;
  const int64_t tot = (int64_t)nbas * nb;
  hipLaunchKernelGGL(project_coeff_kernel, dim3((unsigned)((tot + 255) / 256), (unsigned)nk), dim3(256), 0, s, T, c,
                     nbas, nb, out);
  return hipGetLastError();
}

}  // namespace rpa
