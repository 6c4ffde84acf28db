// Eigenpair refinement of the refined form: the FP32 reduction and
// back-transforms give eigenvectors X of the standard-form matrix A within
// FP32 rounding; a few steps of the iterative refinement of Ogita and Aishima
// (Japan J. Indust. Appl. Math. 35 (2018), "Iterative refinement for
// symmetric eigenvalue decomposition") against the FP64 A bring the wanted
// ones to FP64 accuracy.  The steps stop once the largest correction is at
// most tol (the error left is of the order of its square), or after
// max_steps.  One step, for the first m columns of X:
//   R = I - X^T X,  S = X^T A X          (columns 0 .. m-1, FP64 MFMA)
//   lambda_j = s_jj / (1 - r_jj)         (Rayleigh quotients)
//   delta = 2 (||S - diag(lambda)|| + ||A|| ||R||)
//   e_ij = (s_ij + lambda_j r_ij) / (lambda_j - lambda_i)  if |lambda_j - lambda_i| > delta,
//          r_ij / 2                                        otherwise (and on the diagonal)
//   X[:, j] += X E[:, j]                  (the correction, FP32 MFMA: E is small)
// Every column of X takes part in the correction of the wanted ones: the
// eigenvalues lambda_i of the other columns are their Rayleigh quotients,
// formed once in the first step.  The norms are Frobenius norms (upper
// bounds of the 2-norms) and ||A|| is the largest |lambda|.  Two
// separations are kept: delta over the m x m block of the refined columns,
// which shrinks from step to step and decides the pairs among them, and
// delta over the whole n x m block, which stays at the FP32 error level of
// the columns that are not refined and decides the pairs with one of them.
#include <algorithm>

#include "hsdm_internal.h"
#include "hsdm_phases.h"
#include "hsdm_util.h"

namespace {

constexpr int RB = 256;     // threads per block of the reductions
constexpr int RGRID = 512;  // blocks of the grid-stride reductions

HSDM_DEV double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

HSDM_DEV double block_max(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// lambda_i = (x_i . y_i) / (x_i . x_i) for columns i = i0 + blockIdx.x
__global__ __launch_bounds__(RB) void rayleigh_kernel(int n, int i0, const double* X, long ldx,
                                                      const double* Y, long ldy, double* lam) {
  __shared__ double red[RB];
  const int i = i0 + blockIdx.x;
  const double* x = X + (long)i * ldx;
  const double* y = Y + (long)i * ldy;
  double xy = 0.0, xx = 0.0;
  for (int r = threadIdx.x; r < n; r += RB) {
    xy = fma(x[r], y[r], xy);
    xx = fma(x[r], x[r], xx);
  }
  xy = block_sum(xy, red);
  xx = block_sum(xx, red);
  if (threadIdx.x == 0) lam[i] = xy / xx;
}

// lambda_j = s_jj / g_jj (g = X^T X, so 1 - r_jj = g_jj), j < m
__global__ void diag_lambda_kernel(int m, const double* G, const double* S, long ld,
                                   double* lam) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) lam[j] = S[j + (long)j * ld] / G[j + (long)j * ld];
}

// partial sums of ||S - diag(lambda)||_F^2 and ||R||_F^2 over the m x m
// block (rows i < m) and over the whole n x m block
__global__ __launch_bounds__(RB) void norms_kernel(int n, int m, const double* G,
                                                   const double* S, long ld, const double* lam,
                                                   double* part) {
  __shared__ double red[RB];
  const long tot = (long)n * m;
  double d2 = 0.0, r2 = 0.0, d2a = 0.0, r2a = 0.0;
  for (long e = (long)blockIdx.x * RB + threadIdx.x; e < tot; e += (long)gridDim.x * RB) {
    const int i = (int)(e % n), j = (int)(e / n);
    const double g = G[i + (long)j * ld], sv = S[i + (long)j * ld];
    const double r = (i == j) ? 1.0 - g : -g;
    const double d = (i == j) ? sv - lam[j] : sv;
    if (i < m) {
      d2 = fma(d, d, d2);
      r2 = fma(r, r, r2);
    } else {
      d2a = fma(d, d, d2a);
      r2a = fma(r, r, r2a);
    }
  }
  d2 = block_sum(d2, red);
  r2 = block_sum(r2, red);
  d2a = block_sum(d2a, red);
  r2a = block_sum(r2a, red);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = d2;
    part[4 * blockIdx.x + 1] = r2;
    part[4 * blockIdx.x + 2] = d2a;
    part[4 * blockIdx.x + 3] = r2a;
  }
}

// delta = 2 (||S - diag(lambda)||_F + max_i |lambda_i| ||R||_F) of the m x m
// block into rec[0], of the n x m block into dall[0]
__global__ __launch_bounds__(RB) void delta_kernel(int n, int nblk, const double* part,
                                                   const double* lam, double* rec,
                                                   double* dall) {
  __shared__ double red[RB];
  double d2 = 0.0, r2 = 0.0, d2a = 0.0, r2a = 0.0, am = 0.0;
  for (int b = threadIdx.x; b < nblk; b += RB) {
    d2 += part[4 * b];
    r2 += part[4 * b + 1];
    d2a += part[4 * b + 2];
    r2a += part[4 * b + 3];
  }
  for (int i = threadIdx.x; i < n; i += RB) am = fmax(am, fabs(lam[i]));
  d2 = block_sum(d2, red);
  r2 = block_sum(r2, red);
  d2a = block_sum(d2a, red);
  r2a = block_sum(r2a, red);
  am = block_max(am, red);
  if (threadIdx.x == 0) {
    rec[0] = 2.0 * (sqrt(d2) + am * sqrt(r2));
    dall[0] = 2.0 * (sqrt(d2 + d2a) + am * sqrt(r2 + r2a));
  }
}

// E (n x m, FP32) and the partial maxima of |e_ij|
__global__ __launch_bounds__(RB) void correction_kernel(int n, int m, const double* G,
                                                        const double* S, long ld,
                                                        const double* lam, const double* rec,
                                                        const double* dall, float* E, long lde,
                                                        double* part) {
  __shared__ double red[RB];
  const double delta_in = rec[0], delta_all = dall[0];
  const long tot = (long)n * m;
  double emax = 0.0;
  for (long e = (long)blockIdx.x * RB + threadIdx.x; e < tot; e += (long)gridDim.x * RB) {
    const int i = (int)(e % n), j = (int)(e / n);
    const double g = G[i + (long)j * ld];
    double v;
    if (i == j) {
      v = 0.5 * (1.0 - g);
    } else {
      const double r = -g;
      const double dl = lam[j] - lam[i];
      const double delta = (i < m) ? delta_in : delta_all;
      v = (fabs(dl) > delta) ? fma(lam[j], r, S[i + (long)j * ld]) / dl : 0.5 * r;
    }
    E[i + (long)j * lde] = (float)v;
    emax = fmax(emax, fabs(v));
  }
  emax = block_max(emax, red);
  if (threadIdx.x == 0) part[blockIdx.x] = emax;
}

__global__ __launch_bounds__(RB) void emax_kernel(int nblk, const double* part, double* rec) {
  __shared__ double red[RB];
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += RB) v = fmax(v, part[b]);
  v = block_max(v, red);
  if (threadIdx.x == 0) rec[1] = v;
}

// X[:, j] += C[:, j] and the FP32 copy, j < m
__global__ void update_kernel(int n, int m, double* X, long ldx, float* X32, long ldx32,
                              const float* C, long ldc) {
  const long tot = (long)n * m;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const double x = X[i + (long)j * ldx] + (double)C[i + (long)j * ldc];
    X[i + (long)j * ldx] = x;
    X32[i + (long)j * ldx32] = (float)x;
  }
}

}  // namespace

size_t refine_scratch_bytes(int n, int m) {
  const size_t nm = (size_t)n * m;
  return 2 * nm * sizeof(double) + 2 * nm * sizeof(float) + (4 * RGRID + 64) * sizeof(double);
}

hipError_t refine_run(int n, int m, const double* A, long lda, double* X, long ldx, float* X32,
                      long ldx32, double* Y, long ldy, double* lam, int max_steps, double tol,
                      void* scratch, double* rec, double* host_rec, int* steps_done,
                      hipStream_t s) {
  *steps_done = 0;
  if (n <= 0 || m <= 0 || max_steps <= 0) return hipSuccess;
  char* p = (char*)scratch;
  const size_t nm = (size_t)n * m;
  double* G = (double*)p;
  double* S = G + nm;
  float* E = (float*)(S + nm);
  float* C = E + nm;
  double* part = (double*)(C + nm);
  double* dall = part + 4 * RGRID;
  const unsigned grid = (unsigned)std::min<long>(RGRID, std::max<long>(1, (long)(nm + RB - 1) / RB));
  for (int k = 0; k < max_steps; k++) {
    // Y = A X: every column in the first step (Rayleigh quotients of the
    // columns that are not refined), the wanted ones afterwards
    const int cols = (k == 0) ? n : m;
    GemmArgs g{};
    g.m = n; g.n = cols; g.k = n; g.A = A; g.lda = lda; g.B = X; g.ldb = ldx; g.C = Y; g.ldc = ldy;
    g.alpha = 1.0; g.beta = 0.0; g.flags = GF_A_SYM_LOWER;
    HSDM_TRY(gemm_launch(g, s));
    if (k == 0 && m < n) {
      HSDM_LAUNCH(rayleigh_kernel, dim3(n - m), dim3(RB), 0, s, n, m, X, ldx, Y, ldy, lam);
      HSDM_TRY(hipGetLastError());
    }
    g = GemmArgs{};
    g.m = n; g.n = m; g.k = n; g.A = X; g.lda = ldx; g.B = X; g.ldb = ldx; g.C = G; g.ldc = n;
    g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0;
    HSDM_TRY(gemm_launch(g, s));
    g.B = Y; g.ldb = ldy; g.C = S;
    HSDM_TRY(gemm_launch(g, s));
    HSDM_LAUNCH(diag_lambda_kernel, dim3(ceil_div(m, 256)), dim3(256), 0, s, m, G, S, (long)n,
                lam);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(norms_kernel, dim3(grid), dim3(RB), 0, s, n, m, G, S, (long)n, lam, part);
    HSDM_TRY(hipGetLastError());
    double* rk = rec + 2 * k;
    HSDM_LAUNCH(delta_kernel, dim3(1), dim3(RB), 0, s, n, (int)grid, part, lam, rk, dall);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(correction_kernel, dim3(grid), dim3(RB), 0, s, n, m, G, S, (long)n, lam, rk,
                dall, E, (long)n, part);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(emax_kernel, dim3(1), dim3(RB), 0, s, (int)grid, part, rk);
    HSDM_TRY(hipGetLastError());
    // X[:, :m] += X E in FP32
    GemmArgsF f{};
    f.m = n; f.n = m; f.k = n; f.A = X32; f.lda = ldx32; f.B = E; f.ldb = n; f.C = C; f.ldc = n;
    f.alpha = 1.0; f.beta = 0.0;
    HSDM_TRY(gemm_launch(f, s));
    HSDM_LAUNCH(update_kernel, dim3(grid), dim3(256), 0, s, n, m, X, ldx, X32, ldx32, C,
                (long)n);
    HSDM_TRY(hipGetLastError());
    // the step's record to the host: a correction below tol leaves errors of
    // its square, and the refinement stops
    HSDM_TRY(hipMemcpyAsync(host_rec + 2 * k, rk, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HSDM_TRY(hipStreamSynchronize(s));
    *steps_done = k + 1;
    if (!(host_rec[2 * k + 1] > tol)) break;
  }
  return hipSuccess;
}
