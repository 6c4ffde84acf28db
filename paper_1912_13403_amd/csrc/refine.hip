// Eigenpair refinement of the refined form: the FP32 reduction and
// back-transforms give eigenvectors X of the standard-form matrix A within
// FP32 rounding; a few steps of the iterative refinement of Ogita and Aishima
// (Japan J. Indust. Appl. Math. 35 (2018), "Iterative refinement for
// symmetric eigenvalue decomposition") against the FP64 A bring the wanted
// ones to FP64 accuracy.  The steps stop once the largest correction is at
// most tol (the error left is of the order of its square) and delta has come
// down to the smallest separation FP64 resolves, or after max_steps.  After
// the first step only some columns are corrected: those whose measure of
// what is left (their corrections, and for a pair still too close to
// resolve the correction it would need) exceeds tol / 1000, and the refined
// partners of their unfinished pairs.  One step, for the first m columns of X:
//   R = I - X^T X,  S = X^T A X          (columns 0 .. m-1, FP64 MFMA)
//   lambda_j = s_jj / (1 - r_jj)         (Rayleigh quotients)
//   delta = 2 (||S - diag(lambda)|| + ||A|| ||R||)
//   e_ij = (s_ij + lambda_j r_ij) / (lambda_j - lambda_i)  if |lambda_j - lambda_i| > delta,
//          r_ij / 2                                        otherwise (and on the diagonal)
//   (the measure of what is left to correct counts separations below
//   4 sqrt(n) eps max|lambda| / tol as that separation: closer pairs cannot
//   be resolved to tol in FP64, and their corrections are rounding noise)
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
#include <vector>

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

// X[:, J[c]] -> XJ[:, c] for the mj corrected columns
__global__ void gather_kernel(int n, int mj, const int* J, const double* X, long ldx, double* XJ,
                              long ldj) {
  const long tot = (long)n * mj;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), c = (int)(e / n);
    XJ[i + (long)c * ldj] = X[i + (long)J[c] * ldx];
  }
}

// lambda_j = s_jj / g_jj (g = X^T X, so 1 - r_jj = g_jj) for the corrected
// columns j = J[c] (column c of the blocks)
__global__ void diag_lambda_kernel(int mj, const int* J, const double* G, const double* S,
                                   long ld, double* lam) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= mj) return;
  const int j = J[c];
  lam[j] = S[j + (long)c * ld] / G[j + (long)c * ld];
}

// partial sums of ||S - diag(lambda)||_F^2 and ||R||_F^2 over the rows of
// the refined columns (i < m) and over all rows, for the corrected columns
__global__ __launch_bounds__(RB) void norms_kernel(int n, int m, int mj, const int* J,
                                                   const double* G, const double* S, long ld,
                                                   const double* lam, double* part) {
  __shared__ double red[RB];
  const long tot = (long)n * mj;
  double d2 = 0.0, r2 = 0.0, d2a = 0.0, r2a = 0.0;
  for (long e = (long)blockIdx.x * RB + threadIdx.x; e < tot; e += (long)gridDim.x * RB) {
    const int i = (int)(e % n), c = (int)(e / n), j = J[c];
    const double g = G[i + (long)c * ld], sv = S[i + (long)c * ld];
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
// block into rec[0], of the n x m block into dall[0]; dall[1] = the
// smallest separation at which the rounding of a coupling (an n-term dot
// product: about sqrt(n) eps max|lambda|) stays below tol in the measure of
// what is left
__global__ __launch_bounds__(RB) void delta_kernel(int n, int nblk, const double* part,
                                                   const double* lam, double tol, int first,
                                                   double* rec, double* dall) {
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
    // the columns that are not refined keep their FP32 error: the first
    // step's delta over all rows stays the floor of the later steps', whose
    // blocks hold only the columns still corrected
    const double da = 2.0 * (sqrt(d2 + d2a) + am * sqrt(r2 + r2a));
    if (first) dall[2] = da;
    dall[0] = fmax(da, dall[2]);
    dall[1] = 4.0 * sqrt((double)n) * 2.220446049250313e-16 * am / tol;
  }
}

// E (n x mj, FP32; column c corrects column J[c]), the partial maxima,
// each refined column's largest measure as the partner of a corrected one
// (rmax), and each corrected column's largest measure of what is left to
// correct (cmax, as the
// bit patterns of non-negative doubles, which order like the values;
// zeroed before): |e_ij| for a resolved pair, and for a pair too close to
// resolve in this step the correction it would need at separation delta,
// |s_ij + lambda_j r_ij| / delta, so that a column whose close partner is
// still mixed in keeps being corrected until delta has shrunk below the
// pair's separation
__global__ __launch_bounds__(RB) void correction_kernel(int n, int m, int mj, const int* J,
                                                        const double* G, const double* S,
                                                        long ld, const double* lam,
                                                        const double* rec, const double* dall,
                                                        float* E, long lde, double* part,
                                                        unsigned long long* cmax,
                                                        unsigned long long* rmax) {
  __shared__ double red[RB];
  const double floor_ = dall[1];
  const double delta_in = rec[0], delta_all = dall[0];
  const long tot = (long)n * mj;
  double emax = 0.0;
  for (long e = (long)blockIdx.x * RB + threadIdx.x; e < tot; e += (long)gridDim.x * RB) {
    const int i = (int)(e % n), c = (int)(e / n), j = J[c];
    const double g = G[i + (long)c * ld];
    double v, left;
    if (i == j) {
      v = 0.5 * (1.0 - g);
      left = fabs(v);
    } else {
      const double r = -g;
      const double dl = lam[j] - lam[i];
      const double delta = (i < m) ? delta_in : delta_all;
      const double num = fma(lam[j], r, S[i + (long)c * ld]);
      if (fabs(dl) > delta) {
        v = num / dl;
        left = fabs(num) / fmax(fabs(dl), floor_);
      } else {
        // with a column that is not refined (i >= m), r_ij is that column's
        // own FP32 error, which no step reduces: only the coupling counts
        v = 0.5 * r;
        left = fabs(num) / fmax(delta, floor_);
        if (i < m) left = fmax(left, fabs(v));
      }
    }
    E[i + (long)c * lde] = (float)v;
    emax = fmax(emax, fabs(v));
    if (left > 0.0) {
      const unsigned long long bits = (unsigned long long)__double_as_longlong(left);
      atomicMax(&cmax[c], bits);
      // the partner of the pair, if refined, needs the other half of the
      // pair's rotation
      if (i < m && i != j) atomicMax(&rmax[i], bits);
    }
  }
  emax = block_max(emax, red);
  if (threadIdx.x == 0) part[blockIdx.x] = emax;
}

__global__ void clear_u64_kernel(unsigned long long* p, int cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = 0ull;
}

__global__ __launch_bounds__(RB) void emax_kernel(int nblk, const double* part, double* rec) {
  __shared__ double red[RB];
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += RB) v = fmax(v, part[b]);
  v = block_max(v, red);
  if (threadIdx.x == 0) rec[1] = v;
}

// X[:, J[c]] += C[:, c] and the FP32 copy
__global__ void update_kernel(int n, int mj, const int* J, double* X, long ldx, float* X32,
                              long ldx32, const float* C, long ldc) {
  const long tot = (long)n * mj;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), c = (int)(e / n), j = J[c];
    const double x = X[i + (long)j * ldx] + (double)C[i + (long)c * ldc];
    X[i + (long)j * ldx] = x;
    X32[i + (long)j * ldx32] = (float)x;
  }
}

}  // namespace

size_t refine_scratch_bytes(int n, int m) {
  const size_t nm = (size_t)n * m;
  return 3 * nm * sizeof(double) + 2 * nm * sizeof(float) + (4 * RGRID + 64) * sizeof(double) +
         (size_t)m * (sizeof(int) + 2 * sizeof(unsigned long long)) + 1024;
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
  double* XJ = S + nm;
  float* E = (float*)(XJ + nm);
  float* C = E + nm;
  double* part = (double*)(C + nm);
  double* dall = part + 4 * RGRID;
  unsigned long long* cmax = (unsigned long long*)(dall + 64);
  unsigned long long* rmax = cmax + m;
  int* dJ = (int*)(rmax + m);
  // the corrected columns: all m in the first step
  std::vector<int> J(m);
  for (int j = 0; j < m; j++) J[j] = j;
  std::vector<unsigned long long> hmax(m), hrow(m);
  for (int k = 0; k < max_steps; k++) {
    const int mj = (int)J.size();
    const size_t nmj = (size_t)n * mj;
    const unsigned grid =
        (unsigned)std::min<long>(RGRID, std::max<long>(1, (long)(nmj + RB - 1) / RB));
    HSDM_TRY(hipMemcpyAsync(dJ, J.data(), sizeof(int) * mj, hipMemcpyHostToDevice, s));
    HSDM_LAUNCH(clear_u64_kernel, dim3(ceil_div(2 * m, 256)), dim3(256), 0, s, cmax, 2 * m);
    HSDM_TRY(hipGetLastError());
    const double* Xc;  // the corrected columns (ld n or ldx) and A times them (ld ldy)
    long ldc;
    GemmArgs g{};
    if (k == 0) {
      // every column of Y = A X: the Rayleigh quotients of the columns that
      // are not refined; the corrected columns are X's first m
      g.m = n; g.n = n; g.k = n; g.A = A; g.lda = lda; g.B = X; g.ldb = ldx; g.C = Y;
      g.ldc = ldy; g.alpha = 1.0; g.beta = 0.0; g.flags = GF_A_SYM_LOWER;
      HSDM_TRY(gemm_launch(g, s));
      if (m < n) {
        HSDM_LAUNCH(rayleigh_kernel, dim3(n - m), dim3(RB), 0, s, n, m, X, ldx, Y, ldy, lam);
        HSDM_TRY(hipGetLastError());
      }
      Xc = X;
      ldc = ldx;
    } else {
      HSDM_LAUNCH(gather_kernel, dim3((unsigned)std::min<size_t>(4096, (nmj + 255) / 256)),
                  dim3(256), 0, s, n, mj, dJ, X, ldx, XJ, (long)n);
      HSDM_TRY(hipGetLastError());
      g.m = n; g.n = mj; g.k = n; g.A = A; g.lda = lda; g.B = XJ; g.ldb = n; g.C = Y;
      g.ldc = ldy; g.alpha = 1.0; g.beta = 0.0; g.flags = GF_A_SYM_LOWER;
      HSDM_TRY(gemm_launch(g, s));
      Xc = XJ;
      ldc = n;
    }
    g = GemmArgs{};
    g.m = n; g.n = mj; g.k = n; g.A = X; g.lda = ldx; g.B = Xc; g.ldb = ldc; g.C = G; g.ldc = n;
    g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0;
    HSDM_TRY(gemm_launch(g, s));
    g.B = Y; g.ldb = ldy; g.C = S;
    HSDM_TRY(gemm_launch(g, s));
    HSDM_LAUNCH(diag_lambda_kernel, dim3(ceil_div(mj, 256)), dim3(256), 0, s, mj, dJ, G, S,
                (long)n, lam);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(norms_kernel, dim3(grid), dim3(RB), 0, s, n, m, mj, dJ, G, S, (long)n, lam, part);
    HSDM_TRY(hipGetLastError());
    double* rk = rec + 2 * k;
    HSDM_LAUNCH(delta_kernel, dim3(1), dim3(RB), 0, s, n, (int)grid, part, lam, tol,
                (int)(k == 0), rk, dall);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(correction_kernel, dim3(grid), dim3(RB), 0, s, n, m, mj, dJ, G, S, (long)n, lam,
                rk, dall, E, (long)n, part, cmax, rmax);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(emax_kernel, dim3(1), dim3(RB), 0, s, (int)grid, part, rk);
    HSDM_TRY(hipGetLastError());
    // X[:, J] += X E in FP32
    GemmArgsF f{};
    f.m = n; f.n = mj; f.k = n; f.A = X32; f.lda = ldx32; f.B = E; f.ldb = n; f.C = C; f.ldc = n;
    f.alpha = 1.0; f.beta = 0.0;
    HSDM_TRY(gemm_launch(f, s));
    HSDM_LAUNCH(update_kernel, dim3((unsigned)std::min<size_t>(4096, (nmj + 255) / 256)),
                dim3(256), 0, s, n, mj, dJ, X, ldx, X32, ldx32, C, (long)n);
    HSDM_TRY(hipGetLastError());
    // the step's record and the columns' measures to the host: once every
    // correction is at most tol (errors of its square are left) and delta has
    // come down to the smallest separation FP64 resolves (every resolvable
    // pair has been corrected as a pair), the refinement stops
    HSDM_TRY(hipMemcpyAsync(host_rec + 2 * k, rk, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HSDM_TRY(hipMemcpyAsync(hmax.data(), cmax, sizeof(unsigned long long) * mj,
                            hipMemcpyDeviceToHost, s));
    HSDM_TRY(hipMemcpyAsync(hrow.data(), rmax, sizeof(unsigned long long) * m,
                            hipMemcpyDeviceToHost, s));
    double hd[2] = {0.0, 0.0};
    HSDM_TRY(hipMemcpyAsync(hd, dall, sizeof(hd), hipMemcpyDeviceToHost, s));
    HSDM_TRY(hipStreamSynchronize(s));
    *steps_done = k + 1;
    if (!(host_rec[2 * k + 1] > tol) && !(host_rec[2 * k] > hd[1])) break;
    // next: the columns with something left, and the refined partners of
    // their unfinished pairs
    const double keep_tol = 1e-3 * tol;
    std::vector<char> keep(m, 0);
    for (int c = 0; c < mj; c++)
      if (__builtin_bit_cast(double, hmax[c]) > keep_tol) keep[J[c]] = 1;
    for (int i = 0; i < m; i++)
      if (__builtin_bit_cast(double, hrow[i]) > keep_tol) keep[i] = 1;
    std::vector<int> next;
    for (int j = 0; j < m; j++)
      if (keep[j]) next.push_back(j);
    if (next.empty()) break;
    J.swap(next);
  }
  return hipSuccess;
}
