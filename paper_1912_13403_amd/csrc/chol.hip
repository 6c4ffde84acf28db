// Cholesky factorization S = L L^T together with L^{-1}.
//
// The overlap matrix of Eq. (3) is SPD; its factor is what the paper's
// benchmark section calls the once-per-geometry step.  The path keeps the
// explicit inverse L^{-1}: every later use of the factor (the standard form
// L^{-1} H L^{-T} and the back-transformation C = L^{-T} Y) then becomes a
// plain GEMM on the matrix cores, and L^{-1} is cached with S.
//
// Recursion on [[L11, 0], [L21, L22]]:
//   L11, L11^{-1}      <- recurse on S11
//   L21 = S21 L11^{-T} (GEMM, triangular B)
//   S22 <- S22 - L21 L21^T (GEMM, lower tiles)
//   L22, L22^{-1}      <- recurse on S22
//   (L^{-1})21 = -L22^{-1} L21 L11^{-1} (two GEMMs, triangular operands)
// Leaves of at most 64 columns are factored and inverted by one wavefront in
// LDS.  A non-positive pivot is reported through the device status word with
// its 1-based column.
#include "hsdm_internal.h"
#include "hsdm_util.h"

namespace {

constexpr int LEAF = 64;

HSDM_DEV double lane_value(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// One wavefront factors and inverts a leaf of nb <= 64 columns.  Lane t
// keeps row t of the factor in registers (right-looking: at step k the
// column below the pivot is scaled and each later column j receives
// -L[t][k] L[j][k], with L[j][k] read from lane j); entries above the
// diagonal are computed along and discarded.  The inverse is formed by
// forward substitution, lane c computing column c with the factor
// broadcast from LDS.
__global__ __launch_bounds__(64) void chol_leaf_kernel(int nb, double* A, long lda, double* Li,
                                                       long ldi, DevStatusWord* st, int col0) {
  __shared__ double L[LEAF][LEAF + 1];
  const int t = threadIdx.x;
  double row[LEAF];
#pragma unroll
  for (int j = 0; j < LEAF; j++) row[j] = (t < nb && j < nb && t >= j) ? A[t + (long)j * lda] : 0.0;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < LEAF; k++) {
    if (k < nb && ok) {
      const double piv = lane_value(row[k], k);
      if (!(piv > 0.0)) {
        if (t == 0) dev_set_status(st, DS_NOT_SPD, col0 + k + 1);
        ok = false;
      } else {
        const double lkk = sqrt(piv), rl = 1.0 / lkk;
        row[k] = (t == k) ? lkk : ((t > k) ? row[k] * rl : 0.0);
        const double ltk = row[k];
#pragma unroll
        for (int j = k + 1; j < LEAF; j++) row[j] -= ltk * lane_value(row[k], j);
      }
    }
  }
  // the factor (lower triangle) to LDS and to A
#pragma unroll
  for (int j = 0; j < LEAF; j++) {
    const double v = (t >= j && t < nb && j < nb) ? row[j] : 0.0;
    L[t][j] = v;
    if (t < nb && j < nb) A[t + (long)j * lda] = v;
  }
  __syncthreads();
  // column c = t of the inverse: L x = e_c
  double x[LEAF];
#pragma unroll
  for (int i = 0; i < LEAF; i++) {
    double s = (i == t) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < i; k++) s -= L[i][k] * x[k];
    x[i] = (i < nb) ? s / L[i][i] : 0.0;
  }
  // transpose through LDS so that each store instruction writes a column
  __syncthreads();
#pragma unroll
  for (int j = 0; j < LEAF; j++) L[j][t] = x[j];
  __syncthreads();
  if (t < nb) {
#pragma unroll
    for (int j = 0; j < LEAF; j++) {
      if (j < nb) {
        const bool low = t >= j;
        Li[t + (long)j * ldi] = (low && ok) ? L[t][j] : (low ? NAN : 0.0);
      }
    }
  }
}

hipError_t rec(int n, double* A, long lda, double* Li, long ldi, double* T, long ldt,
               DevStatusWord* st, int col0, hipStream_t s) {
  if (n <= LEAF) {
    HSDM_LAUNCH(chol_leaf_kernel, dim3(1), dim3(64), 0, s, n, A, lda, Li, ldi, st, col0);
    return hipGetLastError();
  }
  int n1 = ((n / 2) / LEAF) * LEAF;
  if (n1 == 0) n1 = LEAF;
  const int n2 = n - n1;
  double* A21 = A + n1;
  double* A22 = A + n1 + (long)n1 * lda;
  double* Li21 = Li + n1;
  double* Li22 = Li + n1 + (long)n1 * ldi;

  HSDM_TRY(rec(n1, A, lda, Li, ldi, T, ldt, st, col0, s));
  // T = S21 * L11^{-T}
  GemmArgs g{};
  g.m = n2; g.n = n1; g.k = n1;
  g.A = A21; g.lda = lda; g.B = Li; g.ldb = ldi; g.C = T; g.ldc = ldt;
  g.alpha = 1.0; g.beta = 0.0; g.ta = 0; g.tb = 1; g.flags = GF_KB_UPPER;
  HSDM_TRY(gemm_launch(g, s));
  HSDM_TRY(dev_copy(T, ldt, A21, lda, n2, n1, s));
  // S22 -= L21 L21^T (lower)
  g = GemmArgs{};
  g.m = n2; g.n = n2; g.k = n1;
  g.A = A21; g.lda = lda; g.B = A21; g.ldb = lda; g.C = A22; g.ldc = lda;
  g.alpha = -1.0; g.beta = 1.0; g.ta = 0; g.tb = 1;
  g.flags = GF_C_LOWER_TILES | GF_C_LOWER_ONLY;
  HSDM_TRY(gemm_launch(g, s));
  HSDM_TRY(rec(n2, A22, lda, Li22, ldi, T, ldt, st, col0 + n1, s));
  // T = L21 * L11^{-1}
  g = GemmArgs{};
  g.m = n2; g.n = n1; g.k = n1;
  g.A = A21; g.lda = lda; g.B = Li; g.ldb = ldi; g.C = T; g.ldc = ldt;
  g.alpha = 1.0; g.beta = 0.0; g.ta = 0; g.tb = 0; g.flags = GF_KB_LOWER;
  HSDM_TRY(gemm_launch(g, s));
  // (L^{-1})21 = -L22^{-1} * T
  g = GemmArgs{};
  g.m = n2; g.n = n1; g.k = n2;
  g.A = Li22; g.lda = ldi; g.B = T; g.ldb = ldt; g.C = Li21; g.ldc = ldi;
  g.alpha = -1.0; g.beta = 0.0; g.ta = 0; g.tb = 0; g.flags = GF_KA_LOWER;
  return gemm_launch(g, s);
}

// Zeros above the diagonal of an n x n matrix: workgroup (x, y) clears rows
// [256 x, 256 x + 256) of columns y, y + gridDim.y, ...
__global__ __launch_bounds__(256) void zero_upper_kernel(double* A, long lda, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  for (int j = blockIdx.y; j < n; j += gridDim.y)
    if (i < j) A[i + (long)j * lda] = 0.0;
}

hipError_t zero_upper(double* A, long lda, int n, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  HSDM_LAUNCH(zero_upper_kernel, dim3(ceil_div(n, 256), n < 16384 ? n : 16384), dim3(256),
                     0, s, A, lda, n);
  return hipGetLastError();
}

}  // namespace

hipError_t chol_inv(int n, double* A, long lda, double* Li, long ldi, double* T, long ldt,
                    DevStatusWord* st, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  // The recursion reads the inverse's blocks above the diagonal as zeros
  // (triangular operands are read by whole tiles) and never reads the
  // factor's; both are cleared once, not block by block.
  HSDM_TRY(zero_upper(Li, ldi, n, s));
  HSDM_TRY(rec(n, A, lda, Li, ldi, T, ldt, st, 0, s));
  return zero_upper(A, lda, n, s);
}
