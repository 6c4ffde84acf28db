// Hermitian pencils (complex H_k, S_k of the unit tasks of Eq. (13), the
// complex solver interfaces of Sec. 2.1) through the real symmetric
// embedding R(A) = [[Re A, -Im A], [Im A, Re A]] of size 2n.
//
// R(H) c = eps R(S) c has the eigenvalues of H u = eps S u, each twice: the
// eigenvector u = x + i y gives the real pair [x; y] and [-y; x].  With one
// occupation per real eigenpair and twice the electron count, the real
// density matrix D_R of the embedded pencil holds D = D_R[:n, :n] +
// i D_R[n:, :n] (the pair adds x x^T + y y^T = Re(u u^H) to the upper left
// block and y x^T - x y^T = Im(u u^H) to the lower left block); the same
// holds for E.  These kernels build R from the lower triangle of a Hermitian
// matrix and read D, E and the eigenvalues back out; every other step runs in
// the real path on the embedded pencil.
#include "hsdm_internal.h"
#include "hsdm_phases.h"
#include "hsdm_util.h"

namespace {

constexpr int TT = 32;

// Lower triangle of R(A) (2n x 2n, leading dimension ldr) from the lower
// triangle of A (n x n, interleaved complex, leading dimension lda in complex
// elements); the imaginary parts of A's diagonal are taken as zero.
// Workgroup (ti, tj), ti >= tj, reads the 32 x 32 tile of A at (32 ti, 32 tj)
// once and writes its pieces of the three lower blocks of R; the transposed
// piece (Im A above the diagonal of the lower left block) goes through LDS so
// that both the reads and the writes are coalesced.
__global__ __launch_bounds__(256) void herm_embed_kernel(int n, const double2* A, long lda,
                                                         double* R, long ldr) {
  const int ti = blockIdx.x, tj = blockIdx.y;
  if (ti < tj) return;
  __shared__ double im[TT][TT + 1];
  const int tx = threadIdx.x & (TT - 1), ty = threadIdx.x / TT;
  const long nn = n;
  for (int c = ty; c < TT; c += 256 / TT) {
    const int i = ti * TT + tx, j = tj * TT + c;
    const bool ok = i < n && j < n && i >= j;
    double re = 0.0, ig = 0.0;
    if (ok) {
      const double2 a = A[i + (long)j * lda];
      re = a.x;
      ig = (i == j) ? 0.0 : a.y;
      R[i + (long)j * ldr] = re;
      R[(nn + i) + (nn + j) * ldr] = re;
      R[(nn + i) + (long)j * ldr] = ig;
    }
    im[tx][c] = ig;
  }
  __syncthreads();
  // R[n + j, i] = Im A[j, i] = -Im A[i, j] for i > j
  for (int c = ty; c < TT; c += 256 / TT) {
    const int i = ti * TT + c, j = tj * TT + tx;
    if (i < n && j < n && i > j) R[(nn + j) + (long)i * ldr] = -im[c][tx];
  }
}

// X[i, j] = R[i, j] + i R[n + i, j] for 0 <= i, j < n.
__global__ __launch_bounds__(256) void herm_extract_kernel(int n, const double* R, long ldr,
                                                           double2* X, long ldx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  for (int j = blockIdx.y; j < n; j += gridDim.y) {
    const double* col = R + (long)j * ldr;
    X[i + (long)j * ldx] = make_double2(col[i], col[n + i]);
  }
}

// eval[l] = mean of the embedded pencil's pair (2l, 2l + 1).
__global__ void herm_pair_eval_kernel(int n, const double* lam2, double* eval) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < n) eval[l] = 0.5 * (lam2[2 * l] + lam2[2 * l + 1]);
}

// X[i, l] = R[i, 2l] + i R[n + i, 2l]: one real eigenvector of each pair.
__global__ __launch_bounds__(256) void herm_extract_pairs_kernel(int n, int m, const double* R,
                                                                 long ldr, double2* X, long ldx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  for (int l = blockIdx.y; l < m; l += gridDim.y) {
    const double* col = R + (long)(2 * l) * ldr;
    X[i + (long)l * ldx] = make_double2(col[i], col[n + i]);
  }
}

// JQ = [-Q_y; Q_x] for the k2 columns of Q = [Q_x; Q_y] (2n rows): the real
// form of multiplication by i.
__global__ __launch_bounds__(256) void herm_jmul_kernel(int n, int k2, const double* Q, long ldq,
                                                        double* JQ, long ldj) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n || j >= k2) return;
  const double x = Q[i + (long)j * ldq], y = Q[n + i + (long)j * ldq];
  JQ[i + (long)j * ldj] = -y;
  JQ[n + i + (long)j * ldj] = x;
}

// X[i, a] = sum_j (Q[i, j] + i Q[n + i, j]) c[j, a] for a < k (c: k2 x k complex).
__global__ __launch_bounds__(256) void herm_combine_kernel(int n, int k2, int k, const double* Q,
                                                           long ldq, const double2* c, double2* X,
                                                           long ldx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int a = blockIdx.y;
  if (i >= n || a >= k) return;
  double re = 0.0, im = 0.0;
  for (int j = 0; j < k2; j++) {
    const double x = Q[i + (long)j * ldq], y = Q[n + i + (long)j * ldq];
    const double2 w = c[j + (long)a * k2];
    re += x * w.x - y * w.y;
    im += x * w.y + y * w.x;
  }
  X[i + (long)a * ldx] = make_double2(re, im);
}

}  // namespace

hipError_t herm_extract_pairs(int n, int m, const double* R, long ldr, void* X, long ldx,
                              hipStream_t s) {
  if (m <= 0) return hipSuccess;
  HSDM_LAUNCH(herm_extract_pairs_kernel, dim3(ceil_div(n, 256), m < 4096 ? m : 4096),
                     dim3(256), 0, s, n, m, R, ldr, (double2*)X, ldx);
  return hipGetLastError();
}

hipError_t herm_jmul(int n, int k2, const double* Q, long ldq, double* JQ, long ldj,
                     hipStream_t s) {
  HSDM_LAUNCH(herm_jmul_kernel, dim3(ceil_div(n, 256), k2), dim3(256), 0, s, n, k2, Q, ldq,
                     JQ, ldj);
  return hipGetLastError();
}

hipError_t herm_combine(int n, int k2, int k, const double* Q, long ldq, const void* c, void* X,
                        long ldx, hipStream_t s) {
  HSDM_LAUNCH(herm_combine_kernel, dim3(ceil_div(n, 256), k), dim3(256), 0, s, n, k2, k, Q,
                     ldq, (const double2*)c, (double2*)X, ldx);
  return hipGetLastError();
}

hipError_t herm_embed(int n, const void* A, long lda, double* R, long ldr, hipStream_t s) {
  const int t = ceil_div(n, TT);
  HSDM_LAUNCH(herm_embed_kernel, dim3(t, t), dim3(256), 0, s, n, (const double2*)A, lda, R,
                     ldr);
  return hipGetLastError();
}

hipError_t herm_extract(int n, const double* R, long ldr, void* X, long ldx, hipStream_t s) {
  HSDM_LAUNCH(herm_extract_kernel, dim3(ceil_div(n, 256), n < 4096 ? n : 4096), dim3(256), 0,
                     s, n, R, ldr, (double2*)X, ldx);
  return hipGetLastError();
}

hipError_t herm_pair_eval(int n, const double* lam2, double* eval, hipStream_t s) {
  HSDM_LAUNCH(herm_pair_eval_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, lam2, eval);
  return hipGetLastError();
}
