// Small memory kernels: fill, 2-D copy, symmetric completion, max-abs
// column sum.  All are HBM-bound element-wise passes.
#include "hsdm_internal.h"
#include "hsdm_util.h"

namespace {

__global__ void fill_kernel(double* a, long lda, int m, int n, double v) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long tot = (long)m * n;
  for (; idx < tot; idx += (long)gridDim.x * blockDim.x) {
    int i = (int)(idx % m), j = (int)(idx / m);
    a[i + (long)j * lda] = v;
  }
}

__global__ void copy_kernel(const double* a, long lda, double* b, long ldb, int m, int n) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long tot = (long)m * n;
  for (; idx < tot; idx += (long)gridDim.x * blockDim.x) {
    int i = (int)(idx % m), j = (int)(idx / m);
    b[i + (long)j * ldb] = a[i + (long)j * lda];
  }
}

// b = full symmetric matrix whose lower triangle is a's lower triangle.
// 32x32 tiles through LDS so that both the direct and the mirrored writes
// are coalesced.
__global__ void sym_full_kernel(const double* a, long lda, double* b, long ldb, int n) {
  __shared__ double t[32][33];
  const int bi = blockIdx.x, bj = blockIdx.y;
  if (bi < bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    int i = bi * 32 + tx, j = bj * 32 + r;
    double v = 0.0;
    if (i < n && j < n) v = (i >= j) ? a[i + (long)j * lda] : a[j + (long)i * lda];
    t[r][tx] = v;
    if (i < n && j < n) b[i + (long)j * ldb] = v;
  }
  __syncthreads();
  if (bi == bj) return;
  for (int r = ty; r < 32; r += 8) {
    int i = bj * 32 + tx, j = bi * 32 + r;  // element (i,j) = t[tx][r] transposed
    if (i < n && j < n) b[i + (long)j * ldb] = t[tx][r];
  }
}

// a (in place): upper triangle := transpose of the lower triangle.
__global__ void mirror_kernel(double* a, long lda, int n) {
  __shared__ double t[32][33];
  const int bi = blockIdx.x, bj = blockIdx.y;
  if (bi < bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    int i = bi * 32 + tx, j = bj * 32 + r;
    t[r][tx] = (i < n && j < n) ? a[i + (long)j * lda] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    int i = bj * 32 + tx, j = bi * 32 + r;  // upper element (i, j), i <= j
    if (i < n && j < n && i < j) a[i + (long)j * lda] = t[tx][r];
  }
}

// norm1 of the symmetric matrix given by its lower triangle: max_j sum_i |a_ij|
__global__ void colsum_kernel(const double* a, long lda, int n, double* colsum) {
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    s += fabs(i >= j ? a[i + (long)j * lda] : a[j + (long)i * lda]);
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) colsum[j] = red[0];
}

__global__ void max_kernel(const double* x, int n, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s = fmax(s, x[i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

inline unsigned grid_for(long tot) {
  long g = (tot + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

hipError_t dev_fill(double* a, long lda, int m, int n, double v, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for((long)m * n)), dim3(256), 0, s, a, lda, m, n, v);
  return hipGetLastError();
}

hipError_t dev_copy(const double* a, long lda, double* b, long ldb, int m, int n, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for((long)m * n)), dim3(256), 0, s, a, lda, b, ldb, m,
                     n);
  return hipGetLastError();
}

hipError_t dev_sym_full(const double* a, long lda, double* b, long ldb, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 g(ceil_div(n, 32), ceil_div(n, 32));
  hipLaunchKernelGGL(sym_full_kernel, g, dim3(256), 0, s, a, lda, b, ldb, n);
  return hipGetLastError();
}

hipError_t dev_mirror_lower(double* a, long lda, int n, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  dim3 g(ceil_div(n, 32), ceil_div(n, 32));
  hipLaunchKernelGGL(mirror_kernel, g, dim3(256), 0, s, a, lda, n);
  return hipGetLastError();
}

hipError_t dev_norm1_sym(const double* a, long lda, int n, double* colsum, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3(n), dim3(256), 0, s, a, lda, n, colsum);
  HSDM_TRY(hipGetLastError());
  hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, s, colsum, n, out);
  return hipGetLastError();
}
