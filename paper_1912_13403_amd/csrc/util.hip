// Small memory kernels: fill, 2-D copy, symmetric completion, max-abs
// column sum.  All are HBM-bound element-wise passes.
#include "hsdm_internal.h"
#include "hsdm_util.h"

#include <algorithm>
#include <mutex>
#include <shared_mutex>

namespace {

__global__ void fill_kernel(double* a, long lda, int m, int n, double v) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long tot = (long)m * n;
  for (; idx < tot; idx += (long)gridDim.x * blockDim.x) {
    int i = (int)(idx % m), j = (int)(idx / m);
    a[i + (long)j * lda] = v;
  }
}

template <class Ti, class To>
__global__ void copy_kernel(const Ti* a, long lda, To* b, long ldb, int m, int n) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long tot = (long)m * n;
  for (; idx < tot; idx += (long)gridDim.x * blockDim.x) {
    int i = (int)(idx % m), j = (int)(idx / m);
    b[i + (long)j * ldb] = (To)a[i + (long)j * lda];
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

// 64-bit content hash of the lower triangle of a (real: double; complex:
// interleaved pairs, the imaginary part of the diagonal left out, as the
// solvers never read it).  Every element contributes mix(bits + position *
// odd constant) and the contributions are added with wrap-around, an
// order-free sum, so the result does not depend on the launch shape.  Used
// to tell whether a cached factorization belongs to the S passed now.
HSDM_DEV unsigned long long mix64(unsigned long long x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

__global__ void hash_clear_kernel(unsigned long long* out, int cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) out[i] = 0ull;
}

__global__ void hash_lower_kernel(const double* a, long lda, int n, int cplx,
                                  unsigned long long* out) {
  const int per = cplx ? 2 : 1;
  const int sh = cplx ? 1 : 0;  // value t of a column: row t >> sh, part t & sh
  unsigned long long acc = 0ull;
  for (int j = blockIdx.y; j < n; j += gridDim.y) {
    const long rows = (long)(n - j) * per;  // values of column j from row j down
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < rows;
         t += (long)gridDim.x * blockDim.x) {
      const long i = j + (t >> sh);
      const int part = (int)(t & sh);
      if (cplx && part == 1 && i == j) continue;
      const double v = a[(i + (long)j * lda) * per + part];
      const unsigned long long pos = (unsigned long long)((i + (long)j * n) * per + part);
      acc += mix64((unsigned long long)__double_as_longlong(v) + pos * 0x9E3779B97F4A7C15ull);
    }
  }
  // one atomic per workgroup (the sum is order-free)
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ unsigned long long wsum[4];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (t) atomicAdd(out, t);
  }
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
  HSDM_LAUNCH(fill_kernel, dim3(grid_for((long)m * n)), dim3(256), 0, s, a, lda, m, n, v);
  return hipGetLastError();
}

template <class Ti, class To>
hipError_t copy_as(const Ti* a, long lda, To* b, long ldb, int m, int n, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  HSDM_LAUNCH((copy_kernel<Ti, To>), dim3(grid_for((long)m * n)), dim3(256), 0, s, a, lda, b,
              ldb, m, n);
  return hipGetLastError();
}

hipError_t dev_copy(const double* a, long lda, double* b, long ldb, int m, int n, hipStream_t s) {
  return copy_as(a, lda, b, ldb, m, n, s);
}
hipError_t dev_copy(const float* a, long lda, float* b, long ldb, int m, int n, hipStream_t s) {
  return copy_as(a, lda, b, ldb, m, n, s);
}
hipError_t dev_convert(const double* a, long lda, float* b, long ldb, int m, int n, hipStream_t s) {
  return copy_as(a, lda, b, ldb, m, n, s);
}
hipError_t dev_convert(const float* a, long lda, double* b, long ldb, int m, int n, hipStream_t s) {
  return copy_as(a, lda, b, ldb, m, n, s);
}

hipError_t dev_sym_full(const double* a, long lda, double* b, long ldb, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 g(ceil_div(n, 32), ceil_div(n, 32));
  HSDM_LAUNCH(sym_full_kernel, g, dim3(256), 0, s, a, lda, b, ldb, n);
  return hipGetLastError();
}

hipError_t dev_mirror_lower(double* a, long lda, int n, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  dim3 g(ceil_div(n, 32), ceil_div(n, 32));
  HSDM_LAUNCH(mirror_kernel, g, dim3(256), 0, s, a, lda, n);
  return hipGetLastError();
}

hipError_t dev_norm1_sym(const double* a, long lda, int n, double* colsum, double* out,
                         hipStream_t s) {
  HSDM_LAUNCH(colsum_kernel, dim3(n), dim3(256), 0, s, a, lda, n, colsum);
  HSDM_TRY(hipGetLastError());
  HSDM_LAUNCH(max_kernel, dim3(1), dim3(256), 0, s, colsum, n, out);
  return hipGetLastError();
}

hipError_t dev_hash_clear(unsigned long long* out, int cnt, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  HSDM_LAUNCH(hash_clear_kernel, dim3(ceil_div(cnt, 256)), dim3(256), 0, s, out, cnt);
  return hipGetLastError();
}

hipError_t dev_hash_lower(const void* a, long lda, int n, int cplx, unsigned long long* out,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long rows = (long)n * (cplx ? 2 : 1);
  const unsigned gx = (unsigned)std::min<long>(ceil_div(rows, 256), 16);
  HSDM_LAUNCH(hash_lower_kernel, dim3(gx, std::min(n, 2048)), dim3(256), 0, s, (const double*)a, lda, n,
                     cplx, out);
  return hipGetLastError();
}

// ---- the launch gate of concurrent solves -------------------------------
namespace {
thread_local bool coop_shared = false;
std::shared_mutex launch_gate;
}  // namespace

void coop_set_shared(bool on) { coop_shared = on; }
bool coop_get_shared() { return coop_shared; }

LaunchGate::LaunchGate() : held(coop_shared) {
  if (held) launch_gate.lock_shared();
}
LaunchGate::~LaunchGate() {
  if (held) launch_gate.unlock_shared();
}

hipError_t coop_launch(const char* name, double flops, double bytes, bool whole_phase,
                       bool cooperative, const void* fn, dim3 grid, dim3 block, void** args,
                       hipStream_t s, int nbound) {
  // Captured into a graph (a solve recorded for replay), the kernel becomes
  // an ordinary node: the graph's nodes run one after another on the device,
  // so the kernel, whose grid never exceeds the resident workgroup count,
  // still has all its workgroups placed at once.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (cooperative && hipStreamIsCapturing(s, &cap) == hipSuccess &&
      cap == hipStreamCaptureStatusActive)
    cooperative = false;
  auto launch = [&]() -> hipError_t {
    kt_begin(name, flops, bytes, nbound, s, whole_phase);
    hipError_t e = cooperative ? hipLaunchCooperativeKernel(fn, grid, block, args, 0, s)
                               : hipLaunchKernel(fn, grid, block, args, 0, s);
    kt_end(s);
    return e;
  };
  if (!coop_shared) return launch();
  // the gate alone: no other concurrent solve submits until this kernel has
  // finished, and the device is drained first, so that every workgroup of
  // the kernel is placed at once on an otherwise idle device
  std::unique_lock<std::shared_mutex> lk(launch_gate);
  HSDM_TRY(hipDeviceSynchronize());
  HSDM_TRY(launch());
  return hipStreamSynchronize(s);
}
