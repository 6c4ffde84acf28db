// Density matrix p_ij = sum_l f_l c_il c_jl (Eq. 4) and energy-weighted
// density matrix q_ij = sum_l eps_l f_l c_il c_jl (Eq. 17) in one pass.
//
// Both are symmetric rank-m products of the same n x m eigenvector block C,
// so one kernel computes the lower-triangular 64x64 tiles of both: the A
// operand (rows of C) is staged once, the B operand (rows of C again) is
// staged twice in LDS, scaled by f_l and by f_l eps_l on the way in, and two
// sets of FP64 MFMA accumulators are kept per wavefront.  A tiled transpose
// then completes the upper triangles.  m can be read from device memory (the
// number of occupied states is only known on the device).
#include "hsdm_internal.h"
#include "hsdm_util.h"

namespace {

constexpr int NT = 256, BT = 64, BK = 16, LD = BT + 16;

__global__ __launch_bounds__(NT, 2) void dm_kernel(int n, int m_host, const int* m_dev,
                                                const double* C, long ldc, const double* f,
                                                const double* eps, double* D, long ldd,
                                                double* E, long lde) {
  const int tm = blockIdx.x, tn = blockIdx.y;
  if (tm < tn) return;
  const int m = m_dev ? *m_dev : m_host;
  __shared__ double As[2][BK * LD];
  __shared__ double Bd[2][BK * LD];
  __shared__ double Be[2][BK * LD];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int i0 = tm * BT, j0 = tn * BT;
  const bool want_e = (E != nullptr);

  dbl4 accd[2][2], acce[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) {
      accd[a][b] = dbl4{0, 0, 0, 0};
      acce[a][b] = dbl4{0, 0, 0, 0};
    }
  // staging: thread t moves rows (t % 64) of the 64 x 16 slices, columns t/64 + 4q
  double ra[4], rb[4], sf[4], se[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int kk = k0 + t / BT + 4 * q;
      const int i = i0 + (t % BT), j = j0 + (t % BT);
      const bool kin = kk < m;
      ra[q] = (kin && i < n) ? C[i + (long)kk * ldc] : 0.0;
      rb[q] = (kin && j < n) ? C[j + (long)kk * ldc] : 0.0;
      const double fk = kin ? f[kk] : 0.0;
      sf[q] = fk;
      se[q] = kin ? fk * eps[kk] : 0.0;
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int r = t / BT + 4 * q, c = t % BT;
      As[b][r * LD + c] = ra[q];
      Bd[b][r * LD + c] = rb[q] * sf[q];
      Be[b][r * LD + c] = rb[q] * se[q];
    }
  };
  int buf = 0;
  if (m > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int k0 = 0; k0 < m; k0 += BK) {
    const bool more = k0 + BK < m;
    if (more) load(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4);
      double fa[2], fd[2], fe[2];
#pragma unroll
      for (int a = 0; a < 2; a++) fa[a] = As[buf][kr * LD + wm * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; b++) {
        fd[b] = Bd[buf][kr * LD + wn * 32 + b * 16 + (lane & 15)];
        fe[b] = Be[buf][kr * LD + wn * 32 + b * 16 + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) {
          accd[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fd[b], accd[a][b], 0, 0, 0);
          if (want_e)
            acce[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fe[b], acce[a][b], 0, 0, 0);
        }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) {
      const int col = j0 + wn * 32 + b * 16 + (lane & 15);
      if (col >= n) continue;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = i0 + wm * 32 + a * 16 + (lane >> 4) + 4 * r;
        if (row >= n || row < col) continue;
        D[row + (long)col * ldd] = accd[a][b][r];
        if (want_e) E[row + (long)col * lde] = acce[a][b][r];
      }
    }
}

}  // namespace

hipError_t density_launch(int n, int m, const double* C, long ldc, const double* f,
                          const double* eps, double* D, long ldd, double* E, long lde,
                          const int* m_dev, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nt = ceil_div(n, BT);
  // algorithmic: lower triangles of D (and E), n (n + 1) m flops each
  kt_begin("dm_kernel", (E ? 2.0 : 1.0) * n * (n + 1.0) * m, 0.0, m_dev ? m : 0, s);
  hipLaunchKernelGGL(dm_kernel, dim3(nt, nt), dim3(NT), 0, s, n, m, m_dev, C, ldc, f, eps, D, ldd,
                     E, lde);
  kt_end(s);
  HSDM_TRY(hipGetLastError());
  HSDM_TRY(dev_mirror_lower(D, ldd, n, s));
  if (E) HSDM_TRY(dev_mirror_lower(E, lde, n, s));
  return hipSuccess;
}
