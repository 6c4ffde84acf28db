// Density matrix p_ij = sum_l f_l c_il c_jl (Eq. 4) and energy-weighted
// density matrix q_ij = sum_l eps_l f_l c_il c_jl (Eq. 17) in one pass.
//
// Both are symmetric rank-m products of the same n x m eigenvector block C,
// so one kernel computes the lower-triangular 128 x 128 tiles of both: a
// workgroup of 16 wavefronts stages the A operand (rows of C) once and the B
// operand (rows of C again) twice in LDS, scaled by f_l and by f_l eps_l on
// the way in; wavefronts 0-7 accumulate the tile of D, 8-15 the tile of E
// (64 x 32 each).  A tiled transpose then completes the upper triangles.  m
// can be read from device memory (the number of occupied states is only
// known on the device).
#include "hsdm_internal.h"
#include "hsdm_util.h"

namespace {

constexpr int NT = 1024, BT = 128, BK = 16, LD = BT + 16;

__global__ __launch_bounds__(NT) void dm_kernel(int n, int m_host, const int* m_dev,
                                                const double* C, long ldc, const double* f,
                                                const double* eps, double* D, long ldd,
                                                double* E, long lde) {
  const int tm = blockIdx.x, tn = blockIdx.y;
  if (tm < tn) return;
  const int m = m_dev ? *m_dev : m_host;
  __shared__ double As[2][BK * LD];
  __shared__ double Bs[2][2][BK * LD];  // [buffer][D or E]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int which = wave >> 3;           // 0: D, 1: E
  const int wm = wave & 1, wn = (wave >> 1) & 3;
  const int i0 = tm * BT, j0 = tn * BT;
  const bool active = (which == 0) || (E != nullptr);

  dbl4 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = dbl4{0, 0, 0, 0};
  // staging: thread t moves row t % 128 of the 128 x 16 slices, columns t / 128 and t / 128 + 8
  double ra[2], rb[2], sf[2], se[2];
  // a tile wholly inside C stages its full slices from workgroup-uniform
  // bases plus fixed per-thread byte offsets (no per-slice address arithmetic)
  const bool whole = (i0 + BT <= n) && (j0 + BT <= n) && (ldc < (1L << 22));
  const unsigned off = (unsigned)(sizeof(double) * ((t % BT) + (long)(t / BT) * ldc));
  const long qstride = (long)sizeof(double) * 8 * ldc;
  auto load = [&](int k0) {
    if (whole && k0 + BK <= m) {
      const char* ca = (const char*)(C + i0 + (long)k0 * ldc);
      const char* cb = (const char*)(C + j0 + (long)k0 * ldc);
#pragma unroll
      for (int q = 0; q < 2; q++) {
        ra[q] = *(const double*)(ca + q * qstride + off);
        rb[q] = *(const double*)(cb + q * qstride + off);
        const int kk = k0 + t / BT + 8 * q;
        const double fk = f[kk];
        sf[q] = fk;
        se[q] = fk * eps[kk];
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const int kk = k0 + t / BT + 8 * q;
      const int i = i0 + (t % BT), j = j0 + (t % BT);
      const bool kin = kk < m;
      const int kc = kin ? kk : 0;
      const double va = C[min(i, n - 1) + (long)kc * ldc];
      const double vb = C[min(j, n - 1) + (long)kc * ldc];
      ra[q] = (kin && i < n) ? va : 0.0;
      rb[q] = (kin && j < n) ? vb : 0.0;
      const double fk = f[kc], ek = eps[kc];
      sf[q] = kin ? fk : 0.0;
      se[q] = kin ? fk * ek : 0.0;
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const int r = t / BT + 8 * q, c = t % BT;
      As[b][r * LD + c] = ra[q];
      Bs[b][0][r * LD + c] = rb[q] * sf[q];
      Bs[b][1][r * LD + c] = rb[q] * se[q];
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
    if (active) {
      const double* as = As[buf];
      const double* bs = Bs[buf][which];
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        const int kr = ks + (lane >> 4);
        double fa[4], fb[2];
#pragma unroll
        for (int a = 0; a < 4; a++) fa[a] = as[kr * LD + wm * 64 + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 2; b++) fb[b] = bs[kr * LD + wn * 32 + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
          for (int b = 0; b < 2; b++)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
      }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (!active) return;
  double* out = which ? E : D;
  const long ldo = which ? lde : ldd;
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) {
      const int col = j0 + wn * 32 + b * 16 + (lane & 15);
      if (col >= n) continue;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = i0 + wm * 64 + a * 16 + (lane >> 4) + 4 * r;
        if (row >= n || row < col) continue;
        out[row + (long)col * ldo] = acc[a][b][r];
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
  kt_begin("dm_kernel", (E ? 2.0 : 1.0) * n * (n + 1.0) * m, 0.0, m_dev ? m : 0, s, true);
  HSDM_LAUNCH(dm_kernel, dim3(nt, nt), dim3(NT), 0, s, n, m, m_dev, C, ldc, f, eps, D, ldd,
                     E, lde);
  kt_end(s);
  HSDM_TRY(hipGetLastError());
  HSDM_TRY(dev_mirror_lower(D, ldd, n, s));
  if (E) HSDM_TRY(dev_mirror_lower(E, lde, n, s));
  return hipSuccess;
}
