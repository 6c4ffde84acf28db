// Back-transformation of eigenvectors through the two reduction stages.
//
// Stage 2 (bulge chasing): the reflectors H_{s,t} of B consecutive sweeps
// that share the task index t are combined into one block reflector
// G = I - V T V^T (V: 2B x B parallelogram, T: B x B upper triangular), so
// that applying them is three small matrix products on the FP64 matrix
// cores.  Ordering: Q2 Z = H_{0,0} H_{0,1} ... Z must apply later sweeps
// first; group (b, t) (sweep block b) overlaps groups (b+1, t-2 .. t) and
// (b, t-1), so all groups with equal  t + 2 (nblk - 1 - b)  are independent
// and one launch per such level applies them, each workgroup one group to
// one slab of 64 columns of Z.
//
// Stage 1 (panels): Z <- (I - V_p T_p V_p^T) Z for p from the last panel to
// the first, as three GEMMs per panel (the tall V_p^T Z with split-K).
#include "hsdm_internal.h"
#include "hsdm_phases.h"

namespace {

constexpr int B = 32;
constexpr int H2 = 2 * B;  // rows of a group

// T factor of every group: T_jj = tau_j, T(0:j, j) = -tau_j T(0:j,0:j) V^T v_j
__global__ __launch_bounds__(256) void group_t_kernel(const double* V2, const double* tau2,
                                                      double* T2) {
  const long gi = blockIdx.x;
  const double* V = V2 + gi * H2 * B;
  const double* tau = tau2 + gi * B;
  __shared__ double Vs[H2][B + 1];
  __shared__ double Gm[B][B + 1];
  __shared__ double Tl[B][B + 1];
  const int t = threadIdx.x;
  for (int e = t; e < H2 * B; e += 256) Vs[e % H2][e / H2] = V[e];
  __syncthreads();
  for (int e = t; e < B * B; e += 256) {
    const int a = e % B, b = e / B;
    double s = 0.0;
    if (a < b)
      for (int r = 0; r < H2; r++) s += Vs[r][a] * Vs[r][b];
    Gm[a][b] = s;
    Tl[a][b] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < B; j++) {
    const double tj = tau[j];
    if (t < j) {
      double s = 0.0;
      for (int k = t; k < j; k++) s += Tl[t][k] * Gm[k][j];
      Tl[t][j] = -tj * s;
    }
    if (t == j) Tl[j][j] = tj;
    __syncthreads();
  }
  double* T = T2 + gi * B * B;
  for (int e = t; e < B * B; e += 256) T[e] = Tl[e % B][e / B];
}

// Apply the groups of one level to Z: workgroup (group, slab of 128 columns),
// 8 wavefronts.  Z block (2B x 128) and W (B x 128) live in LDS; V and T are
// read from L2.  Zero 16x16 blocks of the parallelogram V are skipped:
// V(r, c) != 0 only for c <= r <= c + B - 1.
constexpr int SWA = 128;

__global__ __launch_bounds__(512) void group_apply_kernel(int n, int nblk, int level, int sb_lo,
                                                          const double* V2, const double* T2,
                                                          const long* goff, double* Z, long ldz,
                                                          int m_host, const int* m_dev) {
  const int sb = sb_lo + blockIdx.x;
  const int t = level - 2 * (nblk - 1 - sb);
  const int tg = (n - 1 - sb * B + B - 1) / B;
  if (t < 0 || t >= tg) return;
  const int m = m_dev ? *m_dev : m_host;
  const int c0 = blockIdx.y * SWA;
  if (c0 >= m) return;
  const int nc = min(SWA, m - c0);
  const int rb = sb * B + 1 + t * B;
  const int hh = min(H2, n - rb);
  const long gi = goff[sb] + t;
  const double* V = V2 + gi * H2 * B;   // (H2 x B), column-major
  const double* T = T2 + gi * B * B;    // (B x B), column-major

  __shared__ double Zs[H2][SWA + 1];
  __shared__ double Ws[B][SWA + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int a = w & 1, cb0 = 2 * (w >> 1);
  const int rr = w & 3, cb = 4 * (w >> 2);
  // all V and T operand fragments of this lane, loaded up front so that their
  // latency overlaps the Z block load
  double v1[12], t2[8], v3[8];
#pragma unroll
  for (int q = 0; q < 12; q++) v1[q] = V[(16 * a + 4 * q + l4) + (long)(16 * a + l16) * H2];
#pragma unroll
  for (int q = 0; q < 8; q++) {
    const int k0 = 4 * q;
    t2[q] = (k0 >= 16 * a) ? T[(16 * a + l16) + (long)(k0 + l4) * B] : 0.0;
    v3[q] = -V[(16 * rr + l16) + (long)(k0 + l4) * H2];
  }
  for (int e = tid; e < H2 * SWA; e += 512) {
    const int r = e % H2, c = e / H2;
    Zs[r][c] = (r < hh && c < nc) ? Z[rb + r + (long)(c0 + c) * ldz] : 0.0;
  }
  __syncthreads();
  // phase 1: W = V^T Zs (B x SWA); wave w: row block a = w & 1, column blocks 2(w>>1) + {0,1}
  // (column block a of V is nonzero in rows 16a .. 16a+47 only)
  {
    dbl4 acc0 = dbl4{0, 0, 0, 0}, acc1 = dbl4{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 12; q++) {
      const int k0 = 16 * a + 4 * q;
      const double fa = v1[q];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, Zs[k0 + l4][16 * cb0 + l16], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, Zs[k0 + l4][16 * cb0 + 16 + l16], acc1, 0, 0,
                                                  0);
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
      Ws[16 * a + l4 + 4 * r][16 * cb0 + l16] = acc0[r];
      Ws[16 * a + l4 + 4 * r][16 * cb0 + 16 + l16] = acc1[r];
    }
  }
  __syncthreads();
  // phase 2: W2 = T W (T upper triangular), same block mapping
  {
    dbl4 acc0 = dbl4{0, 0, 0, 0}, acc1 = dbl4{0, 0, 0, 0};
#pragma unroll
    for (int q = 4 * a; q < 8; q++) {
      const int k0 = 4 * q;
      const double fa = t2[q];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, Ws[k0 + l4][16 * cb0 + l16], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, Ws[k0 + l4][16 * cb0 + 16 + l16], acc1, 0, 0,
                                                  0);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; r++) {
      Ws[16 * a + l4 + 4 * r][16 * cb0 + l16] = acc0[r];
      Ws[16 * a + l4 + 4 * r][16 * cb0 + 16 + l16] = acc1[r];
    }
  }
  __syncthreads();
  // phase 3: Zs - V W2; wave w: row block rr = w & 3, column blocks 4(w>>2) + {0..3}
  {
    const int qbeg = (rr == 3) ? 4 : 0, qend = (rr == 0) ? 4 : 8;
    dbl4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
      for (int r = 0; r < 4; r++) acc[q][r] = Zs[16 * rr + l4 + 4 * r][16 * (cb + q) + l16];
#pragma unroll
    for (int kq = 0; kq < 8; kq++) {
      if (kq < qbeg || kq >= qend) continue;
      const int k0 = 4 * kq;
      const double fa = v3[kq];
#pragma unroll
      for (int q = 0; q < 4; q++)
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, Ws[k0 + l4][16 * (cb + q) + l16], acc[q],
                                                      0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int c = 16 * (cb + q) + l16;
      if (c >= nc) continue;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = 16 * rr + l4 + 4 * r;
        if (row < hh) Z[rb + row + (long)(c0 + c) * ldz] = acc[q][r];
      }
    }
  }
}

}  // namespace

hipError_t bt2_prepare(const Sb2stLayout& L, const double* V2, const double* tau2, double* T2,
                       const long* d_goff, hipStream_t s) {
  (void)d_goff;
  if (L.ngroups <= 0) return hipSuccess;
  hipLaunchKernelGGL(group_t_kernel, dim3((unsigned)L.ngroups), dim3(256), 0, s, V2, tau2, T2);
  return hipGetLastError();
}

hipError_t bt2_apply(const Sb2stLayout& L, const double* V2, const double* T2, const long* d_goff,
                     double* Z, long ldz, int m, const int* m_dev, hipStream_t s) {
  if (L.ngroups <= 0 || m <= 0) return hipSuccess;
  const int n = L.n, nblk = L.nblk;
  const int nslab = ceil_div(m, SWA);
  auto tg = [&](int sb) { return (n - 1 - sb * B + B - 1) / B; };
  const int lmax = (tg(0) - 1) + 2 * (nblk - 1);
  for (int level = 0; level <= lmax; level++) {
    int lo = nblk - 1 - level / 2;
    if (lo < 0) lo = 0;
    int hi = -1;  // largest sb with a valid task at this level
    for (int sb = nblk - 1; sb >= lo; sb--) {
      const int t = level - 2 * (nblk - 1 - sb);
      if (t >= 0 && t < tg(sb)) {
        hi = sb;
        break;
      }
    }
    if (hi < 0) continue;
    int first = hi;
    while (first - 1 >= lo) {
      const int t = level - 2 * (nblk - 1 - (first - 1));
      if (t < 0 || t >= tg(first - 1)) break;
      first--;
    }
    hipLaunchKernelGGL(group_apply_kernel, dim3(hi - first + 1, nslab), dim3(512), 0, s, n, nblk,
                       level, first, V2, T2, d_goff, Z, ldz, m, m_dev);
    HSDM_TRY(hipGetLastError());
  }
  return hipSuccess;
}

namespace {

// ---- stage 1 ------------------------------------------------------------------
// GP consecutive panels form one block reflector of width GP*B:
//   (I - V1 T1 V1^T)(I - V2 T2 V2^T) = I - [V1 V2] [[T1, -T1 V1^T V2 T2], [0, T2]] [V1 V2]^T
// applied panel group by panel group, last group first.  The explicit panel
// reflectors are zero above their first row, so the grouped V is dense with a
// staircase of zeros.
constexpr int GP = 4;

// T of one panel group from the per-panel T's and the Gram G = V^T V (ld W).
__global__ __launch_bounds__(256) void group_t1_kernel(int np, int Bp, const double* T1p,
                                                       const double* Gm, double* Tq) {
  const int W = np * Bp;
  __shared__ double X[3 * 32 * 32];  // (i*Bp) x Bp block, i <= 3, Bp <= 32
  const int t = threadIdx.x;
  for (int e = t; e < W * W; e += 256) {
    const int r = e % W, c = e / W;
    const int pr = r / Bp, pc = c / Bp;
    Tq[r + (long)c * W] = (pr == pc) ? T1p[(size_t)pr * Bp * Bp + (r % Bp) + (c % Bp) * Bp] : 0.0;
  }
  __syncthreads();
  for (int i = 1; i < np; i++) {
    const int rows = i * Bp;
    const double* Ti = T1p + (size_t)i * Bp * Bp;
    // X = G[0:rows, iBp:(i+1)Bp] * T_i
    for (int e = t; e < rows * Bp; e += 256) {
      const int r = e % rows, c = e / rows;
      double acc = 0.0;
      for (int q = 0; q <= c; q++) acc += Gm[r + (long)(rows + q) * W] * Ti[q + c * Bp];
      X[r + c * rows] = acc;
    }
    __syncthreads();
    // Tq[0:rows, block] = -Tq[0:rows, 0:rows] * X  (Tq upper triangular)
    for (int e = t; e < rows * Bp; e += 256) {
      const int r = e % rows, c = e / rows;
      double acc = 0.0;
      for (int q = r; q < rows; q++) acc += Tq[r + (long)q * W] * X[q + c * rows];
      Tq[r + (long)(rows + c) * W] = -acc;
    }
    __syncthreads();
  }
}

__global__ void zero_upper_panels_kernel(int n, int B_, double* Vst, long ldv) {
  // rows above each panel's first reflector row: Vst[0 : (p+1)B, pB : (p+1)B] = 0
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = (int)(idx / n), r = (int)(idx % n);
  if (c >= n) return;
  const int p = c / B_;
  if (r < (p + 1) * B_) Vst[r + (long)c * ldv] = 0.0;
}

}  // namespace

static int npanel_of(int n, int B_) { return (n > B_) ? ceil_div(n - 1, B_) : 0; }

size_t bt1_scratch_doubles(int n, int B_, int m) {
  const size_t W = (size_t)GP * B_;
  const size_t nsplit = ceil_div(n, 1024) + 1;
  const size_t ngroup = ceil_div(npanel_of(n, B_), GP) + 1;
  // W, W2 (W x m), split-K partials (nsplit x W x m), Gram + partials, T of each group
  return W * m * (2 + nsplit) + W * W * (1 + nsplit) + ngroup * W * W + 64;
}

hipError_t bt1_zero_fill(int n, int B_, double* Vst, long ldv, hipStream_t s) {
  const long tot = (long)n * n;
  hipLaunchKernelGGL(zero_upper_panels_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     s, n, B_, Vst, ldv);
  return hipGetLastError();
}

hipError_t bt1_apply(int n, int B_, const double* Vst, long ldv, const double* T1, double* Z,
                     long ldz, int m, const int* m_dev, double* scratch, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int np_all = npanel_of(n, B_);
  if (np_all == 0) return hipSuccess;
  const int W = GP * B_;
  const size_t nsplit = ceil_div(n, 1024) + 1;
  double* Wb = scratch;
  double* W2 = Wb + (size_t)W * m;
  double* part = W2 + (size_t)W * m;
  double* Gm = part + nsplit * W * m;
  double* Gpart = Gm + (size_t)W * W;
  double* Tall = Gpart + nsplit * W * W;
  const int ngroup = ceil_div(np_all, GP);
  // T factors of the panel groups
  for (int q = 0; q < ngroup; q++) {
    const int p0 = q * GP, np = min(GP, np_all - p0);
    const int r0 = (p0 + 1) * B_, h = n - r0, w = np * B_;
    const double* Vq = Vst + r0 + (long)p0 * B_ * ldv;
    double* Tq = Tall + (size_t)q * W * W;
    if (np > 1) {
      GemmArgs g{};
      g.m = w; g.n = w; g.k = h; g.A = Vq; g.lda = ldv; g.B = Vq; g.ldb = ldv; g.C = Gm; g.ldc = w;
      g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0;
      HSDM_TRY(gemm_splitk_launch(g, 1024, Gpart, s));
    }
    hipLaunchKernelGGL(group_t1_kernel, dim3(1), dim3(256), 0, s, np, B_,
                       T1 + (size_t)p0 * B_ * B_, Gm, Tq);
    HSDM_TRY(hipGetLastError());
  }
  for (int q = ngroup - 1; q >= 0; q--) {
    const int p0 = q * GP, np = min(GP, np_all - p0);
    const int r0 = (p0 + 1) * B_, h = n - r0, w = np * B_;
    if (h <= 0) continue;
    const double* Vq = Vst + r0 + (long)p0 * B_ * ldv;
    const double* Tq = Tall + (size_t)q * W * W;
    double* Zq = Z + r0;
    GemmArgs g{};
    g.m = w; g.n = m; g.k = h; g.A = Vq; g.lda = ldv; g.B = Zq; g.ldb = ldz; g.C = Wb; g.ldc = w;
    g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0; g.ndev = m_dev;
    HSDM_TRY(gemm_splitk_launch(g, 1024, part, s));
    g = GemmArgs{};
    g.m = w; g.n = m; g.k = w; g.A = Tq; g.lda = w; g.B = Wb; g.ldb = w; g.C = W2; g.ldc = w;
    g.alpha = 1.0; g.beta = 0.0; g.flags = GF_KA_UPPER; g.ndev = m_dev;
    HSDM_TRY(gemm_launch(g, s));
    g = GemmArgs{};
    g.m = h; g.n = m; g.k = w; g.A = Vq; g.lda = ldv; g.B = W2; g.ldb = w; g.C = Zq; g.ldc = ldz;
    g.alpha = -1.0; g.beta = 1.0; g.ndev = m_dev;
    HSDM_TRY(gemm_launch(g, s));
  }
  return hipSuccess;
}
