// Stage 1 of the two-stage tridiagonalization: full symmetric -> band of
// half-bandwidth B (the paper's GPU outlook names the two-stage reduction as
// the part that exposes matrix-matrix work).
//
// For panel p (columns c0 = pB .. c0+B-1, rows r0 = c0+B .. n-1, h = n-r0):
//  1. Householder QR of the h x B panel.  One cooperative launch; workgroup g
//     keeps rows [256g, 256g+256) of the panel in LDS.  Per column a single
//     grid-wide exchange of partial sums is enough: every workgroup
//     contributes sum_i x_i^2 and sum_i x_i a_ic (rows below the pivot) and
//     derives the reflector and the update coefficients locally, in the same
//     fixed reduction order (bitwise reproducible).  The block reflector
//     Q = I - V T V^T (T upper triangular) is formed in the same launch.
//  2. Two-sided update of the trailing block A22 <- Q^T A22 Q, with only the
//     lower triangle of A22 stored:
//        Y = V T,  X = A22 Y (symmetric operand),  M = Y^T X,
//        W = X - V M / 2,  A22 <- A22 - [V W][W V]^T (lower tiles).
//     Both large products run on the FP64 MFMA GEMM.
// After the last panel the band (diagonal blocks and the R factors) is
// copied into band storage for the bulge-chasing stage.
#include <algorithm>
#include <tuple>

#include "hsdm_internal.h"
#include "hsdm_phases.h"
#include "hsdm_util.h"

namespace {

constexpr int NT = 256;
constexpr int CH = 256;      // panel rows per workgroup
constexpr int ACH = 128;     // rows per workgroup of the tall U^T W products
constexpr int SPLITK = 512;  // K slice of the symmetric product X = A22 Y
constexpr int PGROUP = 4;    // panels per trailing update in a single reduction

template <int CTRL>
HSDM_DEV double dpp_mov(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <int PAT>
HSDM_DEV double swizzle(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)u, PAT);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(unsigned)(u >> 32), PAT);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// value of the partner lane (lane ^ 2^S): quad permutations for S = 0, 1,
// swizzles in bit-mask mode for S = 2, 3, 4, a shuffle for S = 5
template <int S>
HSDM_DEV double xchg(double v) {
  if constexpr (S == 0) return dpp_mov<0xB1>(v);             // quad_perm [1,0,3,2]
  else if constexpr (S == 1) return dpp_mov<0x4E>(v);        // quad_perm [2,3,0,1]
  else if constexpr (S <= 4) return swizzle<0x1F | ((1 << S) << 10)>(v);
  else return __shfl_xor(v, 32, 64);
}

template <int S, int NV>
HSDM_DEV void halve(double (&v)[NV], bool hi) {
  constexpr int half = 16 >> S;
#pragma unroll
  for (int k = 0; k < half; k++) {
    const double send = hi ? v[k] : v[half + k];
    const double keep = hi ? v[half + k] : v[k];
    v[k] = keep + xchg<S>(send);
  }
}

// Sum of v[0..31] over the 64 lanes of a wavefront by recursive halving:
// after the exchange with lane ^ 2^S a lane keeps the half of its values
// selected by that lane bit (cheapest exchanges first, for the largest
// halves).  Lane l ends with the sum for index bitrev5(l & 31) (see
// rs_index) over the 32 lanes sharing bit 5; the exchange with lane ^ 32
// completes it over all 64 lanes.
template <int NV>
HSDM_DEV double wave_reduce_scatter(double (&v)[NV]) {
  static_assert(NV == 32, "32 values over 64 lanes");
  const int lane = threadIdx.x & 63;
  halve<0>(v, (lane & 1) != 0);
  halve<1>(v, (lane & 2) != 0);
  halve<2>(v, (lane & 4) != 0);
  halve<3>(v, (lane & 8) != 0);
  halve<4>(v, (lane & 16) != 0);
  return v[0] + xchg<5>(v[0]);
}

// index of the value lane l holds after wave_reduce_scatter
HSDM_DEV int rs_index(int lane) {
  return ((lane & 1) << 4) | ((lane & 2) << 2) | (lane & 4) | ((lane & 8) >> 2) |
         ((lane & 16) >> 4);
}

// Exchange between the workgroups of a panel without a barrier: every slot
// of the exchange buffers holds a NaN before the launch; a workgroup writes
// its values with agent-scope atomic stores (coherent at agent scope without
// cache maintenance), and a reader polls each slot with agent-scope atomic
// loads until it is no longer NaN (sums of finite values never are).
HSDM_DEV void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

HSDM_DEV double ld_ready(const double* p, DevStatusWord* st) {
  double v = __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  long spins = 0;
  while (v != v) {
    if (++spins > (1L << 24) ||
        ((spins & 1023) == 0 &&
         __hip_atomic_load(&st->code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
      dev_set_status(st, DS_SYNC_TIMEOUT, 1);
      return 0.0;
    }
    __builtin_amdgcn_s_sleep(1);
    v = __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return v;
}

HSDM_DEV double ld_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// s + p[q0 stride] + p[(q0 + dq) stride] + ... (q < G, added in that order),
// each slot polled until it is written.  The CHK slots of a chunk are loaded
// together and only the unwritten ones again, so that a chunk whose slots
// are all written costs one round trip to the memory side, not CHK.
template <int CHK>
HSDM_DEV double sum_ready(const double* p, long stride, int q0, int dq, int G, double s,
                          DevStatusWord* st) {
  for (int qb = q0; qb < G; qb += CHK * dq) {
    double v[CHK];
#pragma unroll
    for (int i = 0; i < CHK; i++) {
      const int q = qb + i * dq;
      v[i] = (q < G) ? ld_agent(p + (long)q * stride) : 0.0;
    }
    long spins = 0;
    for (;;) {
      bool pend = false;
#pragma unroll
      for (int i = 0; i < CHK; i++) pend |= (v[i] != v[i]);
      if (!pend) break;
      if (++spins > (1L << 24) ||
          ((spins & 1023) == 0 &&
           __hip_atomic_load(&st->code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
        dev_set_status(st, DS_SYNC_TIMEOUT, 1);
        return s;
      }
      __builtin_amdgcn_s_sleep(1);
#pragma unroll
      for (int i = 0; i < CHK; i++)
        if (v[i] != v[i]) v[i] = ld_agent(p + (long)(qb + i * dq) * stride);
    }
#pragma unroll
    for (int i = 0; i < CHK; i++)
      if (qb + i * dq < G) s += v[i];
  }
  return s;
}

// The arithmetic both panel kernels share (the fused one and the per-column
// launches), with every multiply-add written out so that the compiler has
// no choice of contraction and the two give the same bits.
struct Reflector {
  double tau, beta, scal;
};

// reflector of column j from sigma = sum of squares below the pivot and
// the pivot alpha: beta = -sign(alpha) sqrt(alpha^2 + sigma),
// tau = (beta - alpha) / beta, v_i = a_ij / (alpha - beta)
HSDM_DEV Reflector make_reflector(double sigma, double alpha) {
  Reflector r{0.0, alpha, 0.0};
  if (sigma > 0.0) {
    const double nrm = sqrt(fma(alpha, alpha, sigma));
    r.beta = (alpha >= 0.0) ? -nrm : nrm;
    r.tau = (r.beta - alpha) / r.beta;
    r.scal = 1.0 / (alpha - r.beta);
  }
  return r;
}

// w_k = tau (a_j,j+k + v^T a_:,j+k) for the pivot row value and the sum below it
HSDM_DEV double reflector_w(const Reflector& r, double row, double dd) {
  return r.tau * fma(dd, r.scal, row);
}

// one row's columns j .. j+B-1 (a[0] = column j) after reflector j: below
// the pivot a_i,j+k -= v_i w_k and a_ij becomes v_i; the pivot row gets
// a_j,j+k -= w_k and beta
template <int B>
HSDM_DEV void reflector_apply(double (&a)[B], bool below, bool piv, const Reflector& r,
                              const double* wl) {
  if (below) {
    const double vi = a[0] * r.scal;
#pragma unroll
    for (int k = 1; k < B; k++) a[k] = fma(-vi, wl[k], a[k]);
    a[0] = vi;
  } else if (piv) {
#pragma unroll
    for (int k = 1; k < B; k++) a[k] -= wl[k];
    a[0] = r.beta;
  }
}

// entry (ca, cb) of V^T V over nrows rows of V held in LDS (zero below the
// diagonal of the Gram matrix)
template <int B>
HSDM_DEV double gram_entry(const double (*Pl)[B + 1], int nrows, int ca, int cb) {
  double sum = 0.0;
  if (ca <= cb)
    for (int i = 0; i < nrows; i++) sum = fma(Pl[i][ca], Pl[i][cb], sum);
  return sum;
}

// T (upper triangular, in LDS) from the Gram matrix and the scalars:
// T_jj = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) (V^T v_j)(0:j).
// Thread t forms row t of T and reads only entries of row t it wrote itself
// at earlier steps (T(t, k), t <= k < j), so the steps need no barrier
// between them.
template <int B>
HSDM_DEV void form_t(double (*Tl)[B + 1], const double (*Gm)[B + 1], const double* taul) {
  const int t = threadIdx.x;
  if (t < B) {
    for (int j = 0; j < B; j++) {
      if (t < j) {
        double sum = 0.0;
        for (int k = t; k < j; k++) sum = fma(Tl[t][k], Gm[k][j], sum);
        Tl[t][j] = -taul[j] * sum;
      }
      if (t == j) Tl[j][j] = taul[j];
    }
  }
  __syncthreads();
}

// The three h x B copies that file a panel's V and W for the group's
// held-back updates, in one launch: dv1 = V, dw = W, dv2 = V (ld ldd).
template <class T>
__global__ void file_vw_kernel(int h, int B, const T* V, long ldv, const T* W, long ldw,
                               T* dv1, T* dw, T* dv2, long ldd) {
  const long tot = (long)h * B;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % h), c = (int)(e / h);
    const T v = V[i + (long)c * ldv];
    dv1[i + (long)c * ldd] = v;
    dv2[i + (long)c * ldd] = v;
    dw[i + (long)c * ldd] = W[i + (long)c * ldw];
  }
}

template <class T>
hipError_t file_vw(int h, int B, const T* V, long ldv, const T* W, long ldw, T* dv1, T* dw,
                   T* dv2, long ldd, hipStream_t s) {
  if (h <= 0) return hipSuccess;
  const long tot = (long)h * B;
  const unsigned g = (unsigned)std::min<long>((tot + 255) / 256, 4096);
  HSDM_LAUNCH(file_vw_kernel<T>, dim3(g), dim3(256), 0, s, h, B, V, ldv, W, ldw, dv1, dw, dv2,
              ldd);
  return hipGetLastError();
}

__global__ void fill_nan_kernel(double* p, long cnt) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = __builtin_nan("");
}

// Householder QR of the h x B panel P (ldp); V receives the explicit unit
// lower trapezoidal reflectors, tau the scalars, Tt the B x B triangular
// factor (column-major, ld B).  part, prow, gpart are scratch.
// Workgroup g holds rows [256 g, 256 g + 256) of the panel, one row per
// thread in registers; the column sums of each step are reduced inside the
// wavefronts by shuffles, across the 4 wavefronts through LDS and across
// the workgroups through the exchange slots of global memory.
template <int B>
HSDM_DEV void panel_qr_body(int h, double* P, long ldp, double* V, long ldv, double* tau_out,
                            double* Tt, double* part, double* prow, double* gpart,
                            DevStatusWord* st, int g, int G) {
  static_assert(NT == CH && B == 32, "one row per thread, 32 columns");
  constexpr int NW = NT / 64;
  constexpr int RG = NT / B;  // threads per column when combining partial sums
  __shared__ double red[NW][B];
  __shared__ double ddl[B], wl[B], taul[B], rowl[B];
  __shared__ double Pl[CH][B + 1];
  __shared__ double Gm[B][B + 1], Tl[B][B + 1];
  __shared__ double cmb[RG][B + 1];

  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int row0 = g * CH;
  const int nrows = min(CH, h - row0);
  const int gi = row0 + t;
  const bool rok = t < nrows;
  // a[k] holds column j + k of this thread's row during step j: the array
  // shifts down by one column per step, so every index below is static and
  // finished columns go to Pl[t][j]
  double a[B];
#pragma unroll
  for (int c = 0; c < B; c++) a[c] = rok ? P[gi + (long)c * ldp] : 0.0;

  const int ncol = min(B, h);
  for (int j = 0; j < B; j++) {
    const bool below = rok && gi > j;  // rows strictly below the pivot
    const bool piv = rok && gi == j;   // the pivot row (in workgroup 0)
    if (j < ncol) {
      // partial sums over this workgroup's rows below the pivot:
      // sum_i a_ij a_i,j+k for k = 0 .. B-1-j
      const double aj = a[0];
      double v[B];
#pragma unroll
      for (int k = 0; k < B; k++) v[k] = below ? aj * a[k] : 0.0;
      const double ws = wave_reduce_scatter(v);
      if (lane < 32) red[wv][rs_index(lane)] = ws;
      if (g == 0 && piv) {
#pragma unroll
        for (int k = 0; k < B; k++) rowl[k] = a[k];
      }
      __syncthreads();
      if (G == 1) {
        // single workgroup: the sums and the pivot row are already in LDS
        if (t < B) {
          double sum = 0.0;
#pragma unroll
          for (int w = 0; w < NW; w++) sum += red[w][t];
          ddl[t] = sum;
        }
      } else {
        double* pb = part + (size_t)j * G * B;  // this column's slots (NaN before)
        double* rb = prow + (size_t)j * B;
        double rv = 0.0;
        if (t < B) {
          double sum = 0.0;
#pragma unroll
          for (int w = 0; w < NW; w++) sum += red[w][t];
          st_agent(&pb[(size_t)g * B + t], sum);
          if (g == 0) st_agent(&rb[t], rowl[t]);
          rv = ld_agent(&rb[t]);  // in flight with the partial sums below
        }
        {
          // RG threads per column sum strided subsets, then a fixed-order combine
          const int k = t % B, rg = t / B;
          double s2 = 0.0;
          if (k < B - j) s2 = sum_ready<8>(pb + k, B, rg, RG, G, 0.0, st);
          cmb[rg][k] = s2;
        }
        __syncthreads();
        if (t < B) {
          double s2 = 0.0;
          for (int r = 0; r < RG; r++) s2 += cmb[r][t];
          ddl[t] = s2;
          rowl[t] = (rv == rv) ? rv : ld_ready(&rb[t], st);
        }
      }
      __syncthreads();
      const Reflector r = make_reflector(ddl[0], rowl[0]);
      if (t < B) wl[t] = (t >= 1 && t < B - j) ? reflector_w(r, rowl[t], ddl[t]) : 0.0;
      if (t == 0) taul[j] = r.tau;
      __syncthreads();
      reflector_apply(a, below, piv, r, wl);
    } else if (t == 0) {
      taul[j] = 0.0;
    }
    // column j of this row is final: record it and shift
    Pl[t][j] = a[0];
#pragma unroll
    for (int k = 0; k < B - 1; k++) a[k] = a[k + 1];
    a[B - 1] = 0.0;
  }
  __syncthreads();

  // write back R / V in place and the explicit V (also to LDS for the Gram)
#pragma unroll 4
  for (int c = 0; c < B; c++) {
    const double x = Pl[t][c];
    const double vv = (gi > c) ? x : (gi == c ? 1.0 : 0.0);
    if (rok) {
      P[gi + (long)c * ldp] = x;
      V[gi + (long)c * ldv] = vv;
    }
    Pl[t][c] = rok ? vv : 0.0;
  }
  if (g == 0 && t < B) tau_out[t] = taul[t];
  __syncthreads();
  // partial Gram of this workgroup's rows (gram_entry's values: the upper
  // triangle, zeros below it); workgroup 0 sums them.  Thread t < 136 forms
  // the 2 x 2 block (bi, bj), bi <= bj, of the upper triangle, reading each
  // of its four columns once per row; each entry is gram_entry's chain of
  // fused multiply-adds over the rows in order.
  {
    auto put = [&](int ca, int cb, double v) {
      if (g == 0)
        Gm[ca][cb] = v;
      else
        st_agent(&gpart[(size_t)g * B * B + ca + (size_t)cb * B], v);
    };
    constexpr int NUB = (B / 2) * (B / 2 + 1) / 2;
    static_assert(NUB <= NT, "one 2 x 2 block per thread");
    if (t < NUB) {
      int bj = 0;
      while ((bj + 1) * (bj + 2) / 2 <= t) bj++;
      const int bi = t - bj * (bj + 1) / 2;
      const int c0 = 2 * bi, c1 = 2 * bj;
      double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
      for (int i = 0; i < nrows; i++) {
        const double a0 = Pl[i][c0], a1 = Pl[i][c0 + 1], b0 = Pl[i][c1], b1 = Pl[i][c1 + 1];
        s00 = fma(a0, b0, s00);
        s01 = fma(a0, b1, s01);
        s10 = fma(a1, b0, s10);
        s11 = fma(a1, b1, s11);
      }
      put(c0, c1, s00);
      put(c0, c1 + 1, s01);
      put(c0 + 1, c1, bi == bj ? 0.0 : s10);  // below the diagonal in a diagonal block
      put(c0 + 1, c1 + 1, s11);
    }
    // the blocks below the diagonal
    for (int e = t; e < B * B; e += NT) {
      const int ca = e % B, cb = e / B;
      if (ca / 2 > cb / 2) put(ca, cb, 0.0);
    }
  }
  if (g != 0) return;
  __syncthreads();
  for (int e = t; e < B * B; e += NT) {
    const int ca = e % B, cb = e / B;
    Gm[ca][cb] = sum_ready<16>(gpart + e, (long)B * B, 1, 1, G, Gm[ca][cb], st);
    Tl[ca][cb] = 0.0;
  }
  __syncthreads();
  form_t<B>(Tl, Gm, taul);
  for (int e = t; e < B * B; e += NT) Tt[e] = Tl[e % B][e / B];
}

// The same panel QR for a solve that shares the device with other solves
// (HSDM_KEY_CONCURRENT): the grid-wide exchange per column becomes a kernel
// boundary, so no workgroup waits for another.  Launch j (j = -1 .. B-1) of
// panel_step_kernel: for j >= 0 it combines the partial sums of column j
// that launch j-1 left in `part`, forms reflector j, applies it to the
// workgroup's rows and writes column j of the result (and of V); then it
// writes the partial sums of column j + 1 (launch B-1: the workgroup's
// partial Gram matrix V^T V instead).  panel_t_kernel (one workgroup) sums
// the Gram partials and forms T.  Every step does the fused kernel's
// arithmetic in the fused kernel's order, so the two give the same bits.
template <int B>
__global__ __launch_bounds__(NT) void panel_step_kernel(int h, double* P, long ldp, double* V,
                                                        long ldv, double* tau_out, double* part,
                                                        double* prow, double* gpart, int j) {
  constexpr int NW = NT / 64;
  constexpr int RG = NT / B;
  __shared__ double red[NW][B];
  __shared__ double ddl[B], wl[B], rowl[B];
  __shared__ double cmb[RG][B + 1];
  __shared__ double Pl[CH][B + 1];
  const int g = blockIdx.x, G = gridDim.x;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int row0 = g * CH;
  const int nrows = min(CH, h - row0);
  const int gi = row0 + t;
  const bool rok = t < nrows;
  const int ncol = min(B, h);
  // a[k]: column c0 + k of this thread's row (columns past B read as zero)
  const int c0 = j < 0 ? 0 : j;
  double a[B];
#pragma unroll
  for (int c = 0; c < B; c++) a[c] = (rok && c0 + c < B) ? P[gi + (long)(c0 + c) * ldp] : 0.0;
  if (j >= 0 && j < ncol) {
    const bool below = rok && gi > j;
    const bool piv = rok && gi == j;
    const double* pb = part + (size_t)j * G * B;
    {
      const int k = t % B, rg = t / B;
      double s2 = 0.0;
      if (k < B - j)
        for (int q = rg; q < G; q += RG) s2 += pb[(size_t)q * B + k];
      cmb[rg][k] = s2;
    }
    __syncthreads();
    if (t < B) {
      double s2 = 0.0;
      for (int r = 0; r < RG; r++) s2 += cmb[r][t];
      ddl[t] = s2;
      rowl[t] = prow[(size_t)j * B + t];  // the pivot row as launch j - 1 left it
    }
    __syncthreads();
    const Reflector r = make_reflector(ddl[0], rowl[0]);
    if (t < B) wl[t] = (t >= 1 && t < B - j) ? reflector_w(r, rowl[t], ddl[t]) : 0.0;
    __syncthreads();
    reflector_apply(a, below, piv, r, wl);
    if (g == 0 && t == 0) tau_out[j] = r.tau;
    if (rok) {
#pragma unroll
      for (int c = 0; c < B; c++)
        if (j + c < B) P[gi + (long)(j + c) * ldp] = a[c];
      V[gi + (long)j * ldv] = (gi > j) ? a[0] : (gi == j ? 1.0 : 0.0);
    }
  } else if (j >= 0 && g == 0 && t == 0) {
    tau_out[j] = 0.0;
  }
  const int jn = j + 1;
  if (jn < B) {
    // partial sums of column jn over this workgroup's rows below its pivot
    const int sh = (j >= 0) ? 1 : 0;  // a[sh + k] holds column jn + k
    double v[B];
    if (jn < ncol) {
      const bool below = rok && gi > jn;
      const double ajn = sh ? a[1] : a[0];
#pragma unroll
      for (int k = 0; k < B; k++) {
        const double x = (sh + k < B) ? a[sh + k] : 0.0;
        v[k] = below ? ajn * x : 0.0;
      }
    } else {
#pragma unroll
      for (int k = 0; k < B; k++) v[k] = 0.0;
    }
    const double ws = wave_reduce_scatter(v);
    if (lane < 32) red[wv][rs_index(lane)] = ws;
    // the next pivot row, for every workgroup of the next launch (P itself
    // changes under them in that launch)
    if (rok && gi == jn) {
#pragma unroll
      for (int k = 0; k < B; k++) prow[(size_t)jn * B + k] = (sh + k < B) ? a[sh + k] : 0.0;
    }
    __syncthreads();
    if (t < B) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < NW; w++) sum += red[w][t];
      part[(size_t)jn * G * B + (size_t)g * B + t] = sum;
    }
    return;
  }
  // last launch: this workgroup's partial Gram of the explicit V
  __syncthreads();
  for (int e = t; e < CH * B; e += NT) {
    const int r = e % CH, c = e / CH;
    const int gr = row0 + r;
    Pl[r][c] = (r < nrows) ? ((gr > c) ? P[gr + (long)c * ldp] : (gr == c ? 1.0 : 0.0)) : 0.0;
  }
  __syncthreads();
  for (int e = t; e < B * B; e += NT)
    gpart[(size_t)g * B * B + e] = gram_entry<B>(Pl, nrows, e % B, e / B);
}

template <int B>
__global__ __launch_bounds__(NT) void panel_t_kernel(const double* tau, double* Tt,
                                                     const double* gpart, int G) {
  __shared__ double Gm[B][B + 1], Tl[B][B + 1], taul[B];
  const int t = threadIdx.x;
  if (t < B) taul[t] = tau[t];
  for (int e = t; e < B * B; e += NT) {
    const int ca = e % B, cb = e / B;
    double sum = gpart[e];
    for (int q = 1; q < G; q++) sum += gpart[(size_t)q * B * B + e];
    Gm[ca][cb] = sum;
    Tl[ca][cb] = 0.0;
  }
  __syncthreads();
  form_t<B>(Tl, Gm, taul);
  for (int e = t; e < B * B; e += NT) Tt[e] = Tl[e % B][e / B];
}

template <int B>
__global__ __launch_bounds__(NT) void panel_qr_kernel(int h, double* P, long ldp, double* V,
                                                      long ldv, double* tau_out, double* Tt,
                                                      double* part, double* prow, double* gpart,
                                                      DevStatusWord* st) {
  panel_qr_body<B>(h, P, ldp, V, ldv, tau_out, Tt, part, prow, gpart, st, blockIdx.x, gridDim.x);
}

// The panels of several tasks in one cooperative launch: workgroups g0 ..
// g0 + G - 1 of the grid hold the rows of panel task wg_task[blockIdx.x].
template <int B>
__global__ __launch_bounds__(NT) void panel_qr_group_kernel(const PanelQrTask* tasks,
                                                            const int* wg_task) {
  const int p = __builtin_amdgcn_readfirstlane(wg_task[blockIdx.x]);
  const PanelQrTask& q = tasks[p];
  panel_qr_body<B>(q.h, q.P, q.ldp, q.V, q.ldv, q.tau, q.T, q.part, q.prow, q.gpart, q.st,
                   (int)blockIdx.x - q.g0, q.G);
}

// Exchange slots of the panels of a grouped launch back to NaN (task
// blockIdx.y of the list; span 0 for single-workgroup panels).
__global__ void fill_nan_group_kernel(const PanelQrTask* tasks) {
  const PanelQrTask& q = tasks[blockIdx.y];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < q.span;
       i += (long)gridDim.x * blockDim.x)
    q.part[i] = __builtin_nan("");
}

// Householder QR of one panel (the task's P, V, tau, T and exchange slots;
// span: how many exchange slots to reset first).  Beside other solves
// (a concurrent handle) no workgroup waits for another: one launch per
// column for several workgroups, an ordinary launch for one; otherwise one
// cooperative launch.  Algorithmic: 2 h B^2 flops, the panel read and
// written once.
hipError_t run_panel_qr(PanelQrTask q, hipStream_t s) {
  constexpr int BB = 32;
  const int B = BB;
  if (q.span > 0) {
    HSDM_LAUNCH(fill_nan_kernel, dim3((unsigned)((q.span + 255) / 256)), dim3(256), 0, s,
                q.part, q.span);
    HSDM_TRY(hipGetLastError());
  }
  void* args[] = {(void*)&q.h, (void*)&q.P, (void*)&q.ldp, (void*)&q.V, (void*)&q.ldv,
                  (void*)&q.tau, (void*)&q.T, (void*)&q.part, (void*)&q.prow, (void*)&q.gpart,
                  (void*)&q.st};
  if (coop_get_shared()) {
    if (q.G == 1) {
      HSDM_LAUNCH(panel_qr_kernel<BB>, dim3(1), dim3(NT), 0, s, q.h, q.P, q.ldp, q.V, q.ldv,
                  q.tau, q.T, q.part, q.prow, q.gpart, q.st);
      return hipGetLastError();
    }
    kt_begin("panel_step_kernel<32>", 2.0 * q.h * B * B, 16.0 * q.h * B, 0, s);
    for (int j = -1; j < BB; j++) {
      HSDM_LAUNCH(panel_step_kernel<BB>, dim3(q.G), dim3(NT), 0, s, q.h, q.P, q.ldp, q.V,
                  q.ldv, q.tau, q.part, q.prow, q.gpart, j);
      HSDM_TRY(hipGetLastError());
    }
    HSDM_LAUNCH(panel_t_kernel<BB>, dim3(1), dim3(NT), 0, s, q.tau, q.T, q.gpart, q.G);
    kt_end(s);
    return hipGetLastError();
  }
  return coop_launch("panel_qr_kernel<32>", 2.0 * q.h * B * B, 16.0 * q.h * B, false, true,
                     (const void*)panel_qr_kernel<BB>, dim3(q.G), dim3(NT), args, s);
}

// Band extraction: AB[(r-c) + c*ldab] = A[r + c*lda] for 0 <= r-c <= B, zero
// for B < r-c < ldab.
__global__ void band_extract_kernel(int n, int B, const double* A, long lda, double* AB,
                                    int ldab) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * ldab) return;
  const int off = (int)(idx % ldab), c = (int)(idx / ldab);
  const int r = c + off;
  AB[idx] = (off <= B && r < n) ? A[r + (long)c * lda] : 0.0;
}

// P = U^T W for h x B tall operands: per-workgroup partial sums, then a
// fixed-order reduction (reproducible).  Workgroup g sums rows
// [ACH g, ACH g + ACH).
template <int B>
HSDM_DEV void atb_partial_body(int h, const double* U, long ldu, const double* W, long ldw,
                               double* part, int g) {
  const int t = threadIdx.x;
  const int r0 = g * ACH, nr = min(ACH, h - r0);
  __shared__ double Us[ACH][B + 1], Ws[ACH][B + 1];
  for (int e = t; e < ACH * B; e += NT) {
    const int i = e % ACH, c = e / ACH;
    Us[i][c] = (i < nr) ? U[r0 + i + (long)c * ldu] : 0.0;
    Ws[i][c] = (i < nr) ? W[r0 + i + (long)c * ldw] : 0.0;
  }
  __syncthreads();
  // thread t: entries e = t + NT j, which share the column a = t % B of U
  static_assert(NT % B == 0, "the entries of one thread share a column of U");
  constexpr int PER = B * B / NT;
  const int a = t % B;
  double s[PER];
#pragma unroll
  for (int j = 0; j < PER; j++) s[j] = 0.0;
  for (int i = 0; i < nr; i++) {
    const double u = Us[i][a];
#pragma unroll
    for (int j = 0; j < PER; j++) s[j] += u * Ws[i][(t + NT * j) / B];
  }
#pragma unroll
  for (int j = 0; j < PER; j++) part[(size_t)g * B * B + t + NT * j] = s[j];
}

template <int B>
HSDM_DEV void atb_reduce_body(int G, const double* part, double* out, long ldo, int e) {
  if (e >= B * B) return;
  const double s = sum_in_order(part + e, (long)B * B, G, 0.0);
  out[(e % B) + (long)(e / B) * ldo] = s;
}

// U^T W for U of gridDim.y blocks of B columns: workgroup (g, c) forms the
// partial of rows [ACH g, ACH g + ACH) of column block c (the partials of
// block c follow those of block c - 1); the reduction's blockIdx.y = c sums
// block c's into rows [B c, B c + B) of out.
template <int B>
__global__ __launch_bounds__(NT) void atb_partial_kernel(int h, const double* U, long ldu,
                                                         const double* W, long ldw,
                                                         double* part) {
  atb_partial_body<B>(h, U + (long)blockIdx.y * B * ldu, ldu, W, ldw,
                      part + (size_t)blockIdx.y * gridDim.x * B * B, blockIdx.x);
}

template <int B>
__global__ void atb_reduce_kernel(int G, const double* part, double* out, long ldo) {
  atb_reduce_body<B>(G, part + (size_t)blockIdx.y * G * B * B, out + (long)blockIdx.y * B, ldo,
                     blockIdx.x * blockDim.x + threadIdx.x);
}

// The same for the items of a grouped launch: workgroup blockIdx.x works on
// item wg_item[blockIdx.x]; the reduction takes item blockIdx.y.
template <int B>
__global__ __launch_bounds__(NT) void atb_partial_group_kernel(const AtbGroupItem* items,
                                                               const int* wg_item) {
  const int q = __builtin_amdgcn_readfirstlane(wg_item[blockIdx.x]);
  const AtbGroupItem& it = items[q];
  atb_partial_body<B>(it.h, it.U, it.ldu, it.W, it.ldw, it.part, (int)blockIdx.x - it.b0);
}

template <int B>
__global__ void atb_reduce_group_kernel(const AtbGroupItem* items) {
  const AtbGroupItem& it = items[blockIdx.y];
  atb_reduce_body<B>(it.G, it.part, it.out, it.ldo, blockIdx.x * blockDim.x + threadIdx.x);
}

// Column copies of a grouped launch, item blockIdx.y.
__global__ void copy_group_kernel(const CopyGroupItem* items) {
  const CopyGroupItem& it = items[blockIdx.y];
  const long tot = (long)it.m * it.n;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const long i = idx % it.m, j = idx / it.m;
    it.dst[i + j * it.ldd] = it.src[i + j * it.lds];
  }
}

}  // namespace

size_t sy2sb_scratch_doubles(int n, int B) {
  const int G = ceil_div(n, CH) + 1, AG = ceil_div(n, ACH) + 1;
  // panel exchange slots: part (B columns x G x B) + prow (B x B) + gpart (G B^2);
  // atb parts (AG B^2) + Y (n x B) + VW, WV (n x 2 PGROUP B each) + M (B^2)
  // + Q (2 PGROUP B^2) + split-K partials of the two symmetric passes
  // (nsplit x n x B each)
  const size_t nsplit = ceil_div(n, SPLITK) + 1;
  return (size_t)G * B * B + (size_t)B * B + (size_t)G * B * B + (size_t)AG * B * B +
         (size_t)(1 + 4 * PGROUP) * n * B + (size_t)(1 + 2 * PGROUP) * B * B + 64 +
         2 * nsplit * n * B;
}

// A multi-task reduction takes the panels in pairs with one trailing update
// per pair (a single reduction takes groups of PGROUP panels the same way,
// Sy2sb::group_panel).  For the pair (p, p+1), with A22 the trailing block of
// panel p:
//   panel p:   QR -> V1, T1;  Y1 = V1 T1;  X1 = A22 Y1;  W1 = X1 - V1 (Y1^T X1) / 2;
//              only the B columns of panel p+1 receive the update
//              A22[:, 0:B] -= V1 W1[0:B]^T + W1 V1[0:B]^T;
//   panel p+1: QR -> V2, T2 on the updated columns;  Y2 = V2 T2;
//              X2 = A22'' Y2 with A22'' = A22[B:, B:] - V1b W1b^T - W1b V1b^T
//                 = A22[B:, B:] Y2 - [V1b W1b] ([W1b V1b]^T Y2)   (b: rows B..)
//              W2 = X2 - V2 (Y2^T X2) / 2;
//   then one rank-4B update A22[B:, B:] -= [V1b W1b V2 W2][W1b V1b W2 V2]^T,
// which halves the passes over the trailing matrix.  The products are the
// same as panel by panel; only the order of the roundings differs.
namespace {

// One matrix's full-to-band reduction: its pointers, the layout of its
// scratch, and the steps between panel QRs.
struct Sy2sb {
  static constexpr int BB = 32;
  int n, B;
  double* A;
  long lda;
  double* Vst;
  long ldv;
  double *tau1, *T1, *AB;
  int ldab;
  DevStatusWord* st;
  hipStream_t s;
  int Gmax;
  double *part, *prow, *gpart, *apart, *Y, *VW, *WV, *M, *Qc, *skpart, *skpart2;

  Sy2sb(const Sy2sbArgs& a, int B_, hipStream_t s_)
      : n(a.n), B(B_), A(a.A), lda(a.lda), Vst(a.Vst), ldv(a.ldv), tau1(a.tau1), T1(a.T1),
        AB(a.AB), ldab(a.ldab), st(a.st), s(s_) {
    Gmax = ceil_div(n, CH) + 1;
    part = a.scratch;                      // B x Gmax x B exchange slots
    prow = part + (size_t)B * Gmax * B;    // B x B
    gpart = prow + (size_t)B * B;          // Gmax x B x B
    apart = gpart + (size_t)Gmax * B * B;  // (n / ACH + 1) x B x B
    Y = apart + (size_t)(ceil_div(n, ACH) + 1) * B * B;  // n x B
    VW = Y + (size_t)n * B;                // n x 2 PGROUP B  [V1 W1 V2 W2 ...], row i <-> row r0 + i
    WV = VW + (size_t)n * 2 * PGROUP * B;  // n x 2 PGROUP B  [W1 V1 W2 V2 ...]
    M = WV + (size_t)n * 2 * PGROUP * B;   // B x B
    Qc = M + B * B;                        // 2 PGROUP B x B
    skpart = Qc + 2 * PGROUP * B * B + 64;  // split-K partials
    skpart2 = skpart + (size_t)(ceil_div(n, SPLITK) + 1) * n * B;  // the second pass's
  }
  int npanel() const { return (n > B) ? ceil_div(n - 1, B) : 0; }
  int height(int p) const { return n - (p + 1) * B; }
  // panels reduced after panel p's QR: 1 (alone), 2 (p + 1 with it, its QR next)
  int advance(int p) const {
    const int h = height(p);
    if (h <= 1) return 1;
    return (p + 1 < npanel() && h - B > 1) ? 2 : 1;
  }

  // Householder QR of panel p (rows r0.., columns c0..c0+B-1)
  PanelQrTask qr_desc(int p) const {
    const int c0 = p * B, r0 = c0 + B, h = n - r0;
    PanelQrTask q{};
    q.P = A + r0 + (long)c0 * lda;
    q.V = Vst + r0 + (long)c0 * ldv;
    q.tau = tau1 + c0;
    q.T = T1 + (size_t)p * B * B;
    q.part = part;
    q.prow = prow;
    q.gpart = gpart;
    q.st = st;
    q.ldp = lda;
    q.ldv = ldv;
    q.h = h;
    q.G = ceil_div(h, CH);
    // exchange slots of a multi-workgroup panel back to NaN (part, prow,
    // gpart are contiguous)
    q.span = q.G > 1 ? (long)(gpart - part) + (long)B * B * q.G : 0;
    return q;
  }
  hipError_t qr_panel(int p) { return run_panel_qr(qr_desc(p), s); }
  // W (h x B, ld n, holding X on entry) = X - V M / 2 with Y = V T, X = A[r:, r:] Y,
  // M = Y^T X.  Vp: the panel's V (ld ldv), Tp its T; Y receives V T.
  // In three steps (the middle one, the two passes of the symmetric product,
  // and in a multi-task reduction every step, can run grouped over tasks).
  GemmArgs pre_args(int h, const double* Vp, const double* Tp) const {
    GemmArgs g{};
    g.m = h; g.n = B; g.k = B; g.A = Vp; g.lda = ldv; g.B = Tp; g.ldb = B; g.C = Y; g.ldc = n;
    g.alpha = 1.0; g.beta = 0.0; g.flags = GF_KB_UPPER;
    return g;
  }
  hipError_t make_w_pre(int h, const double* Vp, const double* Tp) {
    return gemm_launch(pre_args(h, Vp, Tp), s);
  }
  // X = A[r:, r:] Y: A symmetric with its lower triangle stored,
  // X = tril(A) Y + strict_tril(A)^T Y, both passes reading the lower triangle
  void sym_args(int r, int h, double* Wp, GemmArgs& tril, GemmArgs& slt) const {
    const double* Ar = A + r + (long)r * lda;
    tril = GemmArgs{};
    tril.m = h; tril.n = B; tril.k = h; tril.A = Ar; tril.lda = lda; tril.B = Y; tril.ldb = n;
    tril.C = Wp; tril.ldc = n; tril.alpha = 1.0; tril.beta = 0.0;
    tril.flags = GF_A_TRIL | GF_KA_LOWER;
    slt = tril;
    slt.ta = 1; slt.beta = 1.0; slt.flags = GF_A_SLT | GF_KA_UPPER;
  }
  hipError_t make_w_sym(int r, int h, double* Wp) {
    GemmArgs t, u;
    sym_args(r, h, Wp, t, u);
    if (h > SPLITK) return gemm_sym_pair_launch(t, SPLITK, skpart, skpart2, s);
    HSDM_TRY(gemm_splitk_launch(t, SPLITK, skpart, s));
    return gemm_splitk_launch(u, SPLITK, skpart, s);
  }
  // the delayed update of the first panel of a pair:
  // X -= [V1b W1b] Qc with Qc = [W1b V1b]^T Y
  GemmArgs corr1_args(int h, const double* WVc) const {
    GemmArgs g{};
    g.m = 2 * B; g.n = B; g.k = h; g.A = WVc; g.lda = n; g.B = Y; g.ldb = n; g.C = Qc;
    g.ldc = 2 * B; g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0;
    return g;
  }
  GemmArgs corr2_args(int h, const double* VWc, double* Wp) const {
    GemmArgs g{};
    g.m = h; g.n = B; g.k = 2 * B; g.A = VWc; g.lda = n; g.B = Qc; g.ldb = 2 * B; g.C = Wp;
    g.ldc = n; g.alpha = -1.0; g.beta = 1.0;
    return g;
  }
  // M = Y^T X (partial sums per ACH rows)
  AtbGroupItem atb_item(int h, const double* Wp) const {
    AtbGroupItem it{};
    it.U = Y; it.ldu = n; it.W = Wp; it.ldw = n; it.part = apart; it.out = M; it.ldo = B;
    it.h = h; it.G = ceil_div(h, ACH);
    return it;
  }
  // W -= V M / 2
  GemmArgs fix_args(int h, const double* Vp, double* Wp) const {
    GemmArgs g{};
    g.m = h; g.n = B; g.k = B; g.A = Vp; g.lda = ldv; g.B = M; g.ldb = B; g.C = Wp; g.ldc = n;
    g.alpha = -0.5; g.beta = 1.0;
    return g;
  }
  // out (nblk B x B, leading dimension ldo) = U^T W for h x (nblk B) U and
  // h x B W; part holds ceil(h / ACH) nblk B^2 partials
  hipError_t atb(int h, const double* U, long ldu, const double* W, long ldw, int nblk,
                 double* part, double* out, long ldo) {
    const int G = ceil_div(h, ACH);
    HSDM_LAUNCH((atb_partial_kernel<BB>), dim3(G, nblk), dim3(NT), 0, s, h, U, ldu, W, ldw,
                part);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH((atb_reduce_kernel<BB>), dim3(ceil_div(B * B, 256), nblk), dim3(256), 0, s, G,
                part, out, ldo);
    return hipGetLastError();
  }
  hipError_t make_w_post(int h, const double* Vp, double* Wp) {
    const AtbGroupItem a = atb_item(h, Wp);
    HSDM_TRY(atb(h, a.U, a.ldu, a.W, a.ldw, 1, a.part, a.out, a.ldo));
    return gemm_launch(fix_args(h, Vp, Wp), s);
  }
  // the panel's V and W into the update operands: VW[:, o:o+2B] = [V W],
  // WV[:, o:o+2B] = [W V] (o = 0 first panel, B rows and 2B columns in for
  // the second panel of a pair)
  void copies(int h, const double* Vp, const double* Wp, long o, CopyGroupItem (&c)[3]) const {
    c[0] = CopyGroupItem{Vp, VW + o, ldv, (long)n, h, B};
    c[1] = CopyGroupItem{Wp, WV + o, (long)n, (long)n, h, B};
    c[2] = CopyGroupItem{Vp, WV + o + (size_t)n * B, ldv, (long)n, h, B};
  }

  // A[r:, r:] -= VWr WVr^T (lower), k columns
  GemmArgs syr2k_args(int r, int h, const double* VWr, const double* WVr, int k) const {
    GemmArgs g{};
    g.m = h; g.n = h; g.k = k; g.A = VWr; g.lda = n; g.B = WVr; g.ldb = n;
    g.C = A + r + (long)r * lda; g.ldc = lda; g.alpha = -1.0; g.beta = 1.0; g.ta = 0; g.tb = 1;
    g.flags = GF_C_LOWER_TILES | GF_C_LOWER_ONLY;
    return g;
  }
  hipError_t syr2k(int r, int h, const double* VWr, const double* WVr, int k) {
    return gemm_launch(syr2k_args(r, h, VWr, WVr, k), s);
  }
  // columns of panel p+1: A[r0:, r0:r0+B] -= [V1 W1] [W1 V1][0:B]^T (lower part)
  GemmArgs col_args(int r0, int h) const {
    GemmArgs g{};
    g.m = h; g.n = B; g.k = 2 * B; g.A = VW; g.lda = n; g.B = WV; g.ldb = n;
    g.C = A + r0 + (long)r0 * lda; g.ldc = lda; g.alpha = -1.0; g.beta = 1.0; g.ta = 0;
    g.tb = 1; g.flags = GF_C_LOWER_ONLY;
    return g;
  }
  // Operands of the multi-task reduction's pair steps (the grouped launches
  // build their descriptors from these): after the QR of panel p, its W and
  // either the trailing update (panel alone) or the update of panel p+1's
  // columns (pair).
  bool first_has_w(int p) const { return height(p) > 1; }
  const double* first_v(int p) const { return Vst + (p + 1) * B + (long)p * B * ldv; }
  const double* first_t(int p) const { return T1 + (size_t)p * B * B; }
  double* first_w() const { return VW + (size_t)n * B; }
  void first_sym(int p, GemmArgs& tril, GemmArgs& slt) const {
    const int r0 = (p + 1) * B;
    sym_args(r0, n - r0, first_w(), tril, slt);
  }

  // after the QR of panel p+1 of a pair: its W (with the first panel's
  // delayed update) and the pair's rank-4B trailing update
  const double* second_v(int p) const { return Vst + (p + 2) * B + (long)(p + 1) * B * ldv; }
  const double* second_t(int p) const { return T1 + (size_t)(p + 1) * B * B; }
  double* second_w() const { return VW + B + (size_t)3 * n * B; }
  static long second_off(int n_, int B_) { return B_ + (long)2 * n_ * B_; }
  void second_sym(int p, GemmArgs& tril, GemmArgs& slt) const {
    const int r1 = (p + 2) * B;
    sym_args(r1, n - r1, second_w(), tril, slt);
  }

  // ---- single reduction: up to PGROUP panels per trailing update ----------
  // For the group of panels p0 .. p0 + P - 1 (panel q at rows r_q =
  // (p0 + q + 1) B, height h_q), every panel's update
  // U_q = V_q W_q^T + W_q V_q^T of its trailing block is held back until the
  // group ends, except on the columns of the next panel, which need it
  // before their QR.  Panel q's symmetric product is then corrected for the
  // held-back updates of panels 0 .. q-1:
  //   X_q = A[r_q:, r_q:] Y_q - [V W]_<q ([W V]_<q^T Y_q),
  // and the group ends with one rank-2PB update of the trailing block of its
  // last panel.  V_q and W_q are kept in VW = [V_0 W_0 V_1 W_1 ...] and
  // WV = [W_0 V_0 W_1 V_1 ...] with row i at global row r_0 + i (panel q's
  // columns valid from row qB on; no product reads above that).
  int group_size(int p0) const {
    int P = 1;
    if (height(p0) <= 1) return 1;
    while (P < PGROUP && p0 + P < npanel() && height(p0 + P) > 1) P++;
    return P;
  }
  hipError_t group_panel(int p0, int q, int P) {
    const int p = p0 + q, rq = (p + 1) * B, h = n - rq;
    HSDM_TRY(qr_panel(p));
    if (h <= 1) return hipSuccess;
    const long o = (long)q * B;                 // row offset of panel q in VW, WV
    const double* Vq = Vst + rq + (long)p * B * ldv;
    double* Wq = VW + o + (size_t)(2 * q + 1) * n * B;
    HSDM_TRY(make_w_pre(h, Vq, T1 + (size_t)p * B * B));
    HSDM_TRY(make_w_sym(rq, h, Wq));
    if (q > 0) {
      // corrections for the held-back updates of panels 0 .. q-1:
      // Qc = [W V]_<q^T Y (2q blocks of B columns, partials in skpart)
      const size_t need = (size_t)ceil_div(h, ACH) * 2 * q * B * B;
      if (need > (size_t)(ceil_div(n, SPLITK) + 1) * n * B) return hipErrorInvalidValue;
      HSDM_TRY(atb(h, WV + o, n, Y, n, 2 * q, skpart, Qc, 2 * B * q));
      GemmArgs g{};
      g.m = h; g.n = B; g.k = 2 * B * q; g.A = VW + o; g.lda = n; g.B = Qc; g.ldb = 2 * B * q;
      g.C = Wq; g.ldc = n; g.alpha = -1.0; g.beta = 1.0;
      HSDM_TRY(gemm_launch(g, s));
    }
    HSDM_TRY(make_w_post(h, Vq, Wq));
    // V_q into VW, [W_q V_q] into WV (W_q is already in VW)
    HSDM_TRY(file_vw(h, B, Vq, ldv, (const double*)Wq, (long)n, VW + o + (size_t)2 * q * n * B,
                     WV + o + (size_t)2 * q * n * B, WV + o + (size_t)(2 * q + 1) * n * B,
                     (long)n, s));
    if (q + 1 < P) {
      // the next panel's columns (rows from r_q) receive the updates of
      // panels 0 .. q
      GemmArgs g{};
      g.m = h; g.n = B; g.k = 2 * B * (q + 1); g.A = VW + o; g.lda = n; g.B = WV + o;
      g.ldb = n; g.C = A + rq + (long)rq * lda; g.ldc = lda; g.alpha = -1.0; g.beta = 1.0;
      g.ta = 0; g.tb = 1; g.flags = GF_C_LOWER_ONLY;
      return gemm_launch(g, s);
    }
    // the group's one trailing update, rank 2PB, of panel q's trailing block
    return syr2k(rq, h, VW + o, WV + o, 2 * B * P);
  }

  hipError_t finish() {
    const long tot = (long)n * ldab;
    HSDM_LAUNCH(band_extract_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       n, B, A, lda, AB, ldab);
    return hipGetLastError();
  }
};

}  // namespace

hipError_t sy2sb_run(int n, int B, double* A, long lda, double* Vst, long ldv, double* tau1,
                     double* T1, double* AB, int ldab, double* scratch, DevStatusWord* st,
                     hipStream_t s) {
  if (B != 32) return hipErrorInvalidValue;
  Sy2sb R(Sy2sbArgs{n, A, lda, Vst, ldv, tau1, T1, AB, ldab, scratch, st}, B, s);
  for (int p = 0; p < R.npanel();) {
    if (R.height(p) <= 0) break;
    const int P = R.group_size(p);
    for (int q = 0; q < P; q++) HSDM_TRY(R.group_panel(p, q, P));
    p += P;
  }
  return R.finish();
}

namespace {

constexpr int PQR_MAX_WG = 256;  // one panel workgroup per compute unit (LDS)

// The rounds of a multi-task reduction: round k performs one pair step of
// every task that still has panels.  Returns, per round, the tasks and the
// panel each starts at.
std::vector<std::vector<std::pair<int, int>>> group_rounds(const std::vector<Sy2sb>& R) {
  std::vector<std::vector<std::pair<int, int>>> rounds;
  std::vector<int> p(R.size(), 0);
  for (;;) {
    std::vector<std::pair<int, int>> r;
    for (size_t t = 0; t < R.size(); t++)
      if (p[t] < R[t].npanel() && R[t].height(p[t]) > 0) r.emplace_back((int)t, p[t]);
    if (r.empty()) break;
    for (auto& e : r) p[e.first] += R[e.first].advance(e.second);
    rounds.push_back(std::move(r));
  }
  return rounds;
}

// Grouped launches (descriptor range [d0, d0 + nd), workgroup map entries
// from m0).  QR lists are cut into launches of at most PQR_MAX_WG
// workgroups; every other step of a round is one launch over the tasks
// taking part in it (nd = 0: none).
struct QrLaunch {
  int d0, nd, m0, nwg;
};
struct GemmLaunch {
  int kind, d0, nd, m0, nwg, max_tot;
  bool split;
  double flops;
};
struct AtbLaunch {
  int d0, nd, m0, nwg;
};
struct CopyLaunch {
  int d0, nd;
  long max_tot;
};
// One round: the first panels' QRs and their W (Y = V T, the two passes of
// X = A22 Y, M = Y^T X, W = X - V M / 2), the copies into the update
// operands, the trailing updates of the single panels and the column update
// of the pairs' second panels, then the same for the second panels with the
// first panel's delayed update (Qc = [W1 V1]^T Y, X -= [V1 W1] Qc) before M,
// and the pairs' trailing updates.
struct Round {
  std::vector<std::pair<int, int>> tasks;
  std::vector<QrLaunch> qr1, qr2;
  GemmLaunch pre1, tril1, slt1, fix1, col1, syr1, pre2, tril2, slt2, corr1, corr2, fix2, syr2;
  AtbLaunch atb1, atb2;
  CopyLaunch cp1, cp2;
};

struct Builder {
  Sy2sbGroupHost& host;
  void qr(const std::vector<PanelQrTask>& list, std::vector<QrLaunch>& out) {
    size_t i = 0;
    while (i < list.size()) {
      QrLaunch L{(int)host.desc.size(), 0, (int)host.wgmap.size(), 0};
      while (i < list.size() && (L.nd == 0 || L.nwg + list[i].G <= PQR_MAX_WG)) {
        PanelQrTask q = list[i++];
        q.g0 = L.nwg;
        for (int w = 0; w < q.G; w++) host.wgmap.push_back(L.nd);  // index within the launch
        L.nwg += q.G;
        L.nd++;
        host.desc.push_back(q);
      }
      out.push_back(L);
    }
  }
  // products (args, K slice (0: in place), split-K partial buffer), all of one kind
  GemmLaunch gemm(const std::vector<std::tuple<GemmArgs, int, double*>>& list) {
    GemmLaunch L{GG_NN, (int)host.gemm.size(), 0, (int)host.gemmmap.size(), 0, 0, false, 0.0};
    for (auto& e : list) {
      GemmGroupItem it;
      double f = 0.0;
      const GemmArgs& g = std::get<0>(e);
      if (g.m <= 0 || g.n <= 0) continue;
      L.kind = gemm_group_kind(g);
      const int w = (int)gemm_group_item(g, std::get<1>(e), std::get<2>(e), it, &f);
      it.b0 = L.nwg;
      for (int q = 0; q < w; q++) host.gemmmap.push_back(L.nd);
      L.nwg += w;
      L.nd++;
      L.flops += f;
      if (it.kchunk > 0) {
        L.split = true;
        L.max_tot = std::max(L.max_tot, it.m * it.n);
      }
      host.gemm.push_back(it);
    }
    return L;
  }
  AtbLaunch atb(const std::vector<AtbGroupItem>& list) {
    AtbLaunch L{(int)host.atb.size(), 0, (int)host.atbmap.size(), 0};
    for (AtbGroupItem it : list) {
      it.b0 = L.nwg;
      for (int q = 0; q < it.G; q++) host.atbmap.push_back(L.nd);
      L.nwg += it.G;
      L.nd++;
      host.atb.push_back(it);
    }
    return L;
  }
  CopyLaunch copy(const std::vector<CopyGroupItem>& list) {
    CopyLaunch L{(int)host.copy.size(), 0, 0};
    for (const CopyGroupItem& it : list) {
      L.max_tot = std::max(L.max_tot, (long)it.m * it.n);
      L.nd++;
      host.copy.push_back(it);
    }
    return L;
  }
};

void build_schedule(const std::vector<Sy2sb>& R, Sy2sbGroupHost& host, std::vector<Round>& S) {
  const auto rounds = group_rounds(R);
  host.desc.clear();
  host.wgmap.clear();
  host.gemm.clear();
  host.gemmmap.clear();
  host.atb.clear();
  host.atbmap.clear();
  host.copy.clear();
  S.assign(rounds.size(), Round{});
  Builder bld{host};
  using GL = std::vector<std::tuple<GemmArgs, int, double*>>;
  for (size_t k = 0; k < rounds.size(); k++) {
    Round& rd = S[k];
    rd.tasks = rounds[k];
    std::vector<PanelQrTask> q1, q2;
    GL pre1, tril1, slt1, fix1, col1, syr1, pre2, tril2, slt2, corr1, corr2, fix2, syr2;
    std::vector<AtbGroupItem> atb1, atb2;
    std::vector<CopyGroupItem> cp1, cp2;
    for (auto& e : rd.tasks) {
      const Sy2sb& T = R[e.first];
      const int p = e.second;
      q1.push_back(T.qr_desc(p));
      if (T.first_has_w(p)) {
        const int r0 = (p + 1) * T.B, h = T.n - r0;
        pre1.emplace_back(T.pre_args(h, T.first_v(p), T.first_t(p)), 0, nullptr);
        GemmArgs t, u;
        T.first_sym(p, t, u);
        tril1.emplace_back(t, SPLITK, T.skpart);
        slt1.emplace_back(u, SPLITK, T.skpart);
        atb1.push_back(T.atb_item(h, T.first_w()));
        fix1.emplace_back(T.fix_args(h, T.first_v(p), T.first_w()), 0, nullptr);
        CopyGroupItem c[3];
        T.copies(h, T.first_v(p), T.first_w(), 0, c);
        cp1.insert(cp1.end(), c, c + 3);
        if (T.advance(p) == 2)
          col1.emplace_back(T.col_args(r0, h), 0, nullptr);
        else
          syr1.emplace_back(T.syr2k_args(r0, h, T.VW, T.WV, 2 * T.B), 0, nullptr);
      }
      if (T.advance(p) == 2) {
        const int r1 = (p + 2) * T.B, h2 = T.n - r1;
        q2.push_back(T.qr_desc(p + 1));
        pre2.emplace_back(T.pre_args(h2, T.second_v(p), T.second_t(p)), 0, nullptr);
        GemmArgs t, u;
        T.second_sym(p, t, u);
        tril2.emplace_back(t, SPLITK, T.skpart);
        slt2.emplace_back(u, SPLITK, T.skpart);
        corr1.emplace_back(T.corr1_args(h2, T.WV + T.B), h2 > SPLITK ? SPLITK : 0, T.skpart);
        corr2.emplace_back(T.corr2_args(h2, T.VW + T.B, T.second_w()), 0, nullptr);
        atb2.push_back(T.atb_item(h2, T.second_w()));
        fix2.emplace_back(T.fix_args(h2, T.second_v(p), T.second_w()), 0, nullptr);
        CopyGroupItem c[3];
        T.copies(h2, T.second_v(p), T.second_w(), Sy2sb::second_off(T.n, T.B), c);
        cp2.insert(cp2.end(), c, c + 3);
        syr2.emplace_back(T.syr2k_args(r1, h2, T.VW + T.B, T.WV + T.B, 4 * T.B), 0, nullptr);
      }
    }
    bld.qr(q1, rd.qr1);
    rd.pre1 = bld.gemm(pre1);
    rd.tril1 = bld.gemm(tril1);
    rd.slt1 = bld.gemm(slt1);
    rd.atb1 = bld.atb(atb1);
    rd.fix1 = bld.gemm(fix1);
    rd.cp1 = bld.copy(cp1);
    rd.col1 = bld.gemm(col1);
    rd.syr1 = bld.gemm(syr1);
    bld.qr(q2, rd.qr2);
    rd.pre2 = bld.gemm(pre2);
    rd.tril2 = bld.gemm(tril2);
    rd.slt2 = bld.gemm(slt2);
    rd.corr1 = bld.gemm(corr1);
    rd.corr2 = bld.gemm(corr2);
    rd.atb2 = bld.atb(atb2);
    rd.fix2 = bld.gemm(fix2);
    rd.cp2 = bld.copy(cp2);
    rd.syr2 = bld.gemm(syr2);
  }
}

struct GroupDev {
  PanelQrTask* desc;
  GemmGroupItem* gemm;
  AtbGroupItem* atb;
  CopyGroupItem* copy;
  int* map;
  int* gemmmap;
  int* atbmap;
};

// device layout: the item arrays (8-byte aligned structures), then the maps
GroupDev group_dev(void* d_buf, const Sy2sbGroupHost& host) {
  GroupDev g{};
  char* p = (char*)d_buf;
  g.desc = (PanelQrTask*)p;
  p += sizeof(PanelQrTask) * (host.desc.size() + 1);
  g.gemm = (GemmGroupItem*)p;
  p += sizeof(GemmGroupItem) * (host.gemm.size() + 1);
  g.atb = (AtbGroupItem*)p;
  p += sizeof(AtbGroupItem) * (host.atb.size() + 1);
  g.copy = (CopyGroupItem*)p;
  p += sizeof(CopyGroupItem) * (host.copy.size() + 1);
  g.map = (int*)p;
  p += sizeof(int) * (host.wgmap.size() + 1);
  g.gemmmap = (int*)p;
  p += sizeof(int) * (host.gemmmap.size() + 1);
  g.atbmap = (int*)p;
  return g;
}

size_t group_bytes(const Sy2sbGroupHost& host) {
  return sizeof(PanelQrTask) * (host.desc.size() + 1) +
         sizeof(GemmGroupItem) * (host.gemm.size() + 1) +
         sizeof(AtbGroupItem) * (host.atb.size() + 1) +
         sizeof(CopyGroupItem) * (host.copy.size() + 1) + sizeof(int) * (host.wgmap.size() + 1) +
         sizeof(int) * (host.gemmmap.size() + 1) + sizeof(int) * (host.atbmap.size() + 1);
}

template <class T>
hipError_t upload(T* d, const std::vector<T>& v, hipStream_t s) {
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s);
}

hipError_t launch_qr_group(const QrLaunch& L, const GroupDev& D, double fl, hipStream_t s) {
  PanelQrTask* tasks = D.desc + L.d0;
  const int* map = D.map + L.m0;
  HSDM_LAUNCH(fill_nan_group_kernel, dim3(64, L.nd), dim3(256), 0, s, tasks);
  HSDM_TRY(hipGetLastError());
  void* args[] = {(void*)&tasks, (void*)&map};
  return coop_launch("panel_qr_group_kernel<32>", fl, 0.0, false, true,
                     (const void*)panel_qr_group_kernel<32>, dim3(L.nwg), dim3(NT), args, s);
}

hipError_t launch_gemm(const GemmLaunch& L, const GroupDev& D, hipStream_t s) {
  if (L.nd == 0) return hipSuccess;
  return gemm_group_launch(L.kind, D.gemm + L.d0, L.nd, D.gemmmap + L.m0, L.nwg, L.max_tot,
                           L.split, L.flops, s);
}

hipError_t launch_atb(const AtbLaunch& L, const GroupDev& D, hipStream_t s) {
  if (L.nd == 0) return hipSuccess;
  HSDM_LAUNCH((atb_partial_group_kernel<32>), dim3(L.nwg), dim3(NT), 0, s, D.atb + L.d0,
                     (const int*)(D.atbmap + L.m0));
  HSDM_TRY(hipGetLastError());
  HSDM_LAUNCH((atb_reduce_group_kernel<32>), dim3(ceil_div(32 * 32, 256), L.nd), dim3(256),
                     0, s, (const AtbGroupItem*)(D.atb + L.d0));
  return hipGetLastError();
}

hipError_t launch_copy(const CopyLaunch& L, const GroupDev& D, hipStream_t s) {
  if (L.nd == 0 || L.max_tot <= 0) return hipSuccess;
  const int bx = (int)std::max(1L, std::min(256L, (L.max_tot + 1023) / 1024));
  HSDM_LAUNCH(copy_group_kernel, dim3(bx, L.nd), dim3(256), 0, s,
                     (const CopyGroupItem*)(D.copy + L.d0));
  return hipGetLastError();
}

}  // namespace

size_t sy2sb_group_bytes(int nt, const Sy2sbArgs* t, int B, Sy2sbGroupHost& host) {
  std::vector<Sy2sb> R;
  for (int i = 0; i < nt; i++) R.emplace_back(t[i], B, nullptr);
  std::vector<Round> S;
  build_schedule(R, host, S);
  return group_bytes(host);
}

hipError_t sy2sb_run_group(int nt, const Sy2sbArgs* t, int B, Sy2sbGroupHost& host, void* d_buf,
                           hipStream_t s) {
  if (B != 32) return hipErrorInvalidValue;
  std::vector<Sy2sb> R;
  for (int i = 0; i < nt; i++) R.emplace_back(t[i], B, s);
  std::vector<Round> S;
  build_schedule(R, host, S);
  const GroupDev D = group_dev(d_buf, host);
  HSDM_TRY(upload(D.desc, host.desc, s));
  HSDM_TRY(upload(D.gemm, host.gemm, s));
  HSDM_TRY(upload(D.atb, host.atb, s));
  HSDM_TRY(upload(D.copy, host.copy, s));
  HSDM_TRY(upload(D.map, host.wgmap, s));
  HSDM_TRY(upload(D.gemmmap, host.gemmmap, s));
  HSDM_TRY(upload(D.atbmap, host.atbmap, s));
  auto qr_flops = [&](const QrLaunch& L) {
    double f = 0.0;
    for (int i = 0; i < L.nd; i++) f += 2.0 * host.desc[L.d0 + i].h * B * B;
    return f;
  };
  for (const Round& rd : S) {
    for (const QrLaunch& L : rd.qr1) HSDM_TRY(launch_qr_group(L, D, qr_flops(L), s));
    HSDM_TRY(launch_gemm(rd.pre1, D, s));
    HSDM_TRY(launch_gemm(rd.tril1, D, s));
    HSDM_TRY(launch_gemm(rd.slt1, D, s));
    HSDM_TRY(launch_atb(rd.atb1, D, s));
    HSDM_TRY(launch_gemm(rd.fix1, D, s));
    HSDM_TRY(launch_copy(rd.cp1, D, s));
    HSDM_TRY(launch_gemm(rd.syr1, D, s));
    HSDM_TRY(launch_gemm(rd.col1, D, s));
    for (const QrLaunch& L : rd.qr2) HSDM_TRY(launch_qr_group(L, D, qr_flops(L), s));
    HSDM_TRY(launch_gemm(rd.pre2, D, s));
    HSDM_TRY(launch_gemm(rd.tril2, D, s));
    HSDM_TRY(launch_gemm(rd.slt2, D, s));
    HSDM_TRY(launch_gemm(rd.corr1, D, s));
    HSDM_TRY(launch_gemm(rd.corr2, D, s));
    HSDM_TRY(launch_atb(rd.atb2, D, s));
    HSDM_TRY(launch_gemm(rd.fix2, D, s));
    HSDM_TRY(launch_copy(rd.cp2, D, s));
    HSDM_TRY(launch_gemm(rd.syr2, D, s));
  }
  for (auto& r : R) HSDM_TRY(r.finish());
  return hipSuccess;
}

// ---- the refined form's reduction -------------------------------------------
// The same reduction with the trailing updates in FP32 on the matrix cores:
// A (lower triangle) is held in FP32; each panel is copied to FP64 for its
// Householder QR (the panel step is latency-bound, so its precision costs
// nothing), the explicit reflectors go to Vst and T1 in FP64 as in the FP64
// reduction, and their FP32 roundings (V32, the panel's T) drive the two-sided
// update of the trailing block, one panel at a time:
//   Y = V T,  X = A22 Y,  M = Y^T X,  W = X - V M / 2,  A22 <- A22 - [V W][W V]^T.
// The result is the band of a matrix within FP32 rounding of an orthogonal
// similarity of A; the refinement that follows the eigensolve restores FP64
// accuracy against the FP64 standard-form matrix.
namespace {

__global__ void band_extract_f32_kernel(int n, int B, const float* A, long lda, double* AB,
                                        int ldab) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * ldab) return;
  const int off = (int)(idx % ldab), c = (int)(idx / ldab);
  const int r = c + off;
  AB[idx] = (off <= B && r < n) ? (double)A[r + (long)c * lda] : 0.0;
}

constexpr int F32_MCHUNK = 1024;  // K slice of M = Y^T X

struct Sy2sbF32Layout {
  double *P64, *part, *prow, *gpart;
  float *T32, *Y, *VW, *WV, *M, *mpart, *sk1, *sk2;
  size_t bytes;
};

Sy2sbF32Layout f32_layout(int n, int B, char* base) {
  const int Gmax = ceil_div(n, CH) + 1;
  const size_t nsplit = ceil_div(n, SPLITK) + 1;
  const size_t msplit = ceil_div(n, F32_MCHUNK) + 1;
  Sy2sbF32Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  L.P64 = (double*)take(sizeof(double) * n * B);
  // part, prow, gpart contiguous (reset to NaN together)
  L.part = (double*)take(sizeof(double) * ((size_t)B * Gmax * B + (size_t)B * B +
                                           (size_t)Gmax * B * B));
  L.prow = L.part ? L.part + (size_t)B * Gmax * B : nullptr;
  L.gpart = L.prow ? L.prow + (size_t)B * B : nullptr;
  L.T32 = (float*)take(sizeof(float) * B * B);
  L.Y = (float*)take(sizeof(float) * n * B);
  L.VW = (float*)take(sizeof(float) * n * 2 * B);
  L.WV = (float*)take(sizeof(float) * n * 2 * B);
  L.M = (float*)take(sizeof(float) * B * B);
  L.mpart = (float*)take(sizeof(float) * msplit * B * B);
  L.sk1 = (float*)take(sizeof(float) * nsplit * n * B);
  L.sk2 = (float*)take(sizeof(float) * nsplit * n * B);
  L.bytes = off;
  return L;
}

}  // namespace

size_t sy2sb_f32_scratch_bytes(int n, int B) { return f32_layout(n, B, nullptr).bytes; }

hipError_t sy2sb_f32_run(int n, int B, float* A, long lda, double* Vst, long ldv, float* V32,
                         long ldv32, double* tau1, double* T1, double* AB, int ldab,
                         void* scratch, DevStatusWord* st, hipStream_t s) {
  if (B != 32) return hipErrorInvalidValue;
  const Sy2sbF32Layout L = f32_layout(n, B, (char*)scratch);
  const int np = (n > B) ? ceil_div(n - 1, B) : 0;
  for (int p = 0; p < np; p++) {
    const int c0 = p * B, r0 = c0 + B, h = n - r0;
    if (h <= 0) break;
    // the panel's QR in FP64
    HSDM_TRY(dev_convert(A + r0 + (long)c0 * lda, lda, L.P64, n, h, B, s));
    PanelQrTask q{};
    q.P = L.P64; q.ldp = n;
    q.V = Vst + r0 + (long)c0 * ldv; q.ldv = ldv;
    q.tau = tau1 + c0;
    q.T = T1 + (size_t)p * B * B;
    q.part = L.part; q.prow = L.prow; q.gpart = L.gpart; q.st = st;
    q.h = h;
    q.G = ceil_div(h, CH);
    q.span = q.G > 1 ? (long)(L.gpart - L.part) + (long)B * B * q.G : 0;
    HSDM_TRY(run_panel_qr(q, s));
    HSDM_TRY(dev_convert(L.P64, n, A + r0 + (long)c0 * lda, lda, h, B, s));  // R for the band
    // the whole column block: the zeros above the panel's first reflector
    // row are part of the grouped reflectors of the back-transform
    HSDM_TRY(dev_convert(Vst + (long)c0 * ldv, ldv, V32 + (long)c0 * ldv32, ldv32, n, B, s));
    float* Vp = V32 + r0 + (long)c0 * ldv32;
    HSDM_TRY(dev_convert(q.T, B, L.T32, B, B, B, s));
    if (h <= 1) continue;
    float* A22 = A + r0 + (long)r0 * lda;
    float* W = L.VW + (size_t)n * B;  // X, then W, in place in [V W]
    GemmArgsF g{};
    g.m = h; g.n = B; g.k = B; g.A = Vp; g.lda = ldv32; g.B = L.T32; g.ldb = B; g.C = L.Y;
    g.ldc = n; g.alpha = 1.0; g.beta = 0.0; g.flags = GF_KB_UPPER;
    HSDM_TRY(gemm_launch(g, s));
    GemmArgsF t{};
    t.m = h; t.n = B; t.k = h; t.A = A22; t.lda = lda; t.B = L.Y; t.ldb = n; t.C = W; t.ldc = n;
    t.alpha = 1.0; t.beta = 0.0; t.flags = GF_A_TRIL | GF_KA_LOWER;
    if (h > SPLITK) {
      HSDM_TRY(gemm_sym_pair_launch(t, SPLITK, L.sk1, L.sk2, s));
    } else {
      HSDM_TRY(gemm_splitk_launch(t, SPLITK, L.sk1, s));
      GemmArgsF u = t;
      u.ta = 1; u.beta = 1.0; u.flags = GF_A_SLT | GF_KA_UPPER;
      HSDM_TRY(gemm_splitk_launch(u, SPLITK, L.sk1, s));
    }
    g = GemmArgsF{};
    g.m = B; g.n = B; g.k = h; g.A = L.Y; g.lda = n; g.B = W; g.ldb = n; g.C = L.M; g.ldc = B;
    g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0;
    HSDM_TRY(gemm_splitk_launch(g, F32_MCHUNK, L.mpart, s));
    g = GemmArgsF{};
    g.m = h; g.n = B; g.k = B; g.A = Vp; g.lda = ldv32; g.B = L.M; g.ldb = B; g.C = W; g.ldc = n;
    g.alpha = -0.5; g.beta = 1.0;
    HSDM_TRY(gemm_launch(g, s));
    HSDM_TRY(file_vw(h, B, (const float*)Vp, ldv32, (const float*)W, (long)n, L.VW, L.WV,
                     L.WV + (size_t)n * B, (long)n, s));
    g = GemmArgsF{};
    g.m = h; g.n = h; g.k = 2 * B; g.A = L.VW; g.lda = n; g.B = L.WV; g.ldb = n; g.C = A22;
    g.ldc = lda; g.alpha = -1.0; g.beta = 1.0; g.ta = 0; g.tb = 1;
    g.flags = GF_C_LOWER_TILES | GF_C_LOWER_ONLY;
    HSDM_TRY(gemm_launch(g, s));
  }
  const long tot = (long)n * ldab;
  HSDM_LAUNCH(band_extract_f32_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n,
              B, A, lda, AB, ldab);
  return hipGetLastError();
}
