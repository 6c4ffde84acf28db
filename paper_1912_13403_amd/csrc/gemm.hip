// FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
// Every dense contraction of the path runs through this kernel: the
// Cholesky/inverse recursion, the standard-form products, the two-sided
// full-to-band update, the divide-and-conquer merges and the
// back-transforms.  Tiles of BM x BN outputs per 256-thread workgroup
// (4 wavefronts in a 2x2 grid, each owning (BM/2) x (BN/2)), K staged
// through LDS in slices of 16 with register prefetch of the next slice
// (double-buffered LDS).  Tile order is XCD-aware: consecutive workgroup ids
// are dealt round-robin over the 8 XCDs, so ids are remapped such that each
// XCD owns a contiguous run of tiles, walked in groups of 8 tile-rows to keep
// the A and B panels of one XCD inside its own L2.
#include "hsdm_internal.h"

namespace {

constexpr int NT = 256;
constexpr int BK = 16;
constexpr int PAD = 4;

template <int BM, int BN>
struct Cfg {
  static constexpr int WM = BM / 2, WN = BN / 2;
  static constexpr int FM = WM / 16, FN = WN / 16;
  static constexpr int LDA_S = BM + PAD, LDB_S = BN + PAD;
  static constexpr int AE = BM * BK / NT;  // A elements staged per thread
  static constexpr int BE = BN * BK / NT;
};

struct Prob {
  int m, n, k;
  const double* A; long lda;
  const double* B; long ldb;
  double* C; long ldc;
  const int* acol;
  const int* ccol;
  const int* ndev;  // optional device-side column count (n is then an upper bound)
};

// Load element (i, kk) of op(A) into a register, zero outside [0,m)x[kb,ke).
template <int BM, int BN>
HSDM_DEV void load_a(const Prob& p, int ta, int flags, int i0, int k0, int kb, int ke,
                     double (&r)[Cfg<BM, BN>::AE]) {
  const int t = threadIdx.x;
  constexpr int AE = Cfg<BM, BN>::AE;
  if (flags & GF_A_SYM_LOWER) {
    // symmetric A, lower triangle stored; choose a coalesced pattern per tile
    const bool all_lower = i0 >= k0 + BK - 1;
    const bool all_upper = i0 + BM - 1 < k0;
    if (all_upper) {
      // element (i,kk) = A[kk + i*lda]: contiguous along kk
#pragma unroll
      for (int q = 0; q < AE; q++) {
        int kk = k0 + (t % BK), i = i0 + t / BK + q * (NT / BK);
        r[q] = (i < p.m && kk >= kb && kk < ke) ? p.A[kk + (long)i * p.lda] : 0.0;
      }
    } else {
#pragma unroll
      for (int q = 0; q < AE; q++) {
        int i = i0 + (t % BM), kk = k0 + t / BM + q * (NT / BM);
        double v = 0.0;
        if (i < p.m && kk >= kb && kk < ke)
          v = (all_lower || i >= kk) ? p.A[i + (long)kk * p.lda] : p.A[kk + (long)i * p.lda];
        r[q] = v;
      }
    }
    return;
  }
  if (ta == 0) {
#pragma unroll
    for (int q = 0; q < AE; q++) {
      int i = i0 + (t % BM), kk = k0 + t / BM + q * (NT / BM);
      double v = 0.0;
      if (i < p.m && kk >= kb && kk < ke) {
        long col = p.acol ? (long)p.acol[kk] : (long)kk;
        v = p.A[i + col * p.lda];
      }
      r[q] = v;
    }
  } else {
#pragma unroll
    for (int q = 0; q < AE; q++) {
      int kk = k0 + (t % BK), i = i0 + t / BK + q * (NT / BK);
      r[q] = (i < p.m && kk >= kb && kk < ke) ? p.A[kk + (long)i * p.lda] : 0.0;
    }
  }
}

template <int BM, int BN>
HSDM_DEV void store_a(int ta, int flags, int i0, int k0, double* As,
                      const double (&r)[Cfg<BM, BN>::AE]) {
  const int t = threadIdx.x;
  constexpr int AE = Cfg<BM, BN>::AE, LD = Cfg<BM, BN>::LDA_S;
  bool trans_pattern = (ta != 0);
  if (flags & GF_A_SYM_LOWER) trans_pattern = (i0 + BM - 1 < k0);
  if (!trans_pattern) {
#pragma unroll
    for (int q = 0; q < AE; q++) As[(t / BM + q * (NT / BM)) * LD + (t % BM)] = r[q];
  } else {
#pragma unroll
    for (int q = 0; q < AE; q++) As[(t % BK) * LD + t / BK + q * (NT / BK)] = r[q];
  }
}

template <int BM, int BN>
HSDM_DEV void load_b(const Prob& p, int tb, int j0, int k0, int kb, int ke,
                     double (&r)[Cfg<BM, BN>::BE]) {
  const int t = threadIdx.x;
  constexpr int BE = Cfg<BM, BN>::BE;
  if (tb == 0) {
    // op(B)[kk, j] = B[kk + j*ldb]: contiguous along kk
#pragma unroll
    for (int q = 0; q < BE; q++) {
      int kk = k0 + (t % BK), j = j0 + t / BK + q * (NT / BK);
      r[q] = (j < p.n && kk >= kb && kk < ke) ? p.B[kk + (long)j * p.ldb] : 0.0;
    }
  } else {
#pragma unroll
    for (int q = 0; q < BE; q++) {
      int j = j0 + (t % BN), kk = k0 + t / BN + q * (NT / BN);
      r[q] = (j < p.n && kk >= kb && kk < ke) ? p.B[j + (long)kk * p.ldb] : 0.0;
    }
  }
}

template <int BM, int BN>
HSDM_DEV void store_b(int tb, double* Bs, const double (&r)[Cfg<BM, BN>::BE]) {
  const int t = threadIdx.x;
  constexpr int BE = Cfg<BM, BN>::BE, LD = Cfg<BM, BN>::LDB_S;
  if (tb == 0) {
#pragma unroll
    for (int q = 0; q < BE; q++) Bs[(t % BK) * LD + t / BK + q * (NT / BK)] = r[q];
  } else {
#pragma unroll
    for (int q = 0; q < BE; q++) Bs[(t / BN + q * (NT / BN)) * LD + (t % BN)] = r[q];
  }
}

// Compute one BM x BN output tile.
template <int BM, int BN>
HSDM_DEV void gemm_tile(const Prob& p, double alpha, double beta, int ta, int tb, int flags,
                        int tm, int tn, double* smem, int klo = 0, int khi = 1 << 30) {
  using C = Cfg<BM, BN>;
  const int i0 = tm * BM, j0 = tn * BN;
  int kb = klo, ke = min(p.k, khi);
  if (flags & GF_KA_LOWER) ke = min(ke, i0 + BM);
  if (flags & GF_KA_UPPER) kb = max(kb, i0);
  if (flags & GF_KB_UPPER) ke = min(ke, j0 + BN);
  if (flags & GF_KB_LOWER) kb = max(kb, j0);
  const int kstart = (kb / BK) * BK;

  double* As[2] = {smem, smem + BK * C::LDA_S};
  double* Bs[2] = {smem + 2 * BK * C::LDA_S, smem + 2 * BK * C::LDA_S + BK * C::LDB_S};

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  dbl4 acc[C::FM][C::FN];
#pragma unroll
  for (int a = 0; a < C::FM; a++)
#pragma unroll
    for (int b = 0; b < C::FN; b++) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

  double ra[C::AE], rb[C::BE];
  int buf = 0;
  if (kstart < ke) {
    load_a<BM, BN>(p, ta, flags, i0, kstart, kb, ke, ra);
    load_b<BM, BN>(p, tb, j0, kstart, kb, ke, rb);
    store_a<BM, BN>(ta, flags, i0, kstart, As[0], ra);
    store_b<BM, BN>(tb, Bs[0], rb);
  }
  __syncthreads();
  for (int k0 = kstart; k0 < ke; k0 += BK) {
    const bool more = k0 + BK < ke;
    if (more) {
      load_a<BM, BN>(p, ta, flags, i0, k0 + BK, kb, ke, ra);
      load_b<BM, BN>(p, tb, j0, k0 + BK, kb, ke, rb);
    }
    const double* as = As[buf];
    const double* bs = Bs[buf];
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double fa[C::FM], fb[C::FN];
      const int kr = ks + (lane >> 4);
#pragma unroll
      for (int a = 0; a < C::FM; a++) fa[a] = as[kr * C::LDA_S + wm * C::WM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < C::FN; b++) fb[b] = bs[kr * C::LDB_S + wn * C::WN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < C::FM; a++)
#pragma unroll
        for (int b = 0; b < C::FN; b++)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    if (more) {
      store_a<BM, BN>(ta, flags, i0, k0 + BK, As[buf ^ 1], ra);
      store_b<BM, BN>(tb, Bs[buf ^ 1], rb);
    }
    __syncthreads();
    buf ^= 1;
  }

  // epilogue: accumulator register r of a lane holds row lane/16 + 4r, column
  // lane%16 of its 16x16 block
#pragma unroll
  for (int a = 0; a < C::FM; a++)
#pragma unroll
    for (int b = 0; b < C::FN; b++) {
      const int col = j0 + wn * C::WN + b * 16 + (lane & 15);
      if (col >= p.n) continue;
      const long ccol = p.ccol ? (long)p.ccol[col] : (long)col;
      double* cp = p.C + ccol * p.ldc;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = i0 + wm * C::WM + a * 16 + (lane >> 4) + 4 * r;
        if (row >= p.m) continue;
        if ((flags & GF_C_LOWER_ONLY) && row < col) continue;
        double v = alpha * acc[a][b][r];
        if (beta != 0.0) v += beta * cp[row];
        cp[row] = v;
      }
    }
}

// Map a workgroup id to a tile: XCD-contiguous runs, then groups of 8 rows.
HSDM_DEV bool map_tile(int bid, int nblk, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int per = nblk / 8;  // nblk is a multiple of 8
  const int t = (bid % 8) * per + bid / 8;
  if (t >= tiles_m * tiles_n) return false;
  constexpr int GROUP = 8;
  const int in_group = GROUP * tiles_n;
  const int g = t / in_group;
  const int first = g * GROUP;
  const int gs = min(tiles_m - first, GROUP);
  const int r = t % in_group;
  tm = first + r % gs;
  tn = r / gs;
  return true;
}

template <int BM, int BN>
constexpr int smem_doubles() {
  return 2 * BK * (Cfg<BM, BN>::LDA_S + Cfg<BM, BN>::LDB_S);
}

template <int BM, int BN>
__global__ __launch_bounds__(NT) void gemm_kernel(Prob p, double alpha, double beta, int ta,
                                                  int tb, int flags, int kchunk, long split_stride) {
  __shared__ double smem[smem_doubles<BM, BN>()];
  if (p.ndev) p.n = min(p.n, *p.ndev);
  if (p.n <= 0) return;
  const int tiles_m = (p.m + BM - 1) / BM, tiles_n = (p.n + BN - 1) / BN;
  int tm, tn;
  if (!map_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn)) return;
  if ((flags & GF_C_LOWER_TILES) && (tm + 1) * BM - 1 < tn * BN) return;
  if (kchunk > 0) {
    // split-K: slice blockIdx.y writes its partial product to C + y*split_stride
    const int klo = blockIdx.y * kchunk;
    p.C += (long)blockIdx.y * split_stride;
    gemm_tile<BM, BN>(p, alpha, 0.0, ta, tb, flags, tm, tn, smem, klo, klo + kchunk);
    return;
  }
  gemm_tile<BM, BN>(p, alpha, beta, ta, tb, flags, tm, tn, smem);
}

template <int BM, int BN>
__global__ __launch_bounds__(NT) void gemm_batched_kernel(const GemmDesc* desc, double alpha,
                                                          double beta, int ta, int tb,
                                                          int flags) {
  __shared__ double smem[smem_doubles<BM, BN>()];
  const GemmDesc d = desc[blockIdx.y];
  if (d.m <= 0 || d.n <= 0) return;
  Prob p{d.m, d.n, d.k, d.A, d.lda, d.B, d.ldb, d.C, d.ldc, d.acol, d.ccol, nullptr};
  const int tiles_m = (p.m + BM - 1) / BM, tiles_n = (p.n + BN - 1) / BN;
  int tm, tn;
  if (!map_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn)) return;
  if ((flags & GF_C_LOWER_TILES) && (tm + 1) * BM - 1 < tn * BN) return;
  if (d.k <= 0) {
    // empty contraction: C = beta * C on the tile
    const int i = tm * BM + (threadIdx.x % BM);
    for (int j = tn * BN + threadIdx.x / BM; j < min(p.n, (tn + 1) * BN); j += NT / BM) {
      if (i >= p.m) break;
      long cc = p.ccol ? (long)p.ccol[j] : (long)j;
      double* c = p.C + cc * p.ldc + i;
      *c = (beta != 0.0) ? beta * *c : 0.0;
    }
    return;
  }
  gemm_tile<BM, BN>(p, alpha, beta, ta, tb, flags, tm, tn, smem);
}

template <int BM, int BN>
hipError_t launch_single(const GemmArgs& g, hipStream_t s) {
  Prob p{g.m, g.n, g.k, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.acol, g.ccol, g.ndev};
  long tiles = (long)ceil_div(g.m, BM) * ceil_div(g.n, BN);
  int nblk = (int)(((tiles + 7) / 8) * 8);
  hipLaunchKernelGGL((gemm_kernel<BM, BN>), dim3(nblk), dim3(NT), 0, s, p,
                     g.alpha, g.beta, g.ta, g.tb, g.flags, 0, 0L);
  return hipGetLastError();
}

// sum of nsplit partial m x n products (ld m) into C: C = sum + beta C
__global__ void splitk_reduce_kernel(int m, int n, int nsplit, const double* part, double* C,
                                     long ldc, double beta, const int* ndev) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = (long)m * n;
  if (idx >= tot) return;
  if (ndev && idx / m >= *ndev) return;
  double s = 0.0;
  for (int z = 0; z < nsplit; z++) s += part[z * tot + idx];
  const int i = (int)(idx % m), j = (int)(idx / m);
  double* c = C + i + (long)j * ldc;
  *c = (beta != 0.0) ? s + beta * *c : s;
}

// C = beta*C when k == 0 (or alpha == 0)
__global__ void scale_kernel(int m, int n, double* C, long ldc, double beta, const int* ccol,
                             const int* ndev) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)m * n) return;
  int i = (int)(idx % m), j = (int)(idx / m);
  if (ndev && j >= *ndev) return;
  long cc = ccol ? (long)ccol[j] : (long)j;
  double* c = C + cc * ldc + i;
  *c = (beta != 0.0) ? beta * *c : 0.0;
}

}  // namespace

hipError_t gemm_launch(const GemmArgs& g, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0) return hipSuccess;
  if (g.k <= 0 || g.alpha == 0.0) {
    if (g.beta == 1.0) return hipSuccess;
    long tot = (long)g.m * g.n;
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, g.m,
                       g.n, g.C, g.ldc, g.beta, g.ccol, g.ndev);
    return hipGetLastError();
  }
  // Large outputs: 128x128 tiles; otherwise 64x64 to keep >= 256 workgroups.
  long big_tiles = (long)ceil_div(g.m, 128) * ceil_div(g.n, 128);
  if (big_tiles >= 512) return launch_single<128, 128>(g, s);
  return launch_single<64, 64>(g, s);
}

hipError_t gemm_splitk_launch(const GemmArgs& g, int kchunk, double* part, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0) return hipSuccess;
  if (g.k <= kchunk || kchunk <= 0) return gemm_launch(g, s);
  if (g.ccol || (g.flags & (GF_C_LOWER_ONLY | GF_C_LOWER_TILES))) return hipErrorInvalidValue;
  const int nsplit = ceil_div(g.k, kchunk);
  Prob p{g.m, g.n, g.k, g.A, g.lda, g.B, g.ldb, part, (long)g.m, g.acol, nullptr, g.ndev};
  const long stride = (long)g.m * g.n;
  long tiles = (long)ceil_div(g.m, 64) * ceil_div(g.n, 64);
  int nblk = (int)(((tiles + 7) / 8) * 8);
  hipLaunchKernelGGL((gemm_kernel<64, 64>), dim3(nblk, nsplit), dim3(NT), 0, s, p, g.alpha, 0.0,
                     g.ta, g.tb, g.flags, kchunk, stride);
  HSDM_TRY(hipGetLastError());
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((stride + 255) / 256)), dim3(256), 0, s,
                     g.m, g.n, nsplit, part, g.C, g.ldc, g.beta, g.ndev);
  return hipGetLastError();
}

hipError_t gemm_batched_launch(const GemmDesc* d_desc, int count, int max_m, int max_n,
                               double alpha, double beta, int ta, int tb, int flags,
                               hipStream_t s) {
  if (count <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  long tiles = (long)ceil_div(max_m, 64) * ceil_div(max_n, 64);
  int nblk = (int)(((tiles + 7) / 8) * 8);
  hipLaunchKernelGGL((gemm_batched_kernel<64, 64>), dim3(nblk, count), dim3(NT), 0, s,
                     d_desc, alpha, beta, ta, tb, flags);
  return hipGetLastError();
}
