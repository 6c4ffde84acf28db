// GEMM on CDNA4 matrix cores: FP64 (v_mfma_f64_16x16x4f64) and, for the
// refined form, FP32 (v_mfma_f32_16x16x4f32, the same 16 x 16 x 4 shape and
// operand layout; only the rows an accumulator register holds differ).
//
// Every dense contraction of the path runs through this kernel: the
// Cholesky/inverse recursion, the standard-form products, the two-sided
// full-to-band update, the divide-and-conquer merges and the
// back-transforms.
//
// A workgroup computes a BM x BN tile with WM x WN wavefronts, each owning a
// (BM/WM) x (BN/WN) sub-tile of 16x16 MFMA blocks.  K is staged through LDS
// in slices of 16 with register prefetch of the next slice (double-buffered
// LDS, one barrier per slice).  Each operand keeps in LDS the orientation it
// has in memory, so global loads are coalesced and LDS stores are
// conflict-free: a row-contiguous tile is stored [k][row] with a row stride
// of (BM + 16) doubles, a k-contiguous tile [row][k] with stride 17; both
// make the MFMA operand reads conflict-free.  Loads are branch-free (clamped
// addresses, masked values).  Tile order is XCD-aware: workgroup ids are
// dealt round-robin over the 8 XCDs, so ids are remapped such that each XCD
// owns a contiguous run of tiles, walked in groups of 8 tile-rows so that the
// A and B panels of one XCD stay in its L2.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "hsdm_internal.h"

namespace {

constexpr int BK = 16;

// A operand modes
constexpr int AM_DENSE = 0;
constexpr int AM_SYM = 1;     // symmetric A, lower triangle stored (TA = 0)
constexpr int AM_GATHER = 2;  // op(A)[:, kk] = A[:, acol[kk]] (TA = 0)
constexpr int AM_TRIL = 3;    // op(A) = lower triangle of A, diagonal included (TA = 0)
constexpr int AM_SLT = 4;     // op(A) = (strict lower triangle of A)^T (TA = 1)

template <class T>
struct ProbT {
  int m, n, k;
  const T* A; long lda;
  const T* B; long ldb;
  T* C; long ldc;
  const int* acol;
  const int* ccol;
  const int* ndev;  // optional device-side column count (n is then an upper bound)
};
using Prob = ProbT<double>;

// The 16 x 16 x 4 matrix-core step per element type.  Operands: lane l holds
// op(A)[l % 16][l / 16] and op(B)[l / 16][l % 16]; accumulator register r
// of lane l holds column l % 16 and row row(l / 16, r) of the block.
template <class T>
struct Mf;
template <>
struct Mf<double> {
  using acc = dbl4;
  static HSDM_DEV acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  static HSDM_DEV acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static HSDM_DEV int row(int l4, int r) { return l4 + 4 * r; }
};
template <>
struct Mf<float> {
  using acc = flt4;
  static HSDM_DEV acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  static HSDM_DEV acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static HSDM_DEV int row(int l4, int r) { return 4 * l4 + r; }
};

template <int BM, int BN, int WM, int WN, int TA, int TB, int AM>
struct G {
  static constexpr int NT = 64 * WM * WN;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int FM = WTM / 16, FN = WTN / 16;
  static constexpr bool A_KC = (TA == 1);  // A tile stored [row][k]
  static constexpr bool B_KC = (TB == 0);  // B tile stored [col][k]
  static constexpr int LDA = A_KC ? (BK + 1) : (BM + 16);
  static constexpr int LDB = B_KC ? (BK + 1) : (BN + 16);
  static constexpr int ASZ = A_KC ? BM * (BK + 1) : BK * (BM + 16);
  static constexpr int BSZ = B_KC ? BN * (BK + 1) : BK * (BN + 16);
  static constexpr int AE = BM * BK / NT;
  static constexpr int BE = BN * BK / NT;
  static constexpr int SMEM = 2 * (ASZ + BSZ);
  static constexpr int BMc = BM, BNc = BN;
  static constexpr bool PF2 = (BM <= 32) || (BN <= 32);
  static_assert(AE >= 1 && BE >= 1, "tile too small for the thread count");
  static_assert(FM >= 1 && FN >= 1, "wave tile below one MFMA block");
};

// ---- global -> registers ------------------------------------------------------
template <class C, int TA, int AM, class T>
HSDM_DEV void load_a(const ProbT<T>& p, int i0, int k0, int kb, int ke, T (&r)[C::AE]) {
  const int t = threadIdx.x;
  if constexpr (TA == 1) {
    // op(A)[i, kk] = A[kk + i*lda]: k-contiguous
#pragma unroll
    for (int q = 0; q < C::AE; q++) {
      const int kk = k0 + (t % BK), i = i0 + t / BK + q * (C::NT / BK);
      bool ok = (i < p.m) && (kk >= kb) && (kk < ke);
      if constexpr (AM == AM_SLT) ok = ok && (kk > i);
      const int ic = min(i, p.m - 1), kc = min(max(kk, kb), ke - 1);
      const T v = p.A[kc + (long)ic * p.lda];
      r[q] = ok ? v : T(0);
    }
  } else {
    constexpr int RS = C::NT / C::BMc;  // k columns per pass
#pragma unroll
    for (int q = 0; q < C::AE; q++) {
      const int i = i0 + (t % C::BMc), kk = k0 + t / C::BMc + q * RS;
      bool ok = (i < p.m) && (kk >= kb) && (kk < ke);
      if constexpr (AM == AM_TRIL) ok = ok && (i >= kk);
      const int ic = min(i, p.m - 1), kc = min(max(kk, kb), ke - 1);
      long addr;
      if constexpr (AM == AM_SYM) {
        addr = (ic >= kc) ? ic + (long)kc * p.lda : kc + (long)ic * p.lda;
      } else if constexpr (AM == AM_GATHER) {
        addr = ic + (long)p.acol[kc] * p.lda;
      } else {
        addr = ic + (long)kc * p.lda;
      }
      const T v = p.A[addr];
      r[q] = ok ? v : T(0);
    }
  }
}

template <class C, int TA, class T>
HSDM_DEV void store_a(T* As, const T (&r)[C::AE]) {
  const int t = threadIdx.x;
  if constexpr (TA == 1) {
#pragma unroll
    for (int q = 0; q < C::AE; q++) As[(t / BK + q * (C::NT / BK)) * C::LDA + (t % BK)] = r[q];
  } else {
    constexpr int RS = C::NT / C::BMc;
#pragma unroll
    for (int q = 0; q < C::AE; q++) As[(t / C::BMc + q * RS) * C::LDA + t % C::BMc] = r[q];
  }
}

template <class C, int TB, class T>
HSDM_DEV void load_b(const ProbT<T>& p, int j0, int k0, int kb, int ke, T (&r)[C::BE]) {
  const int t = threadIdx.x;
  if constexpr (TB == 0) {
    // op(B)[kk, j] = B[kk + j*ldb]: k-contiguous
#pragma unroll
    for (int q = 0; q < C::BE; q++) {
      const int kk = k0 + (t % BK), j = j0 + t / BK + q * (C::NT / BK);
      const bool ok = (j < p.n) && (kk >= kb) && (kk < ke);
      const int jc = min(j, p.n - 1), kc = min(max(kk, kb), ke - 1);
      const T v = p.B[kc + (long)jc * p.ldb];
      r[q] = ok ? v : T(0);
    }
  } else {
    constexpr int RS = C::NT / C::BNc;
#pragma unroll
    for (int q = 0; q < C::BE; q++) {
      const int j = j0 + (t % C::BNc), kk = k0 + t / C::BNc + q * RS;
      const bool ok = (j < p.n) && (kk >= kb) && (kk < ke);
      const int jc = min(j, p.n - 1), kc = min(max(kk, kb), ke - 1);
      const T v = p.B[jc + (long)kc * p.ldb];
      r[q] = ok ? v : T(0);
    }
  }
}

template <class C, int TB, class T>
HSDM_DEV void store_b(T* Bs, const T (&r)[C::BE]) {
  const int t = threadIdx.x;
  if constexpr (TB == 0) {
#pragma unroll
    for (int q = 0; q < C::BE; q++) Bs[(t / BK + q * (C::NT / BK)) * C::LDB + (t % BK)] = r[q];
  } else {
    constexpr int RS = C::NT / C::BNc;
#pragma unroll
    for (int q = 0; q < C::BE; q++) Bs[(t / C::BNc + q * RS) * C::LDB + t % C::BNc] = r[q];
  }
}

// ---- one output tile -------------------------------------------------------------
template <int BM, int BN, int WM, int WN, int TA, int TB, int AM, class T>
HSDM_DEV void gemm_tile(const ProbT<T>& p, double alpha, double beta, int flags, int tm, int tn,
                        T* smem, int klo, int khi) {
  using C = G<BM, BN, WM, WN, TA, TB, AM>;
  const int i0 = tm * BM, j0 = tn * BN;
  int kb = klo, ke = min(p.k, khi);
  if (flags & GF_KA_LOWER) ke = min(ke, i0 + BM);
  if (flags & GF_KA_UPPER) kb = max(kb, i0);
  if (flags & GF_KB_UPPER) ke = min(ke, j0 + BN);
  if (flags & GF_KB_LOWER) kb = max(kb, j0);
  const int kstart = (kb / BK) * BK;

  T* As0 = smem;
  T* As1 = smem + C::ASZ;
  T* Bs0 = smem + 2 * C::ASZ;
  T* Bs1 = Bs0 + C::BSZ;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int l16 = lane & 15, l4 = lane >> 4;

  using M = Mf<T>;
  typename M::acc acc[C::FM][C::FN];
  // With alpha = +-1 the accumulators start from (beta / alpha) C, exact in
  // the element type, so the C tile is read while the first A and B slices
  // load instead of after the contraction.
  const bool cinit = (beta != 0.0) && (alpha == 1.0 || alpha == -1.0);
  if (cinit) {
    const T sc = (T)(beta * alpha);  // beta / alpha for alpha = +-1
#pragma unroll
    for (int b = 0; b < C::FN; b++) {
      const int col = j0 + wn * C::WTN + b * 16 + l16;
      const bool cok = col < p.n;
      const long cc = cok ? (p.ccol ? (long)p.ccol[col] : (long)col) : 0L;
      const T* cp = p.C + cc * p.ldc;
#pragma unroll
      for (int a = 0; a < C::FM; a++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int row = i0 + wm * C::WTM + a * 16 + M::row(l4, r);
          bool ok = cok && row < p.m;
          if (flags & GF_C_LOWER_ONLY) ok = ok && row >= col;
          const T v = cp[min(row, p.m - 1)];  // in bounds for every lane
          acc[a][b][r] = ok ? sc * v : T(0);
        }
    }
  } else {
#pragma unroll
    for (int a = 0; a < C::FM; a++)
#pragma unroll
      for (int b = 0; b < C::FN; b++) acc[a][b] = M::zero();
  }

  // one K slice of the staged tiles: 4 MFMA steps over BK
  auto compute = [&](const T* as, const T* bs) {
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + l4;
      T fa[C::FM], fb[C::FN];
#pragma unroll
      for (int a = 0; a < C::FM; a++) {
        const int row = wm * C::WTM + a * 16 + l16;
        fa[a] = C::A_KC ? as[row * C::LDA + kr] : as[kr * C::LDA + row];
      }
#pragma unroll
      for (int b = 0; b < C::FN; b++) {
        const int col = wn * C::WTN + b * 16 + l16;
        fb[b] = C::B_KC ? bs[col * C::LDB + kr] : bs[kr * C::LDB + col];
      }
#pragma unroll
      for (int a = 0; a < C::FM; a++)
#pragma unroll
        for (int b = 0; b < C::FN; b++)
          acc[a][b] = M::mma(fa[a], fb[b], acc[a][b]);
    }
  };
  // A tile that lies wholly inside its operands stages the slices that need
  // no masking with no per-slice address arithmetic: element q of a thread
  // sits at a fixed byte offset from a base that is the same for the whole
  // workgroup (the slice's corner plus q times a uniform stride).  For a
  // triangular operand these are the slices on the stored side of the
  // tile's diagonal block.
  constexpr bool PLAIN =
      (AM == AM_DENSE) || (AM == AM_TRIL) || (AM == AM_SLT) || (AM == AM_GATHER && TA == 0);
  const bool whole = PLAIN && (i0 + BM <= p.m) && (j0 + BN <= p.n) &&
                     (p.lda < (1L << 22)) && (p.ldb < (1L << 22));
  const int tid = threadIdx.x;
  const unsigned oa = (unsigned)(sizeof(T) * (TA == 0 ? (tid % BM) + (long)(tid / BM) * p.lda
                                                       : (tid % BK) + (long)(tid / BK) * p.lda));
  const unsigned ob = (unsigned)(sizeof(T) * (TB == 0 ? (tid % BK) + (long)(tid / BK) * p.ldb
                                                       : (tid % BN) + (long)(tid / BN) * p.ldb));
  const long sa = (long)sizeof(T) * (TA == 0 ? (C::NT / BM) : (C::NT / BK)) * p.lda;
  const long sb = (long)sizeof(T) * (TB == 0 ? (C::NT / BK) : (C::NT / BN)) * p.ldb;
  auto plain = [&](int k) {
    if (!whole || k < kb || k + BK > ke) return false;
    if constexpr (AM == AM_TRIL) return k + BK - 1 <= i0;  // every k <= every row
    if constexpr (AM == AM_SLT) return k >= i0 + BM;       // every k > every row
    return true;
  };
  auto stage = [&](int k, T (&xa)[C::AE], T (&xb)[C::BE]) {
    if (plain(k)) {
      const char* a = (const char*)(TA == 0 ? p.A + i0 + (long)k * p.lda
                                            : p.A + k + (long)i0 * p.lda);
      const char* b = (const char*)(TB == 0 ? p.B + k + (long)j0 * p.ldb
                                            : p.B + j0 + (long)k * p.ldb);
      if constexpr (AM == AM_GATHER) {
        // column k + kk of op(A) is column acol[k + kk] of A
        const char* ai = (const char*)(p.A + i0) + sizeof(T) * (tid % BM);
#pragma unroll
        for (int q = 0; q < C::AE; q++) {
          const int kk = k + tid / BM + q * (C::NT / BM);
          xa[q] = *(const T*)(ai + (long)sizeof(T) * p.acol[kk] * p.lda);
        }
      } else {
#pragma unroll
        for (int q = 0; q < C::AE; q++) xa[q] = *(const T*)(a + q * sa + oa);
      }
#pragma unroll
      for (int q = 0; q < C::BE; q++) xb[q] = *(const T*)(b + q * sb + ob);
    } else {
      load_a<C, TA, AM>(p, i0, k, kb, ke, xa);
      load_b<C, TB>(p, j0, k, kb, ke, xb);
    }
  };
  T ra[C::AE], rb[C::BE];
  if constexpr (C::PF2) {
    // skinny tiles carry little work per slice: the registers hold two
    // slices ahead.  Loads are unconditional (past the last slice the last
    // one is loaded again and not used) so that every wait can be exact.
    const int nsl = (kstart < ke) ? (ke - kstart + BK - 1) / BK : 0;
    auto ks_of = [&](int j) { return kstart + BK * min(j, nsl - 1); };
    T ra2[C::AE], rb2[C::BE];
    if (nsl > 0) {
      stage(ks_of(0), ra, rb);
      store_a<C, TA>(As0, ra);
      store_b<C, TB>(Bs0, rb);
      stage(ks_of(1), ra2, rb2);
    }
    __syncthreads();
    for (int j = 0; j < nsl; j += 2) {
      // As0/Bs0: slice j; ra2/rb2: slice j+1 in flight
      stage(ks_of(j + 2), ra, rb);
      compute(As0, Bs0);
      store_a<C, TA>(As1, ra2);
      store_b<C, TB>(Bs1, rb2);
      __syncthreads();
      if (j + 1 >= nsl) break;
      stage(ks_of(j + 3), ra2, rb2);
      compute(As1, Bs1);
      store_a<C, TA>(As0, ra);
      store_b<C, TB>(Bs0, rb);
      __syncthreads();
    }
  } else {
    if (kstart < ke) {
      stage(kstart, ra, rb);
      store_a<C, TA>(As0, ra);
      store_b<C, TB>(Bs0, rb);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = kstart; k0 < ke; k0 += BK) {
      const bool more = k0 + BK < ke;
      if (more) stage(k0 + BK, ra, rb);
      compute(buf ? As1 : As0, buf ? Bs1 : Bs0);
      if (more) {
        store_a<C, TA>(buf ? As0 : As1, ra);
        store_b<C, TB>(buf ? Bs0 : Bs1, rb);
      }
      __syncthreads();
      buf ^= 1;
    }
  }

  // epilogue: accumulator register r of a lane holds row M::row(lane / 16, r),
  // column lane % 16 of its 16 x 16 block
#pragma unroll
  for (int a = 0; a < C::FM; a++)
#pragma unroll
    for (int b = 0; b < C::FN; b++) {
      const int col = j0 + wn * C::WTN + b * 16 + l16;
      if (col >= p.n) continue;
      const long cc = p.ccol ? (long)p.ccol[col] : (long)col;
      T* cp = p.C + cc * p.ldc;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = i0 + wm * C::WTM + a * 16 + M::row(l4, r);
        if (row >= p.m) continue;
        if ((flags & GF_C_LOWER_ONLY) && row < col) continue;
        T v = (T)alpha * acc[a][b][r];
        if (beta != 0.0 && !cinit) v += (T)beta * cp[row];
        cp[row] = v;
      }
    }
}

// Map a workgroup id to a tile.  Workgroups are dealt to the 8 XCDs in turn
// (id % 8), so XCD x takes the tile rows x, x + 8, x + 16, ... (tile columns
// when there are more of them): triangular products, whose work grows or
// shrinks with the row, stay balanced across the XCDs.  Within an XCD the
// tiles run in groups of 8 of its rows, column by column, so that both
// operand panels are reused from its L2.  The grid may be larger than needed
// (sizes read on the device); surplus ids return false.
HSDM_DEV bool map_tile(int bid, int tiles_m, int tiles_n, int& tm, int& tn) {
  const bool by_row = tiles_m >= tiles_n;
  const int major = by_row ? tiles_m : tiles_n, minor = by_row ? tiles_n : tiles_m;
  const int x = bid % 8, li = bid / 8;
  const int lines = (major - x + 7) / 8;  // tile rows (columns) of XCD x
  if (lines <= 0 || li >= lines * minor) return false;
  constexpr int GROUP = 8;
  const int in_group = GROUP * minor;
  const int g = li / in_group;
  const int first = g * GROUP;
  const int gs = min(lines - first, GROUP);
  const int r = li % in_group;
  const int a = x + 8 * (first + r % gs), c = r / gs;
  tm = by_row ? a : c;
  tn = by_row ? c : a;
  return true;
}

// workgroups needed for a tiles_m x tiles_n grid of tiles
inline int tile_grid(long tiles_m, long tiles_n) {
  const long major = tiles_m >= tiles_n ? tiles_m : tiles_n;
  const long minor = tiles_m >= tiles_n ? tiles_n : tiles_m;
  return (int)(8 * ((major + 7) / 8) * minor);
}

// Register budgets: the 8-wavefront tiles at two workgroups per CU; the
// skinny 128 x 32 tiles (streaming a tall operand) at three, so that more
// loads are in flight (the transposed strict-lower form then spills a few
// registers and is still faster).
template <int BM, int BN, int WM, int WN, int TA, int AM>
constexpr int waves_per_eu() {
  if (WM * WN == 8 && TA == 0) return 4;
  if (BM == 128 && BN == 32) return 3;
  if (BM == 64 && BN == 64) return 4;
  return 1;
}

template <int BM, int BN, int WM, int WN, int TA, int TB, int AM, class T>
__global__ __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(waves_per_eu<BM, BN, WM, WN, TA, AM>()))) void gemm_kernel(ProbT<T> p, double alpha, double beta,
                                                            int flags, int kchunk,
                                                            long split_stride) {
  using C = G<BM, BN, WM, WN, TA, TB, AM>;
  __shared__ T smem[C::SMEM];
  if (p.ndev) p.n = min(p.n, *p.ndev);
  if (p.n <= 0) return;
  const int tiles_m = (p.m + BM - 1) / BM, tiles_n = (p.n + BN - 1) / BN;
  int tm, tn;
  if (!map_tile(blockIdx.x, tiles_m, tiles_n, tm, tn)) return;
  // a triangular operand makes the k range grow with the tile row (column):
  // the longest tiles go first, so that the launch does not end on a few
  // of them
  if (flags & GF_KA_LOWER) tm = tiles_m - 1 - tm;
  if (flags & GF_KB_UPPER) tn = tiles_n - 1 - tn;
  if ((flags & GF_C_LOWER_TILES) && (tm + 1) * BM - 1 < tn * BN) return;
  if (kchunk > 0) {
    // split-K: slice blockIdx.y writes its partial product to C + y*split_stride
    const int klo = blockIdx.y * kchunk;
    p.C += (long)blockIdx.y * split_stride;
    gemm_tile<BM, BN, WM, WN, TA, TB, AM>(p, alpha, 0.0, flags, tm, tn, smem, klo, klo + kchunk);
    return;
  }
  gemm_tile<BM, BN, WM, WN, TA, TB, AM>(p, alpha, beta, flags, tm, tn, smem, 0, 1 << 30);
}

template <int BM, int BN, int WM, int WN, int TA, int TB, int AM>
__global__ __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(waves_per_eu<BM, BN, WM, WN, TA, AM>()))) void gemm_batched_kernel(const GemmDesc* desc,
                                                                    double alpha, double beta,
                                                                    int flags) {
  using C = G<BM, BN, WM, WN, TA, TB, AM>;
  __shared__ double smem[C::SMEM];
  const GemmDesc d = desc[blockIdx.y];
  if (d.m <= 0 || d.n <= 0) return;
  Prob p{d.m, d.n, d.k, d.A, d.lda, d.B, d.ldb, d.C, d.ldc, d.acol, d.ccol, nullptr};
  const int tiles_m = (p.m + BM - 1) / BM, tiles_n = (p.n + BN - 1) / BN;
  int tm, tn;
  if (!map_tile(blockIdx.x, tiles_m, tiles_n, tm, tn)) return;
  if ((flags & GF_C_LOWER_TILES) && (tm + 1) * BM - 1 < tn * BN) return;
  if (d.k <= 0) {
    // empty contraction: C = beta * C on the tile
    for (int e = threadIdx.x; e < BM * BN; e += C::NT) {
      const int i = tm * BM + e % BM, j = tn * BN + e / BM;
      if (i >= p.m || j >= p.n) continue;
      const long cc = p.ccol ? (long)p.ccol[j] : (long)j;
      double* c = p.C + cc * p.ldc + i;
      *c = (beta != 0.0) ? beta * *c : 0.0;
    }
    return;
  }
  gemm_tile<BM, BN, WM, WN, TA, TB, AM>(p, alpha, beta, flags, tm, tn, smem, 0, 1 << 30);
}

// sum of nsplit partial m x n products (ld m) into C: C = sum + beta C
template <class T>
__global__ void splitk_reduce_kernel(int m, int n, int nsplit, const T* part, T* C, long ldc,
                                     double beta, const int* ndev) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = (long)m * n;
  if (idx >= tot) return;
  if (ndev && idx / m >= *ndev) return;
  const T s = sum_in_order(part + idx, tot, nsplit, T(0));
  const int i = (int)(idx % m), j = (int)(idx / m);
  T* c = C + i + (long)j * ldc;
  *c = (beta != 0.0) ? s + (T)beta * *c : s;
}

// Tall-skinny products of several tasks in one launch, all with the 128 x 32
// tiles (n <= 32): workgroup blockIdx.x is tile (local % tiles, split
// local / tiles) of item wg_item[blockIdx.x].  kchunk > 0: split-K, each
// split writes its partial product (alpha op(A) op(B)) to part, reduced by
// splitk_reduce_group_kernel into C = sum + beta C; kchunk = 0: the tile is
// computed in place, C = alpha op(A) op(B) + beta C.
template <int TA, int TB, int AM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(waves_per_eu<128, 32, 4, 1, TA, AM>()))) void gemm_group_kernel(const GemmGroupItem* items,
                                                         const int* wg_item) {
  using C = G<128, 32, 4, 1, TA, TB, AM>;
  __shared__ double smem[C::SMEM];
  const int q = __builtin_amdgcn_readfirstlane(wg_item[blockIdx.x]);
  const GemmGroupItem& it = items[q];
  const int local = (int)blockIdx.x - it.b0;
  if (it.kchunk > 0) {
    const int split = local / it.tiles;
    Prob p{it.m, it.n, it.k, it.A, it.lda, it.B, it.ldb, it.part + (long)split * it.m * it.n,
           (long)it.m, nullptr, nullptr, nullptr};
    const int klo = split * it.kchunk;
    gemm_tile<128, 32, 4, 1, TA, TB, AM>(p, it.alpha, 0.0, it.flags, local % it.tiles, 0, smem,
                                         klo, klo + it.kchunk);
  } else {
    Prob p{it.m, it.n, it.k, it.A, it.lda, it.B, it.ldb, it.C, it.ldc, nullptr, nullptr, nullptr};
    gemm_tile<128, 32, 4, 1, TA, TB, AM>(p, it.alpha, it.beta, it.flags, local, 0, smem, 0,
                                         1 << 30);
  }
}

// Symmetric rank-k updates of several tasks in one launch: the lower tiles
// (tm >= tn, row by row) of each item's square C in 128 x 128 tiles, only
// elements on or below the diagonal written (GF_C_LOWER_ONLY).
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void syr2k_group_kernel(
    const GemmGroupItem* items, const int* wg_item) {
  using C = G<128, 128, 2, 4, 0, 1, AM_DENSE>;
  __shared__ double smem[C::SMEM];
  const int q = __builtin_amdgcn_readfirstlane(wg_item[blockIdx.x]);
  const GemmGroupItem& it = items[q];
  const int local = (int)blockIdx.x - it.b0;
  int tm = (int)((sqrt(8.0 * local + 1.0) - 1.0) * 0.5);
  while ((tm + 1) * (tm + 2) / 2 <= local) tm++;
  while (tm * (tm + 1) / 2 > local) tm--;
  const int tn = local - tm * (tm + 1) / 2;
  Prob p{it.m, it.n, it.k, it.A, it.lda, it.B, it.ldb, it.C, it.ldc, nullptr, nullptr, nullptr};
  gemm_tile<128, 128, 2, 4, 0, 1, AM_DENSE>(p, it.alpha, it.beta, it.flags, tm, tn, smem, 0,
                                            1 << 30);
}

// The two passes of X = A Y for a symmetric A with its lower triangle stored
// (X = tril(A) Y + strict_tril(A)^T Y), split over K in slices of kchunk
// (a multiple of 128), in one launch.  Pass 1 writes the partial product of
// 128-row tile i over K slice k to part1 (slice k at offset k m n, leading
// dimension m), pass 2 that of its transposed form to part2.  Only the
// (tile, slice) pairs that meet the stored triangle are computed: both
// passes read the kchunk x kchunk block (R, C), R >= C, of the lower
// triangle (pass 1 as the tiles of block row R over slice C, pass 2 as
// those of block row C over slice R), and the workgroups of one block are
// issued together on one XCD (the block is dealt to XCD id % 8, the
// workgroup ids of one XCD in turn), so that the second pass finds the
// block in the caches the first has just filled.
template <class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void sym_pair_kernel(
    ProbT<T> p, T* part1, T* part2, int kchunk, int ns) {
  using C1 = G<128, 32, 4, 1, 0, 0, AM_TRIL>;
  using C2 = G<128, 32, 4, 1, 1, 0, AM_SLT>;
  __shared__ T smem[C1::SMEM > C2::SMEM ? C1::SMEM : C2::SMEM];
  const int tpb = kchunk / 128;  // tiles per block row
  const int per = 2 * tpb;       // workgroups per block
  const int x = blockIdx.x % 8, li = blockIdx.x / 8;
  const int sb = 8 * (li / per) + x, q = li % per;
  if (sb >= ns * (ns + 1) / 2) return;
  int R = (int)((sqrt(8.0 * sb + 1.0) - 1.0) * 0.5);
  while ((R + 1) * (R + 2) / 2 <= sb) R++;
  while (R * (R + 1) / 2 > sb) R--;
  const int Cb = sb - R * (R + 1) / 2;
  const bool second = q >= tpb;
  const int tm = (second ? Cb : R) * tpb + q % tpb;
  const int split = second ? R : Cb;
  if (tm * 128 >= p.m) return;
  const int klo = split * kchunk;
  p.ldc = p.m;
  if (!second) {
    p.C = part1 + (long)split * p.m * p.n;
    gemm_tile<128, 32, 4, 1, 0, 0, AM_TRIL>(p, 1.0, 0.0, GF_A_TRIL | GF_KA_LOWER, tm, 0, smem,
                                            klo, klo + kchunk);
  } else {
    p.C = part2 + (long)split * p.m * p.n;
    gemm_tile<128, 32, 4, 1, 1, 0, AM_SLT>(p, 1.0, 0.0, GF_A_SLT | GF_KA_UPPER, tm, 0, smem,
                                           klo, klo + kchunk);
  }
}

// C = (sum of part2's slices) + (sum of part1's slices), each summed in
// slice order over the slices that meet the row's tile (the others hold
// zeros in the full split-K form, and adding +0 to these sums, which start
// from +0, changes no bit): the same roundings as the first pass reduced
// into C and the second reduced onto it.
template <class T>
__global__ void sym_pair_reduce_kernel(int m, int n, int nsplit, int kchunk, const T* part1,
                                       const T* part2, T* C, long ldc) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = (long)m * n;
  if (idx >= tot) return;
  const int i = (int)(idx % m), j = (int)(idx / m);
  const int t0 = (i / 128) * 128;
  const int z1 = min(nsplit - 1, (t0 + 127) / kchunk);  // last slice of the first pass
  const int z2 = t0 / kchunk;                            // first slice of the second
  const T s1 = sum_in_order(part1 + idx, tot, z1 + 1, T(0));
  const T s2 = sum_in_order(part2 + z2 * tot + idx, tot, nsplit - z2, T(0));
  C[i + (long)j * ldc] = s2 + s1;
}

// C = sum of the item's split partials + beta C, item blockIdx.y (split items only)
__global__ void splitk_reduce_group_kernel(const GemmGroupItem* items) {
  const GemmGroupItem& it = items[blockIdx.y];
  if (it.kchunk <= 0) return;
  const long tot = (long)it.m * it.n;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (long)gridDim.x * blockDim.x) {
    const double s = sum_in_order(it.part + idx, tot, it.nsplit, 0.0);
    const int i = (int)(idx % it.m), j = (int)(idx / it.m);
    double* c = it.C + i + (long)j * it.ldc;
    *c = (it.beta != 0.0) ? s + it.beta * *c : s;
  }
}

// C = beta*C when k == 0 (or alpha == 0)
template <class T>
__global__ void scale_kernel(int m, int n, T* C, long ldc, double beta, const int* ccol,
                             const int* ndev) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)m * n) return;
  int i = (int)(idx % m), j = (int)(idx / m);
  if (ndev && j >= *ndev) return;
  long cc = ccol ? (long)ccol[j] : (long)j;
  T* c = C + cc * ldc + i;
  *c = (beta != 0.0) ? (T)beta * *c : T(0);
}

// ---- dispatch ----------------------------------------------------------------------
template <int BM, int BN, int WM, int WN, int TA, int TB, int AM, class T>
const char* kernel_name() {
  static const std::string nm = "gemm_kernel<" + std::to_string(BM) + ", " + std::to_string(BN) +
                                ", " + std::to_string(WM) + ", " + std::to_string(WN) + ", " +
                                std::to_string(TA) + ", " + std::to_string(TB) + ", " +
                                std::to_string(AM) +
                                (sizeof(T) == 4 ? ", float>" : ">");
  return nm.c_str();
}

template <int BM, int BN, int WM, int WN, int TA, int TB, int AM, class T>
hipError_t launch_cfg(const ProbT<T>& p, double alpha, double beta, int flags, int nsplit,
                      int kchunk, long stride, double flops, hipStream_t s) {
  const int nblk = tile_grid(ceil_div(p.m, BM), ceil_div(p.n, BN));
  kt_begin(kernel_name<BM, BN, WM, WN, TA, TB, AM, T>(), flops, 0.0, p.ndev ? p.n : 0, s);
  HSDM_LAUNCH((gemm_kernel<BM, BN, WM, WN, TA, TB, AM, T>), dim3(nblk, nsplit),
                     dim3(64 * WM * WN), 0, s, p, alpha, beta, flags, kchunk, stride);
  kt_end(s);
  return hipGetLastError();
}

// tile configuration: 0 = 128x128 (8 waves), 1 = 128x64 (4 waves), 2 = 64x64 (4 waves),
// 3 = 128x32 (4 waves, skinny n), 4 = 32x128 (4 waves, skinny m)
// The rule follows the autotuner's choices on the MI355X for the products of
// the n = 16384 solve: 64x64 tiles for a k-contiguous A operand, for
// rank-k updates of a lower triangle with k < 1024 and for products of fewer
// than 4096 128x128 tiles (more, smaller tiles balance better), 128x64 for
// large lower-triangle updates and for products of 16384 or more 128x128
// tiles, 128x128 otherwise.  The tuning table below
// overrides it for the products it has timed.
int pick_cfg(int m, int n, int k, int nsplit, int ta, int flags) {
  if (n <= 32) return 3;
  if (m <= 32) return 4;
  const bool lower = (flags & (GF_C_LOWER_TILES | GF_C_LOWER_ONLY)) != 0;
  const long t128 = (long)ceil_div(m, 128) * ceil_div(n, 128) * nsplit;
  if (ta == 1) return (nsplit > 1 && t128 >= 512) ? 0 : 2;
  if (lower) return (k < 1024 || t128 < 4096) ? 2 : 1;
  if (t128 >= 16384) return 1;
  return t128 >= 4096 ? 0 : 2;
}

template <int TA, int TB, int AM, class T>
hipError_t launch_t(const ProbT<T>& p, double alpha, double beta, int flags, int nsplit,
                    int kchunk, long stride, double fl, int cfg, hipStream_t s) {
  switch (cfg >= 0 ? cfg : pick_cfg(p.m, p.n, kchunk > 0 ? kchunk : p.k, nsplit, TA, flags)) {
    case 0:
      return launch_cfg<128, 128, 2, 4, TA, TB, AM>(p, alpha, beta, flags, nsplit, kchunk, stride,
                                                    fl, s);
    case 1:
      return launch_cfg<128, 64, 2, 2, TA, TB, AM>(p, alpha, beta, flags, nsplit, kchunk, stride,
                                                   fl, s);
    case 3:
      return launch_cfg<128, 32, 4, 1, TA, TB, AM>(p, alpha, beta, flags, nsplit, kchunk, stride,
                                                   fl, s);
    case 4:
      return launch_cfg<32, 128, 1, 4, TA, TB, AM>(p, alpha, beta, flags, nsplit, kchunk, stride,
                                                   fl, s);
    default:
      return launch_cfg<64, 64, 2, 2, TA, TB, AM>(p, alpha, beta, flags, nsplit, kchunk, stride,
                                                  fl, s);
  }
}

template <class T>
hipError_t launch_any(const ProbT<T>& p, int ta, int tb, int am, double alpha, double beta,
                      int flags, int nsplit, int kchunk, long stride, double fl, hipStream_t s,
                      int cfg = -1) {
  if (am == AM_TRIL) {
    if (tb) return launch_t<0, 1, AM_TRIL>(p, alpha, beta, flags, nsplit, kchunk, stride, fl, cfg, s);
    return launch_t<0, 0, AM_TRIL>(p, alpha, beta, flags, nsplit, kchunk, stride, fl, cfg, s);
  }
  if (am == AM_SLT) {
    if (tb) return launch_t<1, 1, AM_SLT>(p, alpha, beta, flags, nsplit, kchunk, stride, fl, cfg, s);
    return launch_t<1, 0, AM_SLT>(p, alpha, beta, flags, nsplit, kchunk, stride, fl, cfg, s);
  }
  if (am == AM_SYM) return launch_t<0, 0, AM_SYM>(p, alpha, beta, flags, nsplit, kchunk, stride, fl, cfg, s);
  if (am == AM_GATHER) {
    if (tb) return launch_t<0, 1, AM_GATHER>(p, alpha, beta, flags, nsplit, kchunk, stride, fl, cfg, s);
    return launch_t<0, 0, AM_GATHER>(p, alpha, beta, flags, nsplit, kchunk, stride, fl, cfg, s);
  }
  if (ta == 0 && tb == 0)
    return launch_t<0, 0, AM_DENSE>(p, alpha, beta, flags, nsplit, kchunk, stride, fl, cfg, s);
  if (ta == 0 && tb == 1)
    return launch_t<0, 1, AM_DENSE>(p, alpha, beta, flags, nsplit, kchunk, stride, fl, cfg, s);
  if (ta == 1 && tb == 0)
    return launch_t<1, 0, AM_DENSE>(p, alpha, beta, flags, nsplit, kchunk, stride, fl, cfg, s);
  return launch_t<1, 1, AM_DENSE>(p, alpha, beta, flags, nsplit, kchunk, stride, fl, cfg, s);
}

// Algorithmic flops of one product: 2 m n k, halved for a lower-triangular
// result (square C), for a triangular op(A) or op(B), and for each half of a
// symmetric operand.
template <class T>
double gemm_flops(const GemmArgsT<T>& g) {
  double f = 2.0 * g.m * g.n * (double)g.k;
  if ((g.flags & (GF_C_LOWER_TILES | GF_C_LOWER_ONLY)) && g.m == g.n) f *= (g.n + 1.0) / (2.0 * g.n);
  if (g.flags & (GF_KA_LOWER | GF_KA_UPPER)) f *= 0.5;
  if (g.flags & (GF_KB_LOWER | GF_KB_UPPER)) f *= 0.5;
  if (g.flags & (GF_A_TRIL | GF_A_SLT)) f *= 0.5;
  return f;
}

template <class T>
int a_mode(const GemmArgsT<T>& g) {
  if (g.flags & GF_A_TRIL) return AM_TRIL;
  if (g.flags & GF_A_SLT) return AM_SLT;
  if (g.flags & GF_A_SYM_LOWER) return AM_SYM;
  if (g.acol) return AM_GATHER;
  return AM_DENSE;
}

// ---- tile autotuner -----------------------------------------------------------
// Products are classed by element size, ta, tb, A mode, lower-triangular
// output and the bit lengths of m, n and k; the process-wide table maps a
// class to the tile that ran it fastest.  While tuning is on, the first
// product of a class not in the table runs each candidate tile (128x128,
// 128x64, 64x64) twice on its own operands, C saved and restored around each
// run, and the faster second run decides; the product is then computed once
// more with the chosen tile.  Every tile computes each element with the same
// sequence of multiply-adds over k (slices of 16 in order; a triangular
// operand only adds exact zeros outside its triangle), so the choice never
// changes a result.  Skinny products (a side <= 32), split-K products and
// products with a device-side column count or scattered columns keep the
// rule.
std::mutex tune_mu;
std::map<unsigned long long, int> tune_table;
std::atomic<bool> tuning{false};

unsigned long long tune_key(int esize, int ta, int tb, int am, int flags, int m, int n, int k) {
  auto bl = [](int x) {
    int b = 0;
    while (x > 0) {
      b++;
      x >>= 1;
    }
    return (unsigned long long)b;
  };
  const unsigned long long lower = (flags & (GF_C_LOWER_TILES | GF_C_LOWER_ONLY)) ? 1ull : 0ull;
  return ((unsigned long long)esize << 40) | ((unsigned long long)ta << 39) |
         ((unsigned long long)tb << 38) | ((unsigned long long)am << 34) | (lower << 33) |
         (bl(m) << 22) | (bl(n) << 11) | bl(k);
}

int tuned_cfg(unsigned long long key) {
  std::lock_guard<std::mutex> lk(tune_mu);
  auto it = tune_table.find(key);
  return it == tune_table.end() ? -1 : it->second;
}

template <class T>
hipError_t tune_product(const GemmArgsT<T>& g, const ProbT<T>& p, int am, unsigned long long key,
                        double fl, hipStream_t s) {
  const size_t row = sizeof(T) * (size_t)g.m;
  T* save = nullptr;
  HSDM_TRY(hipMalloc(&save, row * g.n));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  if (err == hipSuccess)
    err = hipMemcpy2DAsync(save, row, g.C, sizeof(T) * g.ldc, row, g.n, hipMemcpyDeviceToDevice, s);
  int best = -1;
  float best_ms = 0.f;
  for (int c = 0; c < 3 && err == hipSuccess; c++) {
    float ms = 0.f;
    for (int rep = 0; rep < 2 && err == hipSuccess; rep++) {
      err = hipMemcpy2DAsync(g.C, sizeof(T) * g.ldc, save, row, row, g.n,
                             hipMemcpyDeviceToDevice, s);
      if (err == hipSuccess) err = hipEventRecord(e0, s);
      if (err == hipSuccess)
        err = launch_any(p, g.ta, g.tb, am, g.alpha, g.beta, g.flags, 1, 0, 0L, fl, s, c);
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    }
    if (err == hipSuccess && (best < 0 || ms < best_ms)) {
      best = c;
      best_ms = ms;
    }
  }
  if (err == hipSuccess)
    err = hipMemcpy2DAsync(g.C, sizeof(T) * g.ldc, save, row, row, g.n, hipMemcpyDeviceToDevice, s);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(save);
  if (err == hipSuccess && best >= 0) {
    std::lock_guard<std::mutex> lk(tune_mu);
    tune_table[key] = best;
  }
  return err;
}

template <class T>
hipError_t gemm_launch_t(const GemmArgsT<T>& g, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0) return hipSuccess;
  if (g.k <= 0 || g.alpha == 0.0) {
    if (g.beta == 1.0) return hipSuccess;
    long tot = (long)g.m * g.n;
    HSDM_LAUNCH(scale_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, g.m,
                       g.n, g.C, g.ldc, g.beta, g.ccol, g.ndev);
    return hipGetLastError();
  }
  const int am = a_mode(g);
  if ((am == AM_SYM || am == AM_GATHER || am == AM_TRIL) && g.ta != 0) return hipErrorInvalidValue;
  if (am == AM_SLT && g.ta != 1) return hipErrorInvalidValue;
  ProbT<T> p{g.m, g.n, g.k, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.acol, g.ccol, g.ndev};
  int cfg = -1;
  if (g.m > 32 && g.n > 32 && !g.ccol && !g.ndev) {
    const unsigned long long key = tune_key((int)sizeof(T), g.ta, g.tb, am, g.flags, g.m, g.n, g.k);
    cfg = tuned_cfg(key);
    if (cfg < 0 && tuning.load()) {
      HSDM_TRY(tune_product(g, p, am, key, gemm_flops(g), s));
      cfg = tuned_cfg(key);
    }
  }
  return launch_any(p, g.ta, g.tb, am, g.alpha, g.beta, g.flags, 1, 0, 0L, gemm_flops(g), s, cfg);
}

template <class T>
hipError_t gemm_splitk_launch_t(const GemmArgsT<T>& g, int kchunk, T* part, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0) return hipSuccess;
  if (g.k <= kchunk || kchunk <= 0) return gemm_launch_t(g, s);
  const int am = a_mode(g);
  if (g.ccol || (g.flags & (GF_C_LOWER_ONLY | GF_C_LOWER_TILES)) || am == AM_GATHER ||
      am == AM_SYM)
    return hipErrorInvalidValue;
  if ((am == AM_TRIL && g.ta != 0) || (am == AM_SLT && g.ta != 1)) return hipErrorInvalidValue;
  const int nsplit = ceil_div(g.k, kchunk);
  ProbT<T> p{g.m, g.n, g.k, g.A, g.lda, g.B, g.ldb, part, (long)g.m, g.acol, nullptr, g.ndev};
  const long stride = (long)g.m * g.n;
  HSDM_TRY(
      launch_any(p, g.ta, g.tb, am, g.alpha, 0.0, g.flags, nsplit, kchunk, stride, gemm_flops(g), s));
  HSDM_LAUNCH(splitk_reduce_kernel<T>, dim3((unsigned)((stride + 255) / 256)), dim3(256), 0, s,
                     g.m, g.n, nsplit, part, g.C, g.ldc, g.beta, g.ndev);
  return hipGetLastError();
}

template <class T>
hipError_t gemm_sym_pair_launch_t(const GemmArgsT<T>& g, int kchunk, T* part1, T* part2,
                                  hipStream_t s) {
  if (g.m <= 0 || g.n <= 0) return hipSuccess;
  if (g.n > 32 || g.m != g.k || kchunk <= 0 || kchunk % 128 || g.ta || g.tb ||
      !(g.flags & GF_A_TRIL))
    return hipErrorInvalidValue;
  const int nsplit = ceil_div(g.k, kchunk);
  const long nblocks = (long)nsplit * (nsplit + 1) / 2;
  const long per = 2 * (kchunk / 128);
  ProbT<T> p{g.m, g.n, g.k, g.A, g.lda, g.B, g.ldb, nullptr, (long)g.m, nullptr, nullptr, nullptr};
  kt_begin(sizeof(T) == 4 ? "sym_pair_kernel<float>" : "sym_pair_kernel", 2.0 * gemm_flops(g),
           0.0, 0, s);
  HSDM_LAUNCH(sym_pair_kernel<T>, dim3((unsigned)(8 * per * ((nblocks + 7) / 8))), dim3(256), 0,
              s, p, part1, part2, kchunk, nsplit);
  kt_end(s);
  HSDM_TRY(hipGetLastError());
  const long tot = (long)g.m * g.n;
  HSDM_LAUNCH(sym_pair_reduce_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     g.m, g.n, nsplit, kchunk, part1, part2, g.C, g.ldc);
  return hipGetLastError();
}

}  // namespace

void gemm_tuning(bool on) { tuning.store(on); }
bool gemm_tuning_on() { return tuning.load(); }

int gemm_tune_count() {
  std::lock_guard<std::mutex> lk(tune_mu);
  return (int)tune_table.size();
}

void gemm_tune_clear() {
  std::lock_guard<std::mutex> lk(tune_mu);
  tune_table.clear();
}

// text: one "class-key tile" pair per line, keys in hexadecimal
bool gemm_tune_save(const char* path) {
  std::lock_guard<std::mutex> lk(tune_mu);
  FILE* f = fopen(path, "w");
  if (!f) return false;
  bool ok = fprintf(f, "hsdm-gemm-tiles 1\n") > 0;
  for (const auto& kv : tune_table) ok = ok && fprintf(f, "%llx %d\n", kv.first, kv.second) > 0;
  return (fclose(f) == 0) && ok;
}

int gemm_tune_load(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return -1;
  char head[32] = {};
  int ver = 0;
  if (fscanf(f, "%31s %d", head, &ver) != 2 || std::string(head) != "hsdm-gemm-tiles" ||
      ver != 1) {
    fclose(f);
    return -2;
  }
  std::map<unsigned long long, int> add;
  unsigned long long k;
  int c;
  int r;
  while ((r = fscanf(f, "%llx %d", &k, &c)) == 2) {
    if (c < 0 || c > 2) {
      fclose(f);
      return -2;
    }
    add[k] = c;
  }
  fclose(f);
  if (r != EOF) return -2;
  std::lock_guard<std::mutex> lk(tune_mu);
  for (const auto& kv : add) tune_table[kv.first] = kv.second;
  return (int)add.size();
}

hipError_t gemm_launch(const GemmArgs& g, hipStream_t s) { return gemm_launch_t(g, s); }
hipError_t gemm_launch(const GemmArgsF& g, hipStream_t s) { return gemm_launch_t(g, s); }

hipError_t gemm_splitk_launch(const GemmArgs& g, int kchunk, double* part, hipStream_t s) {
  return gemm_splitk_launch_t(g, kchunk, part, s);
}
hipError_t gemm_splitk_launch(const GemmArgsF& g, int kchunk, float* part, hipStream_t s) {
  return gemm_splitk_launch_t(g, kchunk, part, s);
}

hipError_t gemm_sym_pair_launch(const GemmArgs& g, int kchunk, double* part1, double* part2,
                                hipStream_t s) {
  return gemm_sym_pair_launch_t(g, kchunk, part1, part2, s);
}
hipError_t gemm_sym_pair_launch(const GemmArgsF& g, int kchunk, float* part1, float* part2,
                                hipStream_t s) {
  return gemm_sym_pair_launch_t(g, kchunk, part1, part2, s);
}

hipError_t gemm_batched_launch(const GemmDesc* d_desc, int count, int max_m, int max_n,
                               double alpha, double beta, int ta, int tb, int flags,
                               hipStream_t s) {
  if (count <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  if (ta != 0 || tb != 0) return hipErrorInvalidValue;
  const int nblk = tile_grid(ceil_div(max_m, 64), ceil_div(max_n, 64));
  kt_begin("gemm_batched_kernel<64, 64, 2, 2, 0, 0, 2>", 0.0, 0.0, 0, s);
  HSDM_LAUNCH((gemm_batched_kernel<64, 64, 2, 2, 0, 0, AM_GATHER>), dim3(nblk, count),
                     dim3(256), 0, s, d_desc, alpha, beta, flags);
  kt_end(s);
  return hipGetLastError();
}

hipError_t gemm_batched_dense_launch(const GemmDesc* d_desc, int count, int max_m, int max_n,
                                     double alpha, double beta, int flags, hipStream_t s) {
  if (count <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  const int nblk = tile_grid(ceil_div(max_m, 64), ceil_div(max_n, 64));
  kt_begin("gemm_batched_kernel<64, 64, 2, 2, 0, 0, 0>", 0.0, 0.0, 0, s);
  HSDM_LAUNCH((gemm_batched_kernel<64, 64, 2, 2, 0, 0, AM_DENSE>), dim3(nblk, count),
                     dim3(256), 0, s, d_desc, alpha, beta, flags);
  kt_end(s);
  return hipGetLastError();
}

int gemm_group_kind(const GemmArgs& g) {
  if (g.flags & GF_A_TRIL) return GG_TRIL;
  if (g.flags & GF_A_SLT) return GG_SLT;
  if ((g.flags & GF_C_LOWER_TILES) && g.m == g.n && g.ta == 0 && g.tb == 1) return GG_SYR2K;
  if (g.ta) return GG_TN;
  return g.tb ? GG_NT : GG_NN;
}

size_t gemm_group_item(const GemmArgs& g, int kchunk, double* part, GemmGroupItem& it,
                       double* flops) {
  it = GemmGroupItem{};
  if (flops) *flops = gemm_flops(g);
  it.m = g.m; it.n = g.n; it.k = g.k;
  it.A = g.A; it.lda = g.lda; it.B = g.B; it.ldb = g.ldb;
  it.C = g.C; it.ldc = g.ldc; it.part = part;
  it.alpha = g.alpha;
  it.beta = g.beta;
  it.flags = g.flags;
  if (gemm_group_kind(g) == GG_SYR2K) {
    const int t = ceil_div(g.m, 128);
    it.tiles = t * (t + 1) / 2;
    it.kchunk = 0;
    it.nsplit = 1;
    return (size_t)it.tiles;
  }
  it.tiles = ceil_div(g.m, 128);
  it.kchunk = kchunk > 0 ? kchunk : 0;
  it.nsplit = kchunk > 0 ? ceil_div(g.k, kchunk) : 1;
  return (size_t)it.nsplit * it.tiles;
}

hipError_t gemm_group_launch(int kind, const GemmGroupItem* d_items, int count, const int* d_map,
                             int total_wg, int max_tot, bool split, double flops, hipStream_t s) {
  if (count <= 0 || total_wg <= 0) return hipSuccess;
  switch (kind) {
    case GG_TRIL:
      kt_begin("gemm_group_kernel<0, 0, 3>", flops, 0.0, 0, s);
      HSDM_LAUNCH((gemm_group_kernel<0, 0, AM_TRIL>), dim3(total_wg), dim3(256), 0, s,
                         d_items, d_map);
      break;
    case GG_SLT:
      kt_begin("gemm_group_kernel<1, 0, 4>", flops, 0.0, 0, s);
      HSDM_LAUNCH((gemm_group_kernel<1, 0, AM_SLT>), dim3(total_wg), dim3(256), 0, s,
                         d_items, d_map);
      break;
    case GG_NN:
      kt_begin("gemm_group_kernel<0, 0, 0>", flops, 0.0, 0, s);
      HSDM_LAUNCH((gemm_group_kernel<0, 0, AM_DENSE>), dim3(total_wg), dim3(256), 0, s,
                         d_items, d_map);
      break;
    case GG_TN:
      kt_begin("gemm_group_kernel<1, 0, 0>", flops, 0.0, 0, s);
      HSDM_LAUNCH((gemm_group_kernel<1, 0, AM_DENSE>), dim3(total_wg), dim3(256), 0, s,
                         d_items, d_map);
      break;
    case GG_NT:
      kt_begin("gemm_group_kernel<0, 1, 0>", flops, 0.0, 0, s);
      HSDM_LAUNCH((gemm_group_kernel<0, 1, AM_DENSE>), dim3(total_wg), dim3(256), 0, s,
                         d_items, d_map);
      break;
    case GG_SYR2K:
      kt_begin("syr2k_group_kernel", flops, 0.0, 0, s);
      HSDM_LAUNCH(syr2k_group_kernel, dim3(total_wg), dim3(512), 0, s, d_items, d_map);
      break;
    default: return hipErrorInvalidValue;
  }
  kt_end(s);
  HSDM_TRY(hipGetLastError());
  if (!split) return hipSuccess;
  const int bx = std::max(1, std::min(1024, ceil_div(max_tot, 256)));
  HSDM_LAUNCH(splitk_reduce_group_kernel, dim3(bx, count), dim3(256), 0, s, d_items);
  return hipGetLastError();
}
