// Internal declarations shared by the HIP sources of libhsdm (not installed).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

#define HSDM_DEV __device__ __forceinline__

// ---------------------------------------------------------------------------
// GEMM: C = alpha * op(A) * op(B) + beta * C, FP64 (or FP32), column-major.
// op(A) is m x k, op(B) is k x n.
enum GemmFlags {
  GF_C_LOWER_TILES = 1,   // skip output tiles that lie entirely above the diagonal
  GF_C_LOWER_ONLY = 2,    // never write elements with row < col
  GF_KA_LOWER = 4,        // op(A) lower triangular: row i only needs k <= i
  GF_KA_UPPER = 8,        // op(A) upper triangular: row i only needs k >= i
  GF_KB_UPPER = 16,       // op(B) upper triangular: column j only needs k <= j
  GF_KB_LOWER = 32,       // op(B) lower triangular: column j only needs k >= j
  GF_A_SYM_LOWER = 64,    // A symmetric, only its lower triangle is read (m == k)
  GF_A_TRIL = 128,        // op(A) = lower triangle of A (diagonal included), ta = 0
  GF_A_SLT = 256,         // op(A) = transpose of the strict lower triangle of A, ta = 1
};

// Element type T = double (FP64 MFMA) or float (FP32 MFMA, the refined
// form's reduction and back-transform); alpha and beta are given in double.
template <class T>
struct GemmArgsT {
  int m, n, k;
  const T* A; long lda;
  const T* B; long ldb;
  T* C; long ldc;
  double alpha, beta;
  int ta, tb;             // 0: as stored, 1: transposed
  int flags;
  const int* acol;        // optional: op(A)[:, kk] = A[:, acol[kk]] (ta == 0)
  const int* ccol;        // optional: column j of the product goes to C[:, ccol[j]]
  const int* ndev;        // optional: device-side column count, n is its upper bound
};
using GemmArgs = GemmArgsT<double>;
using GemmArgsF = GemmArgsT<float>;

// One GEMM of a device-side batch.  Sizes may be written by an earlier kernel.
struct GemmDesc {
  int m, n, k;
  int pad;
  const double* A; long lda;
  const double* B; long ldb;
  double* C; long ldc;
  const int* acol;
  const int* ccol;
};

hipError_t gemm_launch(const GemmArgs& g, hipStream_t s);
hipError_t gemm_launch(const GemmArgsF& g, hipStream_t s);
// The tile autotuner's process-wide table (gemm.hip): tuning on makes the
// first product of each untimed class time the candidate tiles; save/load
// write and merge the table as text (load returns the entries read, -1 if
// the file cannot be opened, -2 if it is malformed; nothing is merged then).
void gemm_tuning(bool on);
bool gemm_tuning_on();
int gemm_tune_count();
void gemm_tune_clear();
bool gemm_tune_save(const char* path);
int gemm_tune_load(const char* path);
// Split-K: K cut into slices of kchunk; part holds ceil(k/kchunk) * m * n
// partial products, summed in slice order (reproducible), then C = sum + beta C.
hipError_t gemm_splitk_launch(const GemmArgs& g, int kchunk, double* part, hipStream_t s);
hipError_t gemm_splitk_launch(const GemmArgsF& g, int kchunk, float* part, hipStream_t s);
// Batched launch: every descriptor uses the same alpha, beta, ta, tb, flags;
// max_m, max_n bound the sizes any descriptor can take.
hipError_t gemm_batched_launch(const GemmDesc* d_desc, int count, int max_m, int max_n,
                               double alpha, double beta, int ta, int tb, int flags,
                               hipStream_t s);
// The same for plain operands (no gathered columns; acol and ccol unused).
hipError_t gemm_batched_dense_launch(const GemmDesc* d_desc, int count, int max_m, int max_n,
                                     double alpha, double beta, int flags, hipStream_t s);
// Products of several tasks in one launch.  Tall-skinny ones (n <= 32), all
// with the 128 x 32 tiles, of kind GG_TRIL (op(A) = tril(A), as GF_A_TRIL),
// GG_SLT (op(A) = strict_tril(A)^T, as GF_A_SLT), GG_NN, GG_TN (A
// transposed), GG_NT (B transposed); and GG_SYR2K, the lower tiles of a
// square C = alpha A B^T + beta C (GF_C_LOWER_TILES, m = n) in 128 x 128
// tiles, every item in place.  gemm_group_kind tells the kind of a product.
// A tall-skinny item with kchunk > 0 is split over K: its nsplit
// partials (m x n each) go to its part buffer and are reduced into
// C = sum + beta C when `split`; kchunk = 0 computes C = alpha op(A) op(B) +
// beta C in place.  gemm_group_item fills an item from the product's
// arguments (kchunk 0: in place), stores the product's algorithmic flops in
// *flops (if given) and returns its workgroup count; the caller sets b0 (the
// item's first workgroup) and writes the workgroup -> item map.  d_items and
// d_map are device arrays.
enum { GG_TRIL = 0, GG_SLT = 1, GG_NN = 2, GG_TN = 3, GG_NT = 4, GG_SYR2K = 5 };
struct GemmGroupItem {
  const double* A;
  const double* B;
  double* C;
  double* part;
  long lda, ldb, ldc;
  double alpha, beta;
  int m, n, k, flags, kchunk, nsplit, tiles, b0;
};
int gemm_group_kind(const GemmArgs& g);
size_t gemm_group_item(const GemmArgs& g, int kchunk, double* part, GemmGroupItem& it,
                       double* flops);
hipError_t gemm_group_launch(int kind, const GemmGroupItem* d_items, int count, const int* d_map,
                             int total_wg, int max_tot, bool split, double flops, hipStream_t s);

// ---------------------------------------------------------------------------
// Kernel timer (ktimer.hip): per-launch HIP events on the launching stream,
// active for the calling thread between kt_activate(k) and kt_activate(nullptr).
struct KTimer;
KTimer* kt_create();
void kt_destroy(KTimer* k);
void kt_activate(KTimer* k);
void kt_reset(KTimer* k);
// flops / bytes: algorithmic work of this launch; nbound > 0 marks work that
// scales with a device-side count (the occupied states) bounded by nbound.
void kt_begin(const char* name, double flops, double bytes, int nbound, hipStream_t s,
              bool whole_phase = false);
// Restrict a timer to the launches marked whole_phase (one launch per solve).
void kt_set_whole_only(KTimer* k, bool on);
// Restrict a timer to the launches of one kernel (nullptr or "": all).
void kt_set_only(KTimer* k, const char* name);
void kt_end(hipStream_t s);
// Records made after kt_set_tag(t) carry tag t (-1: none); a solve of several
// tasks tags each task's launches with its index.
void kt_set_tag(int t);
// Set the work of the most recent record of kernel `name` (work known only
// after the launch, e.g. from device-side counts read back later).
void kt_set_last_work(const char* name, double flops, double bytes);
// After the stream is synchronized: fold records into per-kernel totals (m =
// the device-side count for records with nbound > 0, < 0 if unknown; a record
// with tag t < ntag uses tag_m[t] instead).
void kt_collect(KTimer* k, int m, const int* tag_m = nullptr, int ntag = 0);
int kt_count(const KTimer* k);
const char* kt_stat(const KTimer* k, int i, double* out4);

// ---------------------------------------------------------------------------
// Launches of a solve that shares the device with other solves
// (HSDM_KEY_CONCURRENT; util.hip).  Some kernels of this library spin on
// other workgroups of their own grid: the cooperative ones (panel QR, bulge
// chasing) on any of them, the stage-2 back-transform on lower-numbered
// ones.  Beside kernels of other streams such a kernel can be held off: the
// compute units it waits for stay full of other kernels' workgroups for as
// long as those streams keep submitting, and two spinning kernels can each
// keep out what the other waits for.  So every launch of a concurrent solve
// passes a gate: ordinary launches share it (HSDM_LAUNCH), a spinning launch
// holds it alone (coop_launch) from its launch until it has finished --
// no other concurrent solve submits work meanwhile, and what they had
// submitted before drains.  Outside concurrent solves the gate is not used.
void coop_set_shared(bool on);
bool coop_get_shared();
struct LaunchGate {
  LaunchGate();
  ~LaunchGate();
  bool held;
};
#define HSDM_LAUNCH(...)          \
  do {                            \
    LaunchGate hsdm_gate_;        \
    hipLaunchKernelGGL(__VA_ARGS__); \
  } while (0)
// A spinning kernel (cooperative: all workgroups resident; else: waits on
// lower-numbered workgroups only), timed by the kernel timer (nbound as in
// kt_begin).
hipError_t coop_launch(const char* name, double flops, double bytes, bool whole_phase,
                       bool cooperative, const void* fn, dim3 grid, dim3 block, void** args,
                       hipStream_t s, int nbound = 0);

// ---------------------------------------------------------------------------
// Device status word shared by all kernels of a solve (first error wins).
enum DevStatus {
  DS_OK = 0,
  DS_NOT_SPD = 1,       // detail: failing column (1-based)
  DS_NO_CONVERGE = 2,   // detail: which phase
  DS_MU_FAIL = 3,
  DS_SYNC_TIMEOUT = 4,  // a bounded inter-workgroup wait ran out
};

struct DevStatusWord {
  int code;
  int detail;
};

HSDM_DEV void dev_set_status(DevStatusWord* st, int code, int detail) {
  if (atomicCAS(&st->code, 0, code) == 0) st->detail = detail;
}

// s + p[0] + p[stride] + ... + p[(cnt - 1) stride], added in that order.  The
// loads go out 16 at a time, so a long sum by few threads (the partials of a
// split product) waits for memory once per 16 terms, not once per term.
template <class T>
HSDM_DEV T sum_in_order(const T* p, long stride, int cnt, T s) {
  for (int z = 0; z < cnt; z += 16) {
    T v[16];
#pragma unroll
    for (int i = 0; i < 16; i++) v[i] = (z + i < cnt) ? p[(long)(z + i) * stride] : T(0);
#pragma unroll
    for (int i = 0; i < 16; i++)
      if (z + i < cnt) s += v[i];
  }
  return s;
}

// Launch-error helper.
#define HSDM_TRY(x)                          \
  do {                                       \
    hipError_t _e = (x);                     \
    if (_e != hipSuccess) return _e;         \
  } while (0)

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }
