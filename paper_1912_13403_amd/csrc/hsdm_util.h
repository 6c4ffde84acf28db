// Host-side launchers of the helper kernels and of each phase of the path.
#pragma once
#include "hsdm_internal.h"

// util.hip
hipError_t dev_fill(double* a, long lda, int m, int n, double v, hipStream_t s);
hipError_t dev_copy(const double* a, long lda, double* b, long ldb, int m, int n, hipStream_t s);
hipError_t dev_sym_full(const double* a, long lda, double* b, long ldb, int n, hipStream_t s);
// b = a (m x n) converted between FP64 and FP32 (round to nearest), and the
// FP32 copy
hipError_t dev_convert(const double* a, long lda, float* b, long ldb, int m, int n, hipStream_t s);
hipError_t dev_convert(const float* a, long lda, double* b, long ldb, int m, int n, hipStream_t s);
hipError_t dev_copy(const float* a, long lda, float* b, long ldb, int m, int n, hipStream_t s);
hipError_t dev_mirror_lower(double* a, long lda, int n, hipStream_t s);
// out[0] += 64-bit content hash of the lower triangle of a (n x n; cplx:
// interleaved complex, lda in complex elements); dev_hash_clear zeroes
// out[0 .. cnt-1] first (a kernel, not a memset, so that it can be captured).
hipError_t dev_hash_clear(unsigned long long* out, int cnt, hipStream_t s);
hipError_t dev_hash_lower(const void* a, long lda, int n, int cplx, unsigned long long* out,
                          hipStream_t s);
hipError_t dev_norm1_sym(const double* a, long lda, int n, double* colsum, double* out,
                         hipStream_t s);

// chol.hip: S = L L^T and L^{-1}, recursively.
//   A (n x n, lda) holds S's lower triangle on entry and L (lower, zeros
//   above) on exit; Li (n x n, ldi) receives L^{-1} (lower, zeros above);
//   T is scratch of at least n x ((n+1)/2) doubles (ldt >= n).
hipError_t chol_inv(int n, double* A, long lda, double* Li, long ldi, double* T, long ldt,
                    DevStatusWord* st, hipStream_t s);

// occ.hip: occupations, mu, band energy and the count m of states whose
// occupation exceeds fcut.  Results go to device memory.  If hnorm (device)
// is given, the kT = 0 degeneracy window is 1e-12 * *hnorm instead of deg_tol.
struct OccOut {
  double mu;
  double band_energy;
  double sum_f;
  int m;
  int iters;
};
hipError_t occupations_launch(int n, const double* eps, double fmax, double ne, double kT,
                              double deg_tol, const double* hnorm, double fcut, double* f,
                              OccOut* out, DevStatusWord* st, hipStream_t s);

// One unit task of a joint occupation (Eq. (16)): its ascending eigenvalues,
// its weight, where its occupations and summary go, and (for the automatic
// degeneracy window) its ||H||_1.
struct OccTask {
  const double* eps;
  double* f;
  OccOut* out;
  const double* hnorm;
  int n;
  double w;
};
// Occupations of nt tasks with one chemical potential fixed by
// sum_p w_p sum_l f_pl = ne.  Each task's OccOut receives the shared mu, its own
// sum_l f eps, sum_l f and m = #{f > fcut}; `total` receives mu,
// sum_p w_p sum_l f eps and sum_p w_p sum_l f.  deg_tol < 0 takes
// 1e-12 max_p ||H_p||_1.  `tasks` is a device array.
hipError_t occupations_joint_launch(int nt, const OccTask* tasks, double fmax, double ne, double kT,
                                    double deg_tol, double fcut, OccOut* total, DevStatusWord* st,
                                    hipStream_t s);

// dm.hip: D = C diag(f) C^T and (optionally) E = C diag(f eps) C^T from the
// first m columns of C (n x m, ldc); both written in full.
hipError_t density_launch(int n, int m, const double* C, long ldc, const double* f,
                          const double* eps, double* D, long ldd, double* E, long lde,
                          const int* m_dev, hipStream_t s);
