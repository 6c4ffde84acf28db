// Occupation numbers and chemical potential from the eigenvalues and the
// electron count (Sec. 2.6; normalization of Eq. (16) for one unit task).
//
// kT > 0: Fermi-Dirac occupations f_max / (1 + exp((eps - mu)/kT)),
//         mu by bisection on sum_l f_l = N_e inside
//         [eps_min - 50 kT - 1, eps_max + 50 kT + 1] until the bracket ends
//         are adjacent doubles (at most 200 halvings).
// kT = 0: step occupations; the states within deg_tol of the Fermi level
//         share the remaining electrons equally (the kT -> 0+ limit).
// One workgroup of 1024 threads; each bisection step is one fixed-order
// block reduction, so the result is reproducible run to run.
#include "hsdm_internal.h"
#include "hsdm_util.h"

namespace {

constexpr int NT = 1024;

HSDM_DEV double fermi(double x, double fmax) {
  if (x >= 0.0) {
    const double t = exp(-x);
    return fmax * t / (1.0 + t);
  }
  return fmax / (1.0 + exp(x));
}

// Fixed-order sum over the block; every thread receives the total.
HSDM_DEV double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NT / 64; i++) s += red[i];
  return s;
}

HSDM_DEV int block_count(int v, double* red) { return (int)block_sum((double)v, red); }

__global__ __launch_bounds__(NT) void occ_kernel(int n, const double* eps, double fmax, double ne,
                                                 double kT, double deg_tol,
                                                 const double* hnorm, double fcut,
                                                 double* f, OccOut* out, DevStatusWord* st) {
  __shared__ double red[NT / 64];
  const int t = threadIdx.x;
  if (hnorm) deg_tol = 1e-12 * *hnorm;
  int bad = 0;
  for (int l = t; l < n; l += NT) bad |= !isfinite(eps[l]);
  if (block_count(bad, red) > 0) {
    if (t == 0) {
      dev_set_status(st, DS_MU_FAIL, 0);
      out->mu = NAN;
      out->band_energy = NAN;
      out->sum_f = NAN;
      out->m = 0;
      out->iters = 0;
    }
    for (int l = t; l < n; l += NT) f[l] = 0.0;
    return;
  }
  double mu;
  int iters = 0;
  if (kT > 0.0) {
    double lo = eps[0] - 50.0 * kT - 1.0, hi = eps[n - 1] + 50.0 * kT + 1.0;
    for (int it = 0; it < 200; it++) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      double s = 0.0;
      for (int l = t; l < n; l += NT) s += fermi((eps[l] - mid) / kT, fmax);
      s = block_sum(s, red);
      if (s < ne) lo = mid; else hi = mid;
      iters = it + 1;
    }
    mu = 0.5 * (lo + hi);
    for (int l = t; l < n; l += NT) f[l] = fermi((eps[l] - mu) / kT, fmax);
  } else if (ne <= 0.0) {
    mu = eps[0];
    for (int l = t; l < n; l += NT) f[l] = 0.0;
  } else {
    int ns = (int)ceil(ne / fmax - 1e-12);
    ns = ns < 1 ? 1 : (ns > n ? n : ns);
    const double ef = eps[ns - 1];
    int nb = 0, ng = 0;
    for (int l = t; l < n; l += NT) {
      if (eps[l] < ef - deg_tol) nb++;
      else if (eps[l] <= ef + deg_tol) ng++;
    }
    nb = block_count(nb, red);
    ng = block_count(ng, red);
    const double share = (ne - fmax * nb) / ng;
    for (int l = t; l < n; l += NT) {
      const double e = eps[l];
      f[l] = (e < ef - deg_tol) ? fmax : ((e <= ef + deg_tol) ? share : 0.0);
    }
    const bool partial = share < fmax * (1.0 - 1e-15);
    mu = (partial || nb + ng >= n) ? ef : 0.5 * (eps[nb + ng - 1] + eps[nb + ng]);
  }
  __syncthreads();
  double eb = 0.0, sf = 0.0;
  int m = 0;
  for (int l = t; l < n; l += NT) {
    const double fl = f[l];
    eb += fl * eps[l];
    sf += fl;
    m += (fl > fcut);
  }
  eb = block_sum(eb, red);
  sf = block_sum(sf, red);
  m = block_count(m, red);
  if (t == 0) {
    out->mu = mu;
    out->band_energy = eb;
    out->sum_f = sf;
    out->m = m;
    out->iters = iters;
  }
}

}  // namespace

hipError_t occupations_launch(int n, const double* eps, double fmax, double ne, double kT,
                              double deg_tol, const double* hnorm, double fcut, double* f,
                              OccOut* out, DevStatusWord* st, hipStream_t s) {
  hipLaunchKernelGGL(occ_kernel, dim3(1), dim3(NT), 0, s, n, eps, fmax, ne, kT, deg_tol, hnorm,
                     fcut, f, out, st);
  return hipGetLastError();
}
