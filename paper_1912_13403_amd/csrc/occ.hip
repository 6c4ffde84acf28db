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
  HSDM_LAUNCH(occ_kernel, dim3(1), dim3(NT), 0, s, n, eps, fmax, ne, kT, deg_tol, hnorm,
                     fcut, f, out, st);
  return hipGetLastError();
}

// ---- one chemical potential for several unit tasks (Eq. (16)) --------------------
//
// The eigenvalues of all tasks are coupled by the electron count
// sum_p w_p sum_l f_pl = N_e (k-point weights w_p; spin channels are separate
// tasks).  kT > 0: the same bisection as above on the weighted sum.  kT = 0:
// the Fermi level is the lowest eigenvalue x of the union at which the
// weighted count f_max sum_{eps <= x} w reaches N_e (found by bisection on x
// down to adjacent doubles, so it is an eigenvalue); the states of the union
// within deg_tol of it share the remaining electrons equally per unit weight.

namespace {

// sum over all tasks of g(task, eps), fixed order per thread, then a block sum
template <class G>
HSDM_DEV double union_sum(int nt, const OccTask* T, double* red, G g) {
  double s = 0.0;
  for (int p = 0; p < nt; p++) {
    const OccTask& q = T[p];
    double sp = 0.0;
    for (int l = threadIdx.x; l < q.n; l += NT) sp += g(q, q.eps[l]);
    s += q.w * sp;
  }
  return block_sum(s, red);
}

HSDM_DEV double block_min(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
  for (int i = 1; i < NT / 64; i++) s = fmin(s, red[i]);
  return s;
}

HSDM_DEV double block_max(double v, double* red) { return -block_min(-v, red); }

__global__ __launch_bounds__(NT) void occ_joint_kernel(int nt, const OccTask* T, double fmax,
                                                       double ne, double kT, double deg_tol,
                                                       double fcut, OccOut* total,
                                                       DevStatusWord* st) {
  __shared__ double red[NT / 64];
  const int t = threadIdx.x;
  double lo_e = INFINITY, hi_e = -INFINITY, hn = 0.0;
  int bad = 0;
  for (int p = 0; p < nt; p++) {
    const OccTask& q = T[p];
    for (int l = t; l < q.n; l += NT) bad |= !isfinite(q.eps[l]);
    if (q.n > 0) {
      lo_e = fmin(lo_e, q.eps[0]);
      hi_e = ::fmax(hi_e, q.eps[q.n - 1]);
    }
    if (q.hnorm) hn = ::fmax(hn, *q.hnorm);
  }
  if (deg_tol < 0.0) deg_tol = 1e-12 * hn;
  if (block_count(bad, red) > 0 || !(lo_e <= hi_e)) {
    for (int p = 0; p < nt; p++) {
      const OccTask& q = T[p];
      for (int l = t; l < q.n; l += NT) q.f[l] = 0.0;
      if (t == 0) {
        q.out->mu = NAN;
        q.out->band_energy = NAN;
        q.out->sum_f = NAN;
        q.out->m = 0;
        q.out->iters = 0;
      }
    }
    if (t == 0) {
      dev_set_status(st, DS_MU_FAIL, 0);
      total->mu = NAN;
      total->band_energy = NAN;
      total->sum_f = NAN;
      total->m = 0;
      total->iters = 0;
    }
    return;
  }
  double mu, share = 0.0, ef = 0.0;
  int iters = 0;
  if (kT > 0.0) {
    double lo = lo_e - 50.0 * kT - 1.0, hi = hi_e + 50.0 * kT + 1.0;
    for (int it = 0; it < 200; it++) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      const double s = union_sum(nt, T, red, [&](const OccTask&, double e) {
        return fermi((e - mid) / kT, fmax);
      });
      if (s < ne) lo = mid; else hi = mid;
      iters = it + 1;
    }
    mu = 0.5 * (lo + hi);
  } else if (ne <= 0.0) {
    mu = lo_e;
  } else {
    // smallest eigenvalue x with f_max * sum_{eps <= x} w >= ne
    const double need = ne - 1e-12 * fmax;
    double lo = lo_e - 1.0, hi = hi_e;
    if (need <= 0.0) lo = hi = lo_e;  // a vanishing count: the lowest state
    for (int it = 0; it < 2100 && lo < hi; it++) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      const double c = fmax * union_sum(nt, T, red, [&](const OccTask&, double e) {
        return e <= mid ? 1.0 : 0.0;
      });
      if (c >= need) hi = mid; else lo = mid;
      iters = it + 1;
    }
    ef = hi;
    const double wb = union_sum(nt, T, red, [&](const OccTask&, double e) {
      return e < ef - deg_tol ? 1.0 : 0.0;
    });
    const double wg = union_sum(nt, T, red, [&](const OccTask&, double e) {
      return (e >= ef - deg_tol && e <= ef + deg_tol) ? 1.0 : 0.0;
    });
    share = (ne - fmax * wb) / wg;
    if (share > fmax) share = fmax;
    // mu: the Fermi level itself when it is partly filled, else the middle of
    // the gap above the highest state of its group
    double gtop = -INFINITY, above = INFINITY;
    for (int p = 0; p < nt; p++) {
      const OccTask& q = T[p];
      for (int l = t; l < q.n; l += NT) {
        const double e = q.eps[l];
        if (e <= ef + deg_tol) gtop = ::fmax(gtop, e);
        else above = fmin(above, e);
      }
    }
    gtop = block_max(gtop, red);
    above = block_min(above, red);
    const bool partial = share < fmax * (1.0 - 1e-15);
    mu = (partial || !(above < INFINITY)) ? ef : 0.5 * (gtop + above);
  }
  // occupations and per-task summaries
  double eb_tot = 0.0, sf_tot = 0.0;
  for (int p = 0; p < nt; p++) {
    const OccTask& q = T[p];
    double eb = 0.0, sf = 0.0;
    int m = 0;
    for (int l = t; l < q.n; l += NT) {
      const double e = q.eps[l];
      double fl;
      if (kT > 0.0) fl = fermi((e - mu) / kT, fmax);
      else if (ne <= 0.0) fl = 0.0;
      else fl = (e < ef - deg_tol) ? fmax : ((e <= ef + deg_tol) ? share : 0.0);
      q.f[l] = fl;
      eb += fl * e;
      sf += fl;
      m += (fl > fcut);
    }
    eb = block_sum(eb, red);
    sf = block_sum(sf, red);
    m = block_count(m, red);
    eb_tot += q.w * eb;
    sf_tot += q.w * sf;
    if (t == 0) {
      q.out->mu = mu;
      q.out->band_energy = eb;
      q.out->sum_f = sf;
      q.out->m = m;
      q.out->iters = iters;
    }
  }
  if (t == 0) {
    total->mu = mu;
    total->band_energy = eb_tot;
    total->sum_f = sf_tot;
    total->m = 0;
    total->iters = iters;
  }
}

}  // namespace

hipError_t occupations_joint_launch(int nt, const OccTask* tasks, double fmax, double ne, double kT,
                                    double deg_tol, double fcut, OccOut* total, DevStatusWord* st,
                                    hipStream_t s) {
  HSDM_LAUNCH(occ_joint_kernel, dim3(1), dim3(NT), 0, s, nt, tasks, fmax, ne, kT, deg_tol,
                     fcut, total, st);
  return hipGetLastError();
}
