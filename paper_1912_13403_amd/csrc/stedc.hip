// Divide and conquer for the symmetric tridiagonal eigenproblem T = Z L Z^T.
//
// Tearing: T = diag(T1', T2') + rho u u^T at every split (Cuppen), with
// rho = |beta|, u = [e_last; sign(beta) e_first], beta the coupling element;
// T1', T2' are T1, T2 with rho removed from the two touching diagonal
// entries.  The recursion tree halves [0, n) until pieces have at most 64
// rows; the leaves are solved by implicit QL in one wavefront each.
//
// Merge of two solved halves (Q1, L1), (Q2, L2):  T = Q (D + rho z z^T) Q^T
// with Q = diag(Q1, Q2), D = diag(L1, L2), z = Q^T u / sqrt(2), rho <- 2 rho.
//  - deflation (sequential scan in ascending d): a component with
//    rho |z_i| <= tol is an eigenpair as it stands; two close d's are rotated
//    (Givens on the two Q columns) so that one z vanishes;
//  - the k remaining roots of 1 + rho sum z_i^2 / (d_i - lambda) = 0 are found
//    one per thread relative to the nearer pole (rational two-pole model
//    steps inside a bisection bracket), so lambda - d_i is always known as
//    (d_origin - d_i) + tau to full relative accuracy;
//  - z is recomputed from the roots (Loewner / Gu-Eisenstat formula), which
//    keeps the eigenvectors u_j = (z_i / (d_i - lambda_j))_i orthogonal;
//  - new vectors = [rotated Q columns] * U on the FP64 matrix cores, top and
//    bottom halves separately so that the zero blocks of diag(Q1, Q2) are
//    never multiplied (columns are grouped top-only | mixed | bottom-only).
// All merges of one tree level run in the same launches; nothing returns to
// the host between levels.
#include <cfloat>
#include <vector>

#include "hsdm_internal.h"
#include "hsdm_phases.h"

namespace {

constexpr int LEAF = 64;
constexpr int META = 8;  // k, ndef, nrot, ntop, nmix, nbot, ncols, limit
constexpr int CHK = 1024;

// Orders LDS accesses between the lanes of one wavefront: the LDS executes a
// wavefront's instructions in order, so a compiler barrier is enough (no wait
// on outstanding global memory operations).
HSDM_DEV void wave_sync() {
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------------------
// Leaves: implicit QL on a piece of at most 64 rows, one wavefront.
__global__ __launch_bounds__(64) void leaf_kernel(int n, const double* d, const double* e,
                                                  const int* leaves, double* lam, double* Q,
                                                  long ldq, DevStatusWord* st) {
  const int lo = leaves[2 * blockIdx.x], hi = leaves[2 * blockIdx.x + 1];
  const int L = hi - lo;
  __shared__ double Z[LEAF][LEAF + 1];
  __shared__ double dd[LEAF], ee[LEAF];
  __shared__ int rank_of[LEAF];
  const int r = threadIdx.x;
  double dv = (r < L) ? d[lo + r] : 0.0;
  if (r == 0 && lo > 0) dv -= fabs(e[lo - 1]);
  if (r == L - 1 && hi < n) dv -= fabs(e[hi - 1]);
  dd[r] = dv;
  ee[r] = (r < L - 1) ? e[lo + r] : 0.0;
  for (int c = 0; c < LEAF; c++) Z[r][c] = (r == c) ? 1.0 : 0.0;
  wave_sync();
  bool fail = false;
  for (int l = 0; l < L && !fail; l++) {
    int steps = 0;
    for (;;) {
      int m = l;
      for (; m < L - 1; m++) {
        const double ds = fabs(dd[m]) + fabs(dd[m + 1]);
        if (fabs(ee[m]) <= DBL_EPSILON * ds || fabs(ee[m]) <= DBL_MIN) break;
      }
      if (m == l) break;
      if (++steps > 30) {
        fail = true;
        break;
      }
      double g = (dd[l + 1] - dd[l]) / (2.0 * ee[l]);
      double rr = hypot(g, 1.0);
      g = dd[m] - dd[l] + ee[l] / (g + copysign(rr, g));
      double s = 1.0, c = 1.0, p = 0.0;
      bool early = false;
      for (int i = m - 1; i >= l; i--) {
        const double f = s * ee[i];
        const double b = c * ee[i];
        rr = hypot(f, g);
        wave_sync();
        ee[i + 1] = rr;
        if (rr == 0.0) {
          dd[i + 1] -= p;
          ee[m] = 0.0;
          early = true;
          wave_sync();
          break;
        }
        s = f / rr;
        c = g / rr;
        g = dd[i + 1] - p;
        rr = (dd[i] - g) * s + 2.0 * c * b;
        p = s * rr;
        wave_sync();
        dd[i + 1] = g + p;
        g = c * rr - b;
        const double zi = Z[r][i], zi1 = Z[r][i + 1];
        Z[r][i + 1] = s * zi + c * zi1;
        Z[r][i] = c * zi - s * zi1;
        wave_sync();
      }
      if (early) continue;
      wave_sync();
      dd[l] -= p;
      ee[l] = g;
      ee[m] = 0.0;
      wave_sync();
    }
  }
  if (fail && r == 0) dev_set_status(st, DS_NO_CONVERGE, 1);
  // ascending order (ties by index)
  if (r < L) {
    const double x = dd[r];
    int rk = 0;
    for (int q = 0; q < L; q++) rk += (dd[q] < x) || (dd[q] == x && q < r);
    rank_of[r] = rk;
    lam[lo + rk] = x;
  }
  wave_sync();
  if (r < L)
    for (int c = 0; c < L; c++) Q[(lo + r) + (long)(lo + rank_of[c]) * ldq] = Z[r][c];
}

// ---------------------------------------------------------------------------
struct LevelBufs {
  const int* merges;  // lo, mid, hi per merge
  int* meta;
  double* rho;
  double* dsort;
  double* zsort;
  int* perm;
  int* msk;
  double* dk;
  double* zk;
  int* colk;
  int* gpos;
  int* acol;
  double* defval;
  int* defcol;
  int* rot_a;
  int* rot_b;
  double* rot_c;
  double* rot_s;
  int* rorg;
  double* rtau;
  double* rlam;
  double* zhat;
  int* orow;
  int* odef;
  double* Qblk;  // node block at Qblk + lo * n, ld N
  double* U;     // node block at U + lo * n, ld k
};

// The test of two neighbouring undeflated entries (prev: pd, pz; current:
// dq, zq): the rotation that zeroes pz has c = zq / r, s = pz / r,
// r = hypot(zq, pz), and leaves the coupling (pd - dq) c s; the test
// |(pd - dq) c s| <= tol is taken as |(pd - dq) zq pz| <= tol r^2 so that r,
// c and s are formed only for a rotation.
HSDM_DEV bool close_pair(double pd, double pz, double dq, double zq, double tol) {
  return fabs((pd - dq) * zq * pz) <= tol * (zq * zq + pz * pz);
}

// Per merge: z, sorted merge of the halves, deflation, grouping.
//
// Deflation is the scan of LAPACK's dlaed2 in the sorted order: an entry
// with rho |z| <= tol is deflated; each other entry is compared with the
// undeflated entry before it and, when the two are close (close_pair), a
// rotation deflates the earlier one and the later one carries on with the
// rotated values.  Only the rotations make the scan sequential: without
// one, the undeflated entries keep their own values in order.  The kernel
// therefore first sorts the entries in parallel (ballots and prefix counts)
// and tests every neighbouring pair with the unrotated values; the first
// pair that the sequential scan would rotate is among them (no rotation
// precedes it), so when no pair is close the result is the scan's exactly,
// and otherwise the sequential scan runs (by one thread).
__global__ __launch_bounds__(256) void merge_prep_kernel(int n, const double* e, const double* lam,
                                                         const double* Qcur, long ldq,
                                                         LevelBufs b, int m0) {
  const int mi = m0 + blockIdx.x;
  const int lo = b.merges[3 * mi], mid = b.merges[3 * mi + 1], hi = b.merges[3 * mi + 2];
  const int n1 = mid - lo, N = hi - lo;
  const double beta = e[mid - 1];
  const double rho = 2.0 * fabs(beta);
  const double sgn = (beta >= 0.0) ? 1.0 : -1.0;
  const double rs2 = 0.70710678118654752440;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const unsigned long long lanes_below = (1ull << lane) - 1ull;
  // sorted merge of the two ascending halves (ties: first half first), by
  // merge path: thread t writes outputs [t per, t per + per); it finds how
  // many of them before its first come from the first half by one binary
  // search along its diagonal, then merges its run sequentially
  const int n2 = N - n1;
  const int per = (N + 255) / 256;
  const int d0 = min(N, t * per), d1 = min(N, d0 + per);
  if (d0 < d1) {
    const double* A = lam + lo;   // first half, n1 ascending
    const double* Bh = lam + mid;  // second half, n2 ascending
    int a = max(0, d0 - n2), z = min(d0, n1);
    while (a < z) {
      const int h = (a + z) >> 1;
      if (A[h] <= Bh[d0 - h - 1]) a = h + 1; else z = h;
    }
    int i = a, j = d0 - a;
    for (int pos = d0; pos < d1; pos++) {
      const bool first = (j >= n2) || (i < n1 && A[i] <= Bh[j]);
      b.dsort[lo + pos] = first ? A[i] : Bh[j];
      b.perm[lo + pos] = first ? i : n1 + j;
      b.msk[lo + pos] = first ? 1 : 2;
      if (first) i++; else j++;
    }
  }
  __syncthreads();
  // z of each sorted entry: the last row of its top-half vector or the first
  // row of its bottom-half vector (times the sign of beta), over sqrt 2
  for (int pos = t; pos < N; pos += 256) {
    const int c = b.perm[lo + pos];
    const bool first = c < n1;
    b.zsort[lo + pos] = first ? Qcur[(mid - 1) + (long)(lo + c) * ldq] * rs2
                              : sgn * Qcur[mid + (long)(lo + c) * ldq] * rs2;
  }
  __syncthreads();
  __shared__ double cd[CHK], cz[CHK];
  __shared__ int cp[CHK], cm[CHK];
  __shared__ int wcnt[2][3][4];  // per chunk parity: counts of each wavefront
  __shared__ int close_seen, kk_s;
  const double dmax = fmax(fabs(b.dsort[lo]), fabs(b.dsort[lo + N - 1]));
  const double tol = 8.0 * DBL_EPSILON * fmax(dmax, rho);
  if (t == 0) close_seen = 0;
  // undeflated entries (in order) to dk/zk/colk/gpos, deflated ones to defval/defcol
  int kb = 0, db = 0;
  for (int base = 0, par = 0; base < N; base += 256, par ^= 1) {
    const int q = base + t;
    const bool valid = q < N;
    double dq = 0.0, zq = 0.0;
    int pq = 0, mq = 0;
    if (valid) {
      dq = b.dsort[lo + q];
      zq = b.zsort[lo + q];
      pq = b.perm[lo + q];
      mq = b.msk[lo + q];
    }
    const bool defl = valid && (rho * fabs(zq) <= tol);
    const bool keep = valid && !defl;
    const unsigned long long bk = __ballot(keep), bd = __ballot(defl);
    if (lane == 0) {
      wcnt[par][0][wv] = __popcll(bk);
      wcnt[par][1][wv] = __popcll(bd);
    }
    __syncthreads();
    int ko = kb + __popcll(bk & lanes_below), dof = db + __popcll(bd & lanes_below);
#pragma unroll
    for (int w = 0; w < 4; w++) {
      if (w < wv) {
        ko += wcnt[par][0][w];
        dof += wcnt[par][1][w];
      }
      kb += wcnt[par][0][w];
      db += wcnt[par][1][w];
    }
    if (keep) {
      b.dk[lo + ko] = dq;
      b.zk[lo + ko] = zq;
      b.colk[lo + ko] = pq;
      b.gpos[lo + ko] = mq;  // mask for now
    }
    if (defl) {
      b.defval[lo + dof] = dq;
      b.defcol[lo + dof] = pq;
    }
  }
  __syncthreads();
  for (int j = 1 + t; j < kb; j += 256)
    if (close_pair(b.dk[lo + j - 1], b.zk[lo + j - 1], b.dk[lo + j], b.zk[lo + j], tol))
      close_seen = 1;
  __syncthreads();
  int k = kb, ndef = db, nrot = 0;
  if (close_seen) {
    // sequential scan by thread 0 over LDS-staged chunks (it rewrites every
    // output above)
    k = 0;
    ndef = 0;
    bool have_prev = false;
    double pd = 0.0, pz = 0.0;
    int pc = 0, pm = 0;
    for (int base = 0; base < N; base += CHK) {
      const int cnt = min(CHK, N - base);
      __syncthreads();
      for (int q = t; q < cnt; q += 256) {
        cd[q] = b.dsort[lo + base + q];
        cz[q] = b.zsort[lo + base + q];
        cp[q] = b.perm[lo + base + q];
        cm[q] = b.msk[lo + base + q];
      }
      __syncthreads();
      if (t == 0) {
        for (int q = 0; q < cnt; q++) {
          const double dq = cd[q], zq = cz[q];
          if (rho * fabs(zq) <= tol) {
            b.defval[lo + ndef] = dq;
            b.defcol[lo + ndef] = cp[q];
            ndef++;
            continue;
          }
          if (!have_prev) {
            have_prev = true;
            pd = dq; pz = zq; pc = cp[q]; pm = cm[q];
            continue;
          }
          if (close_pair(pd, pz, dq, zq, tol)) {
            const double r = hypot(zq, pz);
            const double c = zq / r, s = pz / r;
            // rotate: new prev column = c q_prev - s q_cur (z -> 0), cur = s q_prev + c q_cur
            b.rot_a[lo + nrot] = pc;
            b.rot_b[lo + nrot] = cp[q];
            b.rot_c[lo + nrot] = c;
            b.rot_s[lo + nrot] = s;
            nrot++;
            const double dprev = c * c * pd + s * s * dq;
            const double dcur = s * s * pd + c * c * dq;
            b.defval[lo + ndef] = dprev;
            b.defcol[lo + ndef] = pc;
            ndef++;
            pd = dcur; pz = r; pc = cp[q]; pm = pm | cm[q];
          } else {
            b.dk[lo + k] = pd;
            b.zk[lo + k] = pz;
            b.colk[lo + k] = pc;
            b.gpos[lo + k] = pm;  // mask for now
            k++;
            pd = dq; pz = zq; pc = cp[q]; pm = cm[q];
          }
        }
      }
    }
    if (t == 0 && have_prev) {
      b.dk[lo + k] = pd;
      b.zk[lo + k] = pz;
      b.colk[lo + k] = pc;
      b.gpos[lo + k] = pm;
      k++;
    }
  }
  if (t == 0) {
    int* meta = b.meta + (long)mi * META;
    meta[0] = k;
    meta[1] = ndef;
    meta[2] = nrot;
    b.rho[mi] = rho;
    kk_s = k;
  }
  __syncthreads();
  // grouping: top-only (mask 1) | mixed (3) | bottom-only (2), stable: the
  // totals of each kind first, then each entry's place from ballots
  const int kk = kk_s;
  __shared__ int tot3[3];
  if (t < 3) tot3[t] = 0;
  __syncthreads();
  {
    int c3[3] = {0, 0, 0};
    for (int j = t; j < kk; j += 256) {
      const int mk = b.gpos[lo + j];
      c3[0] += (mk == 1);
      c3[1] += (mk == 3);
      c3[2] += (mk == 2);
    }
#pragma unroll
    for (int y = 0; y < 3; y++)
      if (c3[y]) atomicAdd(&tot3[y], c3[y]);
  }
  __syncthreads();
  const int nt = tot3[0], nm = tot3[1], nb = tot3[2];
  int run[3] = {0, nt, nt + nm};
  for (int base = 0, par = 0; base < kk; base += 256, par ^= 1) {
    const int j = base + t;
    const int mk = (j < kk) ? b.gpos[lo + j] : 0;
    const int ty = (mk == 1) ? 0 : ((mk == 3) ? 1 : 2);
    unsigned long long bm[3];
#pragma unroll
    for (int y = 0; y < 3; y++) bm[y] = __ballot(j < kk && ty == y);
    if (lane == 0) {
#pragma unroll
      for (int y = 0; y < 3; y++) wcnt[par][y][wv] = __popcll(bm[y]);
    }
    __syncthreads();
    int pos = 0;
#pragma unroll
    for (int y = 0; y < 3; y++) {
      int pre = 0, tot = 0;
#pragma unroll
      for (int w = 0; w < 4; w++) {
        if (w < wv) pre += wcnt[par][y][w];
        tot += wcnt[par][y][w];
      }
      if (y == ty) pos = run[y] + pre + __popcll(bm[y] & lanes_below);
      run[y] += tot;
    }
    if (j < kk) {
      b.gpos[lo + j] = pos;
      b.acol[lo + pos] = b.colk[lo + j];
    }
  }
  if (t == 0) {
    int* meta = b.meta + (long)mi * META;
    meta[3] = nt;
    meta[4] = nm;
    meta[5] = nb;
    meta[6] = kk;  // columns to form (may be lowered for the final merge)
    meta[7] = N;   // output columns limit
  }
}

// Qblk = diag(Q1, Q2) of the node (dense N x N): workgroup (x, y) of merge
// blockIdx.z fills rows [256 x, 256 x + 256) of columns [QB y, QB y + QB).
constexpr int QB = 32;
__global__ __launch_bounds__(256) void qblk_fill_kernel(const double* Qcur, long ldq, LevelBufs b,
                                                        int m0, int n) {
  const int mi = m0 + blockIdx.z;
  const int lo = b.merges[3 * mi], mid = b.merges[3 * mi + 1], hi = b.merges[3 * mi + 2];
  const int n1 = mid - lo, N = hi - lo;
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int c0 = blockIdx.y * QB;
  if (r >= N || c0 >= N) return;
  double* Qb = b.Qblk + (long)lo * n;
  const bool top = r < n1;
  const int c1 = min(N, c0 + QB);
  for (int c = c0; c < c1; c++) {
    const bool ctop = c < n1;
    Qb[r + (long)c * N] = (top == ctop) ? Qcur[(lo + r) + (long)(lo + c) * ldq] : 0.0;
  }
}

// The recorded deflation rotations applied to the rows of Qblk.
__global__ __launch_bounds__(256) void qblk_rotate_kernel(int n, LevelBufs b, int m0) {
  const int mi = m0 + blockIdx.y;
  const int lo = b.merges[3 * mi], hi = b.merges[3 * mi + 2];
  const int N = hi - lo;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  double* Qb = b.Qblk + (long)lo * n;
  // The rotations in order, RG at a time: the group's 2 RG entries of the
  // row are loaded together, the rotations applied in registers (an entry
  // that an earlier rotation of the group wrote is taken from that rotation's
  // result), then stored in order, so one memory latency covers RG rotations.
  constexpr int RG = 8;
  const int nrot = b.meta[(long)mi * META + 2];
  for (int q0 = 0; q0 < nrot; q0 += RG) {
    const int cnt = min(RG, nrot - q0);
    int ca[RG], cb[RG];
    double va[RG], vb[RG], cs[RG], sn[RG];
#pragma unroll
    for (int j = 0; j < RG; j++) {
      if (j < cnt) {
        ca[j] = b.rot_a[lo + q0 + j];
        cb[j] = b.rot_b[lo + q0 + j];
        cs[j] = b.rot_c[lo + q0 + j];
        sn[j] = b.rot_s[lo + q0 + j];
        va[j] = Qb[r + (long)ca[j] * N];
        vb[j] = Qb[r + (long)cb[j] * N];
      } else {
        ca[j] = cb[j] = -1;
        va[j] = vb[j] = cs[j] = sn[j] = 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < RG; j++) {
      double qa = va[j], qb = vb[j];
#pragma unroll
      for (int i = 0; i < j; i++) {
        if (ca[i] == ca[j]) qa = va[i];
        else if (cb[i] == ca[j]) qa = vb[i];
        if (ca[i] == cb[j]) qb = va[i];
        else if (cb[i] == cb[j]) qb = vb[i];
      }
      va[j] = cs[j] * qa - sn[j] * qb;
      vb[j] = sn[j] * qa + cs[j] * qb;
    }
#pragma unroll
    for (int j = 0; j < RG; j++) {
      if (j < cnt) {
        Qb[r + (long)ca[j] * N] = va[j];
        Qb[r + (long)cb[j] * N] = vb[j];
      }
    }
  }
}

HSDM_DEV double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

HSDM_DEV double wave_prod(double v) {
  for (int o = 32; o > 0; o >>= 1) v *= __shfl_xor(v, o, 64);
  return v;
}

// Secular equation, one root per wavefront (the sums over the k poles are
// split over the 64 lanes and combined in a fixed order).
__global__ __launch_bounds__(256) void secular_kernel(LevelBufs b, int m0, DevStatusWord* st) {
  const int mi = m0 + blockIdx.y;
  const int lo = b.merges[3 * mi];
  const int k = b.meta[(long)mi * META];
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= k) return;
  const double rho = b.rho[mi];
  const double* dk = b.dk + lo;
  const double* zk = b.zk + lo;
  int o;
  double tl, th;
  if (j < k - 1) {
    const double gap = dk[j + 1] - dk[j];
    const double mid = 0.5 * gap;
    double f = 0.0;
    for (int i = lane; i < k; i += 64) f += zk[i] * zk[i] / ((dk[i] - dk[j]) - mid);
    f = 1.0 / rho + wave_sum(f);
    if (f >= 0.0) {
      o = j; tl = 0.0; th = mid;
    } else {
      o = j + 1; tl = mid - gap; th = 0.0;
    }
  } else {
    double zz = 0.0;
    for (int i = lane; i < k; i += 64) zz += zk[i] * zk[i];
    zz = wave_sum(zz);
    o = j; tl = 0.0; th = rho * zz * (1.0 + 8.0 * DBL_EPSILON);
  }
  const double dorg = dk[o];
  const bool last = (j == k - 1);
  double tau = 0.5 * (tl + th);
  bool conv = false;
  for (int it = 0; it < 200; it++) {
    double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
    for (int i = lane; i < k; i += 64) {
      const double del = (dk[i] - dorg) - tau;
      const double q = zk[i] / del;
      if (i <= j) { psi += zk[i] * q; dpsi += q * q; }
      else { phi += zk[i] * q; dphi += q * q; }
    }
    psi = wave_sum(psi);
    dpsi = wave_sum(dpsi);
    phi = wave_sum(phi);
    dphi = wave_sum(dphi);
    const double f = 1.0 / rho + psi + phi;
    // converged once f is within the rounding error of its own evaluation
    // (psi <= 0 <= phi, so the absolute sum is 1/rho - psi + phi; the second
    // term covers the rounding of the differences (d_i - d_origin) - tau)
    const double ferr =
        8.0 * DBL_EPSILON * ((1.0 / rho - psi + phi) + fabs(tau) * (dpsi + dphi));
    if (f == 0.0 || fabs(f) <= ferr) { conv = true; break; }
    if (f < 0.0) tl = tau; else th = tau;
    if (th - tl <= 4.0 * DBL_EPSILON * fmax(fabs(tl), fabs(th))) {
      tau = 0.5 * (tl + th);
      conv = true;
      break;
    }
    const double DL = (dk[j] - dorg) - tau;
    double eta;
    bool ok = true;
    if (!last) {
      const double DR = (dk[j + 1] - dorg) - tau;
      const double sL = DL * DL * dpsi, sR = DR * DR * dphi;
      const double cc = f - DL * dpsi - DR * dphi;
      const double a1 = -(cc * (DL + DR) + sL + sR);
      const double a0 = cc * DL * DR + sL * DR + sR * DL;
      if (cc == 0.0) {
        eta = -a0 / a1;
      } else {
        double disc = a1 * a1 - 4.0 * cc * a0;
        if (disc < 0.0) disc = 0.0;
        const double q = -0.5 * (a1 + copysign(sqrt(disc), a1));
        const double e1 = q / cc, e2 = a0 / q;
        eta = (e1 > DL && e1 < DR) ? e1 : e2;
      }
    } else {
      const double sL = DL * DL * dpsi;
      const double cc = f - DL * dpsi;
      if (cc > 0.0) eta = DL + sL / cc; else ok = false;
    }
    double tn = ok ? tau + eta : 0.5 * (tl + th);
    if (!(tn > tl && tn < th)) tn = 0.5 * (tl + th);
    if (tn <= tl || tn >= th) { conv = true; break; }  // bracket exhausted
    const bool small = fabs(tn - tau) <= 2.0 * DBL_EPSILON * fabs(tn);
    tau = tn;
    if (small) { conv = true; break; }
  }
  if (lane == 0) {
    if (!conv) dev_set_status(st, DS_NO_CONVERGE, 2);
    b.rorg[lo + j] = o;
    b.rtau[lo + j] = tau;
    b.rlam[lo + j] = dorg + tau;
  }
}

// Loewner: z_i from the roots, one wavefront per i (the product over the
// roots is split over the lanes; every factor is a ratio below one).
__global__ __launch_bounds__(256) void zhat_kernel(LevelBufs b, int m0) {
  const int mi = m0 + blockIdx.y;
  const int lo = b.merges[3 * mi];
  const int k = b.meta[(long)mi * META];
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= k) return;
  const double rho = b.rho[mi];
  const double* dk = b.dk + lo;
  const double di = dk[i];
  double p = 1.0;
  for (int j = lane; j < k - 1; j += 64) {
    const double num = (dk[b.rorg[lo + j]] - di) + b.rtau[lo + j];
    const double den = (j < i) ? (dk[j] - di) : (dk[j + 1] - di);
    p *= num / den;
  }
  p = wave_prod(p) * (((dk[b.rorg[lo + k - 1]] - di) + b.rtau[lo + k - 1]) / rho);
  if (lane == 0) b.zhat[lo + i] = copysign(sqrt(fmax(p, 0.0)), b.zk[lo + i]);
}

// Order of the merged eigenvalues (roots and deflated values), ascending;
// ties put deflated values first, then by index.
__global__ __launch_bounds__(256) void order_kernel(double* lam, LevelBufs b, int m0) {
  const int mi = m0 + blockIdx.y;
  const int lo = b.merges[3 * mi], hi = b.merges[3 * mi + 2];
  const int N = hi - lo;
  const int k = b.meta[(long)mi * META], nd = b.meta[(long)mi * META + 1];
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= N) return;
  const double* rl = b.rlam + lo;
  const double* dv = b.defval + lo;
  if (x < k) {
    const double v = rl[x];
    int rk = x;  // roots before it
    for (int q = 0; q < nd; q++) rk += (dv[q] <= v);
    lam[lo + rk] = v;
    b.orow[lo + x] = lo + rk;
  } else {
    const int q = x - k;
    const double v = dv[q];
    int rk = 0;
    for (int p = 0; p < nd; p++) rk += (dv[p] < v) || (dv[p] == v && p < q);
    int a = 0, z = k;  // roots strictly below v
    while (a < z) {
      const int h = (a + z) >> 1;
      if (rl[h] < v) a = h + 1; else z = h;
    }
    rk += a;
    lam[lo + rk] = v;
    b.odef[lo + q] = lo + rk;
  }
}

// Columns of U (rows in group order), one workgroup per column.
__global__ __launch_bounds__(256) void vectors_kernel(LevelBufs b, int m0, int n) {
  const int mi = m0 + blockIdx.y;
  const int lo = b.merges[3 * mi];
  const int* meta = b.meta + (long)mi * META;
  const int k = meta[0], ncols = meta[6];
  const int j = blockIdx.x;
  if (j >= ncols) return;
  const double* dk = b.dk + lo;
  const double dorg = dk[b.rorg[lo + j]];
  const double tj = b.rtau[lo + j];
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < k; i += 256) {
    const double u = b.zhat[lo + i] / ((dk[i] - dorg) - tj);
    s += u * u;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double inv = 1.0 / sqrt(red[0]);
  double* U = b.U + (long)lo * n + (long)j * k;
  for (int i = threadIdx.x; i < k; i += 256)
    U[b.gpos[lo + i]] = b.zhat[lo + i] / ((dk[i] - dorg) - tj) * inv;
}

// GEMM descriptors: top rows and bottom rows of the new vectors.
__global__ void desc_kernel(LevelBufs b, int m0, int cnt, double* Qnext, long ldq, int n,
                            GemmDesc* desc) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= cnt) return;
  const int mi = m0 + x;
  const int lo = b.merges[3 * mi], mid = b.merges[3 * mi + 1], hi = b.merges[3 * mi + 2];
  const int n1 = mid - lo, N = hi - lo;
  const int* meta = b.meta + (long)mi * META;
  const int k = meta[0], nt = meta[3], nm = meta[4], nb = meta[5], ncols = meta[6];
  const double* Qb = b.Qblk + (long)lo * n;
  const double* U = b.U + (long)lo * n;
  GemmDesc top{}, bot{};
  top.m = n1; top.n = (k > 0) ? ncols : 0; top.k = nt + nm;
  top.A = Qb; top.lda = N; top.acol = b.acol + lo;
  top.B = U; top.ldb = k > 0 ? k : 1;
  top.C = Qnext + lo; top.ldc = ldq; top.ccol = b.orow + lo;
  bot.m = N - n1; bot.n = (k > 0) ? ncols : 0; bot.k = nm + nb;
  bot.A = Qb + n1; bot.lda = N; bot.acol = b.acol + lo + nt;
  bot.B = U + nt; bot.ldb = k > 0 ? k : 1;
  bot.C = Qnext + mid; bot.ldc = ldq; bot.ccol = b.orow + lo;
  desc[2 * x] = top;
  desc[2 * x + 1] = bot;
}

// Deflated eigenvectors are the (rotated) columns as they stand.
__global__ __launch_bounds__(256) void deflated_copy_kernel(LevelBufs b, int m0, double* Qnext,
                                                            long ldq, int n) {
  const int mi = m0 + blockIdx.y;
  const int lo = b.merges[3 * mi], hi = b.merges[3 * mi + 2];
  const int N = hi - lo;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  const int* meta = b.meta + (long)mi * META;
  const int nd = meta[1], limit = meta[7];
  const double* Qb = b.Qblk + (long)lo * n;
  for (int q = 0; q < nd; q++) {
    const int oc = b.odef[lo + q];
    if (oc - lo >= limit) continue;
    Qnext[(lo + r) + (long)oc * ldq] = Qb[r + (long)b.defcol[lo + q] * N];
  }
}

// Final merge with a wanted-vector count: columns formed = roots whose
// position in the merged order is below *m_dev; deflated copies likewise.
__global__ void limit_kernel(LevelBufs b, int mi, const int* m_dev) {
  if (threadIdx.x != 0) return;
  const int lo = b.merges[3 * mi];
  int* meta = b.meta + (long)mi * META;
  const int k = meta[0];
  const int lim = *m_dev;
  int a = 0, z = k;  // roots are in ascending order, so are their positions
  while (a < z) {
    const int h = (a + z) >> 1;
    if (b.orow[lo + h] - lo < lim) a = h + 1; else z = h;
  }
  meta[6] = a;
  meta[7] = lim;
}

__global__ void copy_cols_kernel(const double* Q, long ldq, double* Z, long ldz, int n, int m_host,
                                 const int* m_dev) {
  const int m = m_dev ? *m_dev : m_host;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * m) return;
  const int i = (int)(idx % n), j = (int)(idx / n);
  Z[i + (long)j * ldz] = Q[i + (long)j * ldq];
}

}  // namespace

struct StedcPlan {
  int n = 0;
  int nleaf = 0;
  std::vector<int> leaves;                 // lo, hi
  std::vector<std::vector<int>> levels;    // merges (lo, mid, hi) by height
  std::vector<int> level_first;            // first merge index of each level
  std::vector<int> level_maxN;
  int nmerge = 0;
  int* d_leaves = nullptr;
  int* d_merges = nullptr;
  GemmDesc* d_desc = nullptr;
  std::vector<int> merges_host;
};

static int build_tree(StedcPlan* p, int lo, int hi) {
  if (hi - lo <= LEAF) {
    p->leaves.push_back(lo);
    p->leaves.push_back(hi);
    return 0;
  }
  const int mid = lo + (hi - lo) / 2;
  const int h1 = build_tree(p, lo, mid);
  const int h2 = build_tree(p, mid, hi);
  const int h = 1 + (h1 > h2 ? h1 : h2);
  if ((int)p->levels.size() < h) p->levels.resize(h);
  p->levels[h - 1].push_back(lo);
  p->levels[h - 1].push_back(mid);
  p->levels[h - 1].push_back(hi);
  return h;
}

static void plan_tree(StedcPlan* p, int n) {
  p->n = n;
  if (n <= 0) return;
  build_tree(p, 0, n);
  p->nleaf = (int)p->leaves.size() / 2;
  std::vector<int>& all = p->merges_host;
  all.clear();
  for (auto& lv : p->levels) {
    p->level_first.push_back((int)all.size() / 3);
    int mx = 0;
    for (size_t q = 0; q < lv.size(); q += 3) mx = std::max(mx, lv[q + 2] - lv[q]);
    p->level_maxN.push_back(mx);
    all.insert(all.end(), lv.begin(), lv.end());
  }
  p->nmerge = (int)all.size() / 3;
}

size_t stedc_plan_device_bytes(int n) {
  StedcPlan p;
  plan_tree(&p, n);
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return up(sizeof(int) * p.leaves.size()) + up(sizeof(int) * p.merges_host.size()) +
         up(sizeof(GemmDesc) * 2 * (size_t)p.nmerge);
}

StedcPlan* stedc_plan_create_in(int n, void* dev) {
  StedcPlan* p = new StedcPlan();
  plan_tree(p, n);
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char* c = (char*)dev;
  p->d_leaves = (int*)c;
  c += up(sizeof(int) * p->leaves.size());
  p->d_merges = (int*)c;
  c += up(sizeof(int) * p->merges_host.size());
  p->d_desc = (GemmDesc*)c;
  return p;
}

hipError_t stedc_plan_upload(StedcPlan* p, hipStream_t s) {
  if (!p || p->n <= 0) return hipSuccess;
  HSDM_TRY(hipMemcpyAsync(p->d_leaves, p->leaves.data(), sizeof(int) * p->leaves.size(),
                          hipMemcpyHostToDevice, s));
  if (p->nmerge > 0)
    HSDM_TRY(hipMemcpyAsync(p->d_merges, p->merges_host.data(),
                            sizeof(int) * p->merges_host.size(), hipMemcpyHostToDevice, s));
  return hipSuccess;
}

void stedc_plan_destroy(StedcPlan* p) { delete p; }

// doubles: Q, Qblk, U (3 n^2) + 11 vectors of n;  ints: 11 vectors of n + meta
size_t stedc_scratch_doubles(int n) { return (size_t)3 * n * n + (size_t)16 * n + 64; }
static size_t stedc_scratch_ints(int n) { return (size_t)16 * n + (size_t)META * n + 64; }

hipError_t stedc_run(StedcPlan* p, const double* d, const double* e, double* lam, double* Z,
                     long ldz, double* scratch, int* iscratch, const int* m_dev,
                     StedcEigvalHook hook, void* hook_ctx, DevStatusWord* st, hipStream_t s) {
  const int n = p->n;
  if (n <= 0) return hipSuccess;
  (void)stedc_scratch_ints;
  // One eigenvector buffer: every node's block lives at Q[lo:hi, lo:hi].  A
  // merge reads its children only while building Qblk (and z), and the new
  // block is produced from Qblk and U, so it is written back in place.
  double* Qa = scratch;
  LevelBufs b{};
  b.merges = p->d_merges;
  b.Qblk = Qa + (size_t)n * n;
  b.U = b.Qblk + (size_t)n * n;
  double* dv = b.U + (size_t)n * n;
  b.rho = dv; dv += n;
  b.dsort = dv; dv += n;
  b.zsort = dv; dv += n;
  b.dk = dv; dv += n;
  b.zk = dv; dv += n;
  b.defval = dv; dv += n;
  b.rot_c = dv; dv += n;
  b.rot_s = dv; dv += n;
  b.rtau = dv; dv += n;
  b.rlam = dv; dv += n;
  b.zhat = dv; dv += n;
  int* iv = iscratch;
  b.meta = iv; iv += (size_t)META * n;
  b.perm = iv; iv += n;
  b.msk = iv; iv += n;
  b.colk = iv; iv += n;
  b.gpos = iv; iv += n;
  b.acol = iv; iv += n;
  b.defcol = iv; iv += n;
  b.rot_a = iv; iv += n;
  b.rot_b = iv; iv += n;
  b.rorg = iv; iv += n;
  b.orow = iv; iv += n;
  b.odef = iv; iv += n;

  HSDM_LAUNCH(leaf_kernel, dim3(p->nleaf), dim3(64), 0, s, n, d, e, p->d_leaves, lam, Qa,
                     (long)n, st);
  HSDM_TRY(hipGetLastError());
  double* Qcur = Qa;
  double* Qnext = Qa;
  const int nlev = (int)p->levels.size();
  if (nlev == 0 && hook) HSDM_TRY(hook(hook_ctx, lam, s));
  for (int lv = 0; lv < nlev; lv++) {
    const int m0 = p->level_first[lv];
    const int cnt = (int)p->levels[lv].size() / 3;
    const int maxN = p->level_maxN[lv];
    const bool final_level = (lv == nlev - 1);
    HSDM_LAUNCH(merge_prep_kernel, dim3(cnt), dim3(256), 0, s, n, e, lam, Qcur, (long)n, b,
                       m0);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(qblk_fill_kernel, dim3(ceil_div(maxN, 256), ceil_div(maxN, QB), cnt),
                       dim3(256), 0, s, Qcur, (long)n, b, m0, n);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(qblk_rotate_kernel, dim3(ceil_div(maxN, 256), cnt), dim3(256), 0, s, n, b,
                       m0);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(secular_kernel, dim3(ceil_div(maxN, 4), cnt), dim3(256), 0, s, b, m0, st);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(zhat_kernel, dim3(ceil_div(maxN, 4), cnt), dim3(256), 0, s, b, m0);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(order_kernel, dim3(ceil_div(maxN, 256), cnt), dim3(256), 0, s, lam, b, m0);
    HSDM_TRY(hipGetLastError());
    if (final_level) {
      if (hook) HSDM_TRY(hook(hook_ctx, lam, s));
      if (m_dev) {
        HSDM_LAUNCH(limit_kernel, dim3(1), dim3(64), 0, s, b, m0, m_dev);
        HSDM_TRY(hipGetLastError());
      }
    }
    HSDM_LAUNCH(vectors_kernel, dim3(maxN, cnt), dim3(256), 0, s, b, m0, n);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(desc_kernel, dim3(ceil_div(cnt, 64)), dim3(64), 0, s, b, m0, cnt, Qnext,
                       (long)n, n, p->d_desc + 2 * m0);
    HSDM_TRY(hipGetLastError());
    HSDM_TRY(gemm_batched_launch(p->d_desc + 2 * m0, 2 * cnt, (maxN + 1) / 2 + 1, maxN, 1.0, 0.0,
                                 0, 0, 0, s));
    HSDM_LAUNCH(deflated_copy_kernel, dim3(ceil_div(maxN, 256), cnt), dim3(256), 0, s, b,
                       m0, Qnext, (long)n, n);
    HSDM_TRY(hipGetLastError());
  }
  const long tot = (long)n * (m_dev ? n : n);
  HSDM_LAUNCH(copy_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Qcur,
                     (long)n, Z, ldz, n, n, m_dev);
  return hipGetLastError();
}

size_t stedc_iscratch_ints(int n) { return stedc_scratch_ints(n); }

double stedc_last_flops(const StedcPlan* p) {
  if (!p || p->nmerge <= 0) return 0.0;
  std::vector<GemmDesc> h(2 * (size_t)p->nmerge);
  if (hipMemcpy(h.data(), p->d_desc, sizeof(GemmDesc) * h.size(), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return -1.0;
  double f = 0.0;
  for (const GemmDesc& g : h) f += 2.0 * (double)g.m * g.n * g.k;
  return f;
}
