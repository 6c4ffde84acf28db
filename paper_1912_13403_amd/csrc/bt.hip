// Back-transformation of eigenvectors through the two reduction stages.
//
// Stage 2 (bulge chasing): the reflectors H_{s,t} of B consecutive sweeps
// (sweep block b) that share the task index t are combined into one block
// reflector G = I - V T V^T (V: 2B x B parallelogram, T: B x B upper
// triangular) acting on rows r B + 1 .. r B + 2B, r = b + t, so that applying
// it is three small products on the FP64 matrix cores.  Q2 Z applies later
// sweeps first: group (b, r) must follow (b+1, r-1 .. r+1) and (b, r-1).
//
// Stage 1 (panels): Z <- (I - V_p T_p V_p^T) Z for p from the last panel to
// the first, as three GEMMs per panel (the tall V_p^T Z with split-K).
#include "hsdm_internal.h"
#include "hsdm_phases.h"
#include "hsdm_util.h"

namespace {

constexpr int B = 32;
constexpr int H2 = 2 * B;  // rows of a group

// Compact record of one group (GREC doubles): the parallelogram of V by
// columns, Vc[32 j + i] = V[j + i][j] (i, j < B), then the upper triangle of
// T folded into 16 rows of B + 1: row p holds column p (entries 0 .. p) and
// then column B-1-p (entries 0 .. B-1-p), then zeros up to a multiple of 64
// doubles (one coalesced load per lane and step).
constexpr int TPACK = (B / 2) * (B + 1);                  // 528
constexpr int GREC = ((B * B + TPACK + 63) / 64) * 64;  // 1600

// (row, column) of T held at position e of the folded triangle
HSDM_DEV void tpack_index(int e, int& i, int& j) {
  const int p = e / (B + 1), o = e - p * (B + 1);
  if (o <= p) {
    i = o;
    j = p;
  } else {
    i = o - p - 1;
    j = B - 1 - p;
  }
}

// T factor of every group (T_jj = tau_j, T(0:j, j) = -tau_j T(0:j,0:j) V^T v_j),
// then the compact record.
__global__ __launch_bounds__(256) void group_pack_kernel(const double* V2, const double* tau2,
                                                         double* F2) {
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
  double* F = F2 + gi * (long)GREC;
  for (int e = t; e < B * B; e += 256) {
    const int j = e / B, i = e % B;
    F[e] = Vs[j + i][j];
  }
  for (int e = t; e < GREC - B * B; e += 256) {
    int i = 0, j = 0;
    if (e < TPACK) tpack_index(e, i, j);
    F[B * B + e] = (e < TPACK) ? Tl[i][j] : 0.0;
  }
}

// Z <- Q2 Z for one strip of 16 columns per workgroup.  Columns of Z are
// independent, so a workgroup applies every group to its strip with no
// other workgroup involved.  Its PW wavefronts take the sweep blocks in turn
// (wavefront w: b = nblk-1-w, nblk-1-w-PW, ...); each walks its block's
// groups upward (r = b + t, t = 0, 1, ...), keeping the group's 64 x 16
// window of Z in registers in MFMA accumulator layout: lane l holds rows
// 4i + l/16 of each 16-row block at column l%16, which is also the layout
// of a B operand, so the three products chain with no data movement.  After
// group (b, r) the lower half (rows of block r) is final for sweep block b
// and is stored; the upper half becomes the next window's lower half.
// Group (b, r) needs (b+1, r+1) done (and with it (b+1, r-1 .. r), and (b, r-1)
// by construction).  A wavefront stays one group further behind its
// predecessor than that requires, so the row block and the compact record
// of its next group are loaded while the current group is computed; the
// record is staged in the wavefront's own LDS area, from which the MFMA A
// operands (V^T, T, -V, zero parts skipped) are read.  Progress counters
// live in LDS; their keys grow monotonically across a wavefront's sweep
// blocks.
__global__ void fill_i32_kernel(int* p, int cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = 0;
}

constexpr int PW = 8;            // wavefronts per workgroup (two per SIMD)
constexpr int KEYM = 1 << 13;    // > tasks per sweep block
constexpr int NFRAG = 60;        // A operands per group: 24 (V^T) + 12 (T) + 24 (-V)
constexpr int VS = B + 2;        // LDS column stride of V (conflict-free operand reads)
constexpr int TS = B + 1;        // LDS column stride of T
constexpr int NST = GREC / 64;   // record doubles per lane

HSDM_DEV int key_of(int nblk, int b) { return (nblk - 1 - b) * KEYM; }

// The sweep blocks are cut into NSPLIT ranges of about equal work; workgroup
// (k, strip) applies range k (k = 0 holds the last sweep blocks, which come
// first) to its strip once workgroup (k-1, strip) has finished, so that the
// strips' work is spread over NSPLIT times as many workgroups.

// Workgroup blk of one Z's launch: strip blk % nstrip, range blk / nstrip.
HSDM_DEV void bt2_strip_body(int n, int nblk, const SplitRanges& R, int nstrip,
                             const double* F2, const long* goff, double* Z, long ldz, int m,
                             int* done, DevStatusWord* st, int blk) {
  const int strip = blk % nstrip, kr = blk / nstrip;
  const int c0 = strip * 16;
  if (c0 >= m) return;  // (every range of this strip returns here)
  __shared__ int prog[PW];
  __shared__ int wg_failed;
  __shared__ double Vl_all[PW][B * VS];
  __shared__ double Tl_all[PW][B * TS];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* Vl = Vl_all[w];
  double* Tl = Tl_all[w];
  if (lane == 0) prog[w] = -1;
  for (int e = lane; e < B * TS; e += 64) Tl[e] = 0.0;  // below T's diagonal stays zero
  if (threadIdx.x == 0) {
    // range kr - 1 of this strip must be complete (its workgroup has a lower
    // index, so it was dispatched earlier and is running or finished)
    int bad = 0;
    if (kr > 0) {
      long spins = 0;
      while (__hip_atomic_load(&done[strip], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < kr) {
        if (++spins > (1L << 26) ||
            ((spins & 4095) == 0 &&
             __hip_atomic_load(&st->code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
          bad = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    wg_failed = bad;
  }
  __syncthreads();
  if (wg_failed) {
    if (threadIdx.x == 0) dev_set_status(st, DS_SYNC_TIMEOUT, 3);
    return;
  }
  const int l16 = lane & 15, l4 = lane >> 4;
  const int col = c0 + l16;
  const bool cok = col < m;
  double* Zc = Z + (long)(cok ? col : 0) * ldz;
  const int pw = (w + PW - 1) % PW;
  bool failed = false;

  auto tgb = [&](int b) { return (n - 1 - b * B + B - 1) / B; };
  auto ld4 = [&](int r0, dbl4& z) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int row = r0 + 4 * i + l4;
      z[i] = (cok && row < n) ? Zc[row] : 0.0;
    }
  };
  auto st4 = [&](int r0, const dbl4& z) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int row = r0 + 4 * i + l4;
      if (cok && row < n) Zc[row] = z[i];
    }
  };
  // record of a group -> registers (coalesced) -> this wavefront's LDS area
  auto ld_rec = [&](const double* G, double* r) {
#pragma unroll
    for (int q = 0; q < NST; q++) r[q] = G[q * 64 + lane];
  };
  auto put_rec = [&](const double* r) {
#pragma unroll
    for (int q = 0; q < NST; q++) {
      const int e = q * 64 + lane;
      if (q < B * B / 64) {
        Vl[(e >> 5) * VS + (e & 31)] = r[q];
      } else if (e - B * B < TPACK) {
        int i, j;
        tpack_index(e - B * B, i, j);
        Tl[j * TS + i] = r[q];
      }
    }
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
  };
  // A operands from LDS: lane l gets A[row l%16][k l/16] of each 16 x 4 block
  auto get_ops = [&](double* f) {
#pragma unroll
    for (int q = 0; q < 24; q++) {  // V^T: row block a, k step 4a .. 4a+11
      const int a = q / 12, kq = 4 * a + q % 12;
      const int j = 16 * a + l16, i = 4 * kq + l4 - j;
      const double v = Vl[j * VS + (i & 31)];
      f[q] = (i >= 0 && i < B) ? v : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 12; q++) {  // T: a = 0, k steps 0..7; a = 1, k steps 4..7
      const int a = (q < 8) ? 0 : 1, kq = (q < 8) ? q : q - 4;
      f[24 + q] = Tl[(4 * kq + l4) * TS + 16 * a + l16];
    }
#pragma unroll
    for (int q = 0; q < 24; q++) {  // -V: Z row block rq, k steps by rq
      int rq, kq;
      if (q < 4) { rq = 0; kq = q; }
      else if (q < 12) { rq = 1; kq = q - 4; }
      else if (q < 20) { rq = 2; kq = q - 12; }
      else { rq = 3; kq = q - 16; }
      const int j = 4 * kq + l4, i = 16 * rq + l16 - j;
      const double v = Vl[j * VS + (i & 31)];
      f[36 + q] = (i >= 0 && i < B) ? -v : 0.0;
    }
  };
  auto publish = [&](int v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) __hip_atomic_store(&prog[w], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  auto wait_for = [&](int target) {
    long spins = 0;
    while (__hip_atomic_load(&prog[pw], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
      if (++spins > (1L << 26)) {
        failed = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  };

  for (int b = R.hi[kr] - w; b >= R.lo[kr] && !failed; b -= PW) {
    const int T = tgb(b);
    const bool has_pred = (b + 1 <= R.hi[kr]);
    const int T1 = has_pred ? tgb(b + 1) : 0;
    const int kb = key_of(nblk, b), kp = has_pred ? key_of(nblk, b + 1) : 0;
    const double* Gb = F2 + goff[b] * (long)GREC;
    double f[NFRAG], rec[NST];
    dbl4 z0, z1, z2, z3, n0, n1;
    ld_rec(Gb, rec);
    put_rec(rec);
    if (has_pred) wait_for(kp + min(1, T1));
    if (failed) break;
    ld4(b * B + 1, z0);
    ld4(b * B + 17, z1);
    ld4(b * B + 33, z2);
    ld4(b * B + 49, z3);
    for (int t = 0; t < T; t++) {
      const int rb = (b + t) * B + 1;  // first row of the group
      const bool more = t + 1 < T;
      if (more) {
        // record and new row block of group t + 1 (the latter needs (b+1, t+1))
        ld_rec(Gb + (long)(t + 1) * GREC, rec);
        if (has_pred) wait_for(kp + min(t + 2, T1));
        if (failed) break;
        ld4(rb + 64, n0);
        ld4(rb + 80, n1);
      }
      get_ops(f);
      // W = V^T Z (two 16-row blocks)
      dbl4 w0 = dbl4{0, 0, 0, 0}, w1 = dbl4{0, 0, 0, 0};
#pragma unroll
      for (int kq = 0; kq < 12; kq++) {
        const dbl4& zq = (kq < 4) ? z0 : (kq < 8) ? z1 : z2;
        w0 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[kq], zq[kq & 3], w0, 0, 0, 0);
      }
#pragma unroll
      for (int kq = 4; kq < 16; kq++) {
        const dbl4& zq = (kq < 8) ? z1 : (kq < 12) ? z2 : z3;
        w1 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[12 + kq - 4], zq[kq & 3], w1, 0, 0, 0);
      }
      // W2 = T W
      dbl4 u0 = dbl4{0, 0, 0, 0}, u1 = dbl4{0, 0, 0, 0};
#pragma unroll
      for (int kq = 0; kq < 8; kq++)
        u0 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[24 + kq], (kq < 4) ? w0[kq] : w1[kq - 4], u0,
                                                  0, 0, 0);
#pragma unroll
      for (int kq = 4; kq < 8; kq++)
        u1 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[32 + kq - 4], w1[kq - 4], u1, 0, 0, 0);
      // Z += (-V) W2
#pragma unroll
      for (int kq = 0; kq < 4; kq++)
        z0 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[36 + kq], u0[kq], z0, 0, 0, 0);
#pragma unroll
      for (int kq = 0; kq < 8; kq++) {
        const double uk = (kq < 4) ? u0[kq] : u1[kq - 4];
        z1 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[40 + kq], uk, z1, 0, 0, 0);
        z2 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[48 + kq], uk, z2, 0, 0, 0);
      }
#pragma unroll
      for (int kq = 4; kq < 8; kq++)
        z3 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[56 + kq - 4], u1[kq - 4], z3, 0, 0, 0);
      st4(rb, z0);
      st4(rb + 16, z1);
      if (!more) {
        st4(rb + 32, z2);
        st4(rb + 48, z3);
      }
      z0 = z2;
      z1 = z3;
      z2 = n0;
      z3 = n1;
      if (more) put_rec(rec);
      publish(kb + t + 1);
    }
  }
  if (failed && lane == 0) dev_set_status(st, DS_SYNC_TIMEOUT, 3);
  // every wavefront's stores reach agent scope before the range is marked done
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&done[strip], kr + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Held to 256 registers per lane so that two wavefronts share each SIMD.
__global__ __launch_bounds__(64 * PW) __attribute__((amdgpu_waves_per_eu(2))) void bt2_strip_kernel(
    int n, int nblk, SplitRanges R, int nstrip, const double* F2, const long* goff, double* Z,
    long ldz, int m_host, const int* m_dev, int* done, DevStatusWord* st) {
  const int m = m_dev ? *m_dev : m_host;
  bt2_strip_body(n, nblk, R, nstrip, F2, goff, Z, ldz, m, done, st, blockIdx.x);
}

// Several Z's in one launch: workgroup blockIdx.x is workgroup
// blk_task[2 blockIdx.x + 1] of task blk_task[2 blockIdx.x] (the host orders
// them so that a range still waits only for a workgroup with a lower index).
__global__ __launch_bounds__(64 * PW) __attribute__((amdgpu_waves_per_eu(2))) void bt2_group_kernel(
    const Bt2Task* tasks, const int* blk_task) {
  const int p = __builtin_amdgcn_readfirstlane(blk_task[2 * blockIdx.x]);
  const int blk = __builtin_amdgcn_readfirstlane(blk_task[2 * blockIdx.x + 1]);
  const Bt2Task& q = tasks[p];
  const int m = q.m_dev ? *q.m_dev : q.m;
  bt2_strip_body(q.n, q.nblk, q.R, q.nstrip, q.F2, q.goff, q.Z, q.ldz, m, q.done, q.st, blk);
}

}  // namespace

size_t bt2_pack_doubles(const Sb2stLayout& L) { return (size_t)L.ngroups * GREC; }

hipError_t bt2_prepare(const Sb2stLayout& L, const double* V2, const double* tau2, double* F2,
                       hipStream_t s) {
  if (L.ngroups <= 0) return hipSuccess;
  HSDM_LAUNCH(group_pack_kernel, dim3((unsigned)L.ngroups), dim3(256), 0, s, V2, tau2, F2);
  return hipGetLastError();
}

Bt2Task bt2_task(const Sb2stLayout& L, const double* F2, const long* d_goff, double* Z,
                 long ldz, int m, const int* m_dev, int* iscratch, DevStatusWord* st) {
  const int n = L.n, nblk = L.nblk;
  // sweep-block ranges of about equal work (tasks), last blocks first
  auto tgb = [&](int b) { return (n - 1 - b * B + B - 1) / B; };
  long tot = 0;
  for (int b = 0; b < nblk; b++) tot += tgb(b);
  Bt2Task q{};
  int b = nblk - 1;
  for (int k = 0; k < NSPLIT; k++) {
    q.R.hi[k] = b;
    const long want = tot * (k + 1) / NSPLIT;
    long acc = 0;
    for (int r = nblk - 1; r > b; r--) acc += tgb(r);
    while (b >= 0 && (acc < want || k == NSPLIT - 1)) acc += tgb(b--);
    q.R.lo[k] = b + 1;
  }
  q.n = n;
  q.nblk = nblk;
  q.nstrip = ceil_div(m, 16);
  q.F2 = F2;
  q.goff = d_goff;
  q.Z = Z;
  q.ldz = ldz;
  q.m = m;
  q.m_dev = m_dev;
  q.done = iscratch;
  q.st = st;
  return q;
}

double bt2_flops(const Sb2stLayout& L, int m) {
  // algorithmic: each of the B reflectors of a group (length B) applied to a
  // column of Z is 4 B flops (about 2 n^2 m in all); the product with the
  // block reflector's triangular factor T is this kernel's own extra work
  // and is not counted
  return 4.0 * (double)L.ngroups * B * B * m;
}

hipError_t bt2_apply(const Sb2stLayout& L, const double* F2, const long* d_goff, double* Z,
                     long ldz, int m, const int* m_dev, int* iscratch, DevStatusWord* st,
                     hipStream_t s) {
  if (L.ngroups <= 0 || m <= 0) return hipSuccess;
  const Bt2Task q = bt2_task(L, F2, d_goff, Z, ldz, m, m_dev, iscratch, st);
  HSDM_LAUNCH(fill_i32_kernel, dim3(ceil_div(q.nstrip, 256)), dim3(256), 0, s, iscratch,
                     q.nstrip);
  HSDM_TRY(hipGetLastError());
  if (coop_get_shared()) {
    // beside other solves: one workgroup per strip applies every sweep
    // block (range 0 is all of them), so no workgroup waits for another; the
    // groups reach each column in the same order as with eight ranges
    SplitRanges R1 = q.R;
    for (int k = 0; k < NSPLIT; k++) {
      R1.hi[k] = -1;
      R1.lo[k] = 0;
    }
    R1.hi[0] = q.nblk - 1;
    R1.lo[0] = 0;
    kt_begin("bt2_strip_kernel", bt2_flops(L, m), 0.0, m_dev ? m : 0, s, true);
    HSDM_LAUNCH(bt2_strip_kernel, dim3(q.nstrip), dim3(64 * PW), 0, s, q.n, q.nblk, R1, q.nstrip,
                F2, d_goff, Z, ldz, m, m_dev, iscratch, st);
    kt_end(s);
    return hipGetLastError();
  }
  // workgroups wait for lower-numbered ones: a spinning kernel (see coop_launch)
  int n_ = q.n, nblk = q.nblk, nstrip = q.nstrip, m_ = m;
  SplitRanges R = q.R;
  long ldz_ = ldz;
  void* args[] = {(void*)&n_, (void*)&nblk, (void*)&R, (void*)&nstrip, (void*)&F2,
                  (void*)&d_goff, (void*)&Z, (void*)&ldz_, (void*)&m_, (void*)&m_dev,
                  (void*)&iscratch, (void*)&st};
  return coop_launch("bt2_strip_kernel", bt2_flops(L, m), 0.0, true, false,
                     (const void*)bt2_strip_kernel, dim3(q.nstrip * NSPLIT), dim3(64 * PW), args,
                     s, m_dev ? m : 0);
}

size_t bt2_group_map_ints(int nt, const Bt2Task* tasks) {
  size_t c = 0;
  for (int i = 0; i < nt; i++) c += (size_t)tasks[i].nstrip * NSPLIT;
  return 2 * c;
}

// Workgroup order of the grouped launch: range by range, and within a range
// task by task, strip by strip, so that a workgroup's predecessor (the
// previous range of its strip) has a lower index and the workgroups resident
// at any time are mostly of one range, not waiting.  The map holds (task,
// workgroup within the task) per workgroup.
hipError_t bt2_group_apply(int nt, Bt2Task* tasks, std::vector<int>& hmap, Bt2Task* d_tasks,
                           int* d_map, hipStream_t s) {
  hmap.clear();
  int b0 = 0;  // workgroups of the launch
  for (int i = 0; i < nt; i++) {
    Bt2Task& q = tasks[i];
    q.b0 = b0;
    const int cnt = (q.nblk > 0 && q.m > 0) ? q.nstrip * NSPLIT : 0;
    b0 += cnt;
    if (cnt > 0) {
      HSDM_LAUNCH(fill_i32_kernel, dim3(ceil_div(q.nstrip, 256)), dim3(256), 0, s, q.done,
                         q.nstrip);
      HSDM_TRY(hipGetLastError());
    }
  }
  for (int k = 0; k < NSPLIT; k++)
    for (int i = 0; i < nt; i++) {
      const Bt2Task& q = tasks[i];
      if (q.nblk <= 0 || q.m <= 0) continue;
      for (int strip = 0; strip < q.nstrip; strip++) {
        hmap.push_back(i);
        hmap.push_back(k * q.nstrip + strip);
      }
    }
  if (b0 == 0) return hipSuccess;
  HSDM_TRY(hipMemcpyAsync(d_tasks, tasks, sizeof(Bt2Task) * nt, hipMemcpyHostToDevice, s));
  HSDM_TRY(hipMemcpyAsync(d_map, hmap.data(), sizeof(int) * hmap.size(), hipMemcpyHostToDevice,
                          s));
  void* args[] = {(void*)&d_tasks, (void*)&d_map};
  return coop_launch("bt2_group_kernel", 0.0, 0.0, true, false, (const void*)bt2_group_kernel,
                     dim3(b0), dim3(64 * PW), args, s);
}

namespace {

// ---- stage 1 ------------------------------------------------------------------
// GP consecutive panels form one block reflector of width W = GP*B:
//   (I - V1 T1 V1^T)(I - V2 T2 V2^T) = I - [V1 V2] [[T1, -T1 V1^T V2 T2], [0, T2]] [V1 V2]^T
// applied panel group by panel group, last group first.  The explicit panel
// reflectors are zero above their first row, so the grouped V is dense with a
// staircase of zeros.  T of a group is built from the panel T's by doubling
// the block size: at each level the blocks of size b pair up and the
// off-diagonal block of the pair is -T_a (G_ab T_b), G = V^T V, two batched
// products for all pairs of all groups.  A wide group makes the update of Z
// (read and written once per group) compute-bound.
constexpr int GP = 16;

__global__ void group_t_init_kernel(int ngroup, int np_all, int Bp, const double* T1p,
                                    double* Tall) {
  // Tall[q] (W x W): the panel T's on the diagonal, zero elsewhere
  const int W = GP * Bp;
  const long tot = (long)ngroup * W * W;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const int q = (int)(e / ((long)W * W));
    const int rc = (int)(e % ((long)W * W));
    const int r = rc % W, c = rc / W;
    const int pr = r / Bp, pc = c / Bp, p = q * GP + pr;
    double v = 0.0;
    if (pr == pc && p < np_all) v = T1p[(size_t)p * Bp * Bp + (r % Bp) + (size_t)(c % Bp) * Bp];
    Tall[e] = v;
  }
}

// Descriptors of one doubling level (block size b): for group q and pair j,
// a = rows [2jb, (2j+1)b), c = columns [(2j+1)b, (2j+2)b) of the group, both
// cut to the group's width w:  X = G[a, c] T[c, c];  T[a, c] = -T[a, a] X.
__global__ void group_t_desc_kernel(int ngroup, int np_all, int Bp, int b, const double* Gall,
                                    double* Tall, double* Xall, GemmDesc* d1, GemmDesc* d2) {
  const int W = GP * Bp, pairs = W / (2 * b);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ngroup * pairs) return;
  const int q = idx / pairs, j = idx % pairs;
  const int w = min(GP, np_all - q * GP) * Bp;
  const int a0 = 2 * j * b, c0 = a0 + b;
  const int ma = max(0, min(b, w - a0)), nc = max(0, min(b, w - c0));
  const double* G = Gall + (size_t)q * W * W;
  double* T = Tall + (size_t)q * W * W;
  double* X = Xall + (size_t)idx * b * b;
  GemmDesc e{};
  e.m = (nc > 0) ? ma : 0; e.n = nc; e.k = nc;
  e.A = G + a0 + (long)c0 * W; e.lda = W;
  e.B = T + c0 + (long)c0 * W; e.ldb = W;
  e.C = X; e.ldc = b;
  d1[idx] = e;
  GemmDesc f{};
  f.m = (nc > 0) ? ma : 0; f.n = nc; f.k = ma;
  f.A = T + a0 + (long)a0 * W; f.lda = W;
  f.B = X; f.ldb = b;
  f.C = T + a0 + (long)c0 * W; f.ldc = W;
  d2[idx] = f;
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

// Panels the full-to-band reduction produced: panel p has rows below
// (p + 1) B, so it exists iff (p + 1) B < n.
static int npanel_of(int n, int B_) { return (n > B_) ? ceil_div(n - B_, B_) : 0; }

namespace {
constexpr int BT1_MAXSPLIT = 4;    // split-K slices of V^T Z
constexpr int BT1_GCHUNK = 2048;   // k slice of the Gram products
}  // namespace

size_t bt1_scratch_doubles(int n, int B_, int m) {
  const size_t W = (size_t)GP * B_;
  const size_t ngroup = ceil_div(npanel_of(n, B_), GP) + 1;
  const size_t gsplit = ceil_div(n, BT1_GCHUNK) + 1;
  const size_t ndesc = ngroup * GP;
  // V^T Z and T (V^T Z) (W x m each), split-K partials, one group's V^T
  // (W x n), the Gram of every group with the partials of one, T of every
  // group, the pair products of one level, two descriptor arrays
  return W * m * (2 + BT1_MAXSPLIT) + W * (size_t)n + W * W * (2 * ngroup + gsplit) +
         ngroup * W * W / 2 + 2 * ndesc * (sizeof(GemmDesc) / sizeof(double) + 1) + 64;
}

hipError_t bt1_zero_fill(int n, int B_, double* Vst, long ldv, hipStream_t s) {
  const long tot = (long)n * n;
  HSDM_LAUNCH(zero_upper_panels_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     s, n, B_, Vst, ldv);
  return hipGetLastError();
}

namespace {

// Gram matrices and T of every panel group (FP64, from the FP64 reflectors)
// into the scratch; returns the pointers the application needs.
struct Bt1Groups {
  int np_all, W, ngroup;
  double *Wb, *W2, *part, *Vt, *Tall;
};

hipError_t bt1_groups(int n, int B_, const double* Vst, long ldv, const double* T1, int m,
                      double* scratch, Bt1Groups& out, hipStream_t s) {
  const int np_all = npanel_of(n, B_);
  const int W = GP * B_;
  const int ngroup = ceil_div(np_all, GP);
  const size_t gsplit = ceil_div(n, BT1_GCHUNK) + 1;
  const size_t ndesc = (size_t)ngroup * GP;
  double* Wb = scratch;
  double* W2 = Wb + (size_t)W * m;
  double* part = W2 + (size_t)W * m;
  double* Vt = part + (size_t)BT1_MAXSPLIT * W * m;
  double* Gall = Vt + (size_t)W * n;
  double* Tall = Gall + (size_t)ngroup * W * W;
  double* Gpart = Tall + (size_t)ngroup * W * W;
  double* Xall = Gpart + gsplit * W * W;
  GemmDesc* d1 = reinterpret_cast<GemmDesc*>(Xall + (size_t)ngroup * W * W / 2);
  GemmDesc* d2 = d1 + ndesc;
  out = Bt1Groups{np_all, W, ngroup, Wb, W2, part, Vt, Tall};
  // Gram V_q^T V_q of every group (upper blocks are used)
  for (int q = 0; q < ngroup; q++) {
    const int p0 = q * GP, np = min(GP, np_all - p0);
    if (np < 2) continue;
    const int r0 = (p0 + 1) * B_, h = n - r0, w = np * B_;
    const double* Vq = Vst + r0 + (long)p0 * B_ * ldv;
    GemmArgs g{};
    g.m = w; g.n = w; g.k = h; g.A = Vq; g.lda = ldv; g.B = Vq; g.ldb = ldv;
    g.C = Gall + (size_t)q * W * W; g.ldc = W;
    g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0;
    HSDM_TRY(gemm_splitk_launch(g, BT1_GCHUNK, Gpart, s));
  }
  // T of every group: panel T's on the diagonal, then the doubling levels
  HSDM_LAUNCH(group_t_init_kernel, dim3(1024), dim3(256), 0, s, ngroup, np_all, B_, T1,
                     Tall);
  HSDM_TRY(hipGetLastError());
  for (int b = B_; b < W; b *= 2) {
    const int cnt = ngroup * (W / (2 * b));
    HSDM_LAUNCH(group_t_desc_kernel, dim3(ceil_div(cnt, 64)), dim3(64), 0, s, ngroup,
                       np_all, B_, b, Gall, Tall, Xall, d1, d2);
    HSDM_TRY(hipGetLastError());
    HSDM_TRY(gemm_batched_dense_launch(d1, cnt, b, b, 1.0, 0.0, GF_KB_UPPER, s));
    HSDM_TRY(gemm_batched_dense_launch(d2, cnt, b, b, -1.0, 0.0, GF_KA_UPPER, s));
  }
  return hipSuccess;
}

// Vt (w x h, leading dimension w) = V^T for V h x w (leading dimension ldv):
// 32 x 32 tiles through LDS, so that both the reads and the writes coalesce
template <class T>
__global__ __launch_bounds__(256) void transpose_kernel(int h, int w, const T* V, long ldv, T* Vt) {
  __shared__ T tile[32][33];
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int i = i0 + tx, j = j0 + k;
    tile[k][tx] = (i < h && j < w) ? V[i + (long)j * ldv] : T(0);
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int j = j0 + tx, i = i0 + k;
    if (i < h && j < w) Vt[j + (long)i * w] = tile[tx][k];
  }
}

// Z <- (I - V_q T_q V_q^T) Z for the groups q, last first, in element type T
// (V, Tall, Z and the work buffers Wb, W2, part of that type).  With Vt
// (room for w x h) each group's V^T is formed there first, so that V^T Z
// reads its A operand along its columns, as the 128 x 128 tiles stage it.
template <class T>
hipError_t bt1_groups_apply(int n, int B_, const Bt1Groups& G_, const T* V, long ldv,
                            const T* Tall, T* Z, long ldz, int m, const int* m_dev, T* Wb, T* W2,
                            T* part, T* Vt, hipStream_t s) {
  const int W = G_.W;
  for (int q = G_.ngroup - 1; q >= 0; q--) {
    const int p0 = q * GP, np = min(GP, G_.np_all - p0);
    const int r0 = (p0 + 1) * B_, h = n - r0, w = np * B_;
    if (h <= 0) continue;
    const T* Vq = V + r0 + (long)p0 * B_ * ldv;
    const T* Tq = Tall + (size_t)q * W * W;
    T* Zq = Z + r0;
    // V^T Z: split K so that the product fills the chip.  With the vectors
    // counted on the device m is only a bound: the split then follows the
    // rows alone.
    const long tiles = (long)ceil_div(w, 128) * ceil_div(m, 128);
    int nsp = m_dev ? std::min(BT1_MAXSPLIT, std::max(1, h / 2048))
                    : (int)std::min<long>(BT1_MAXSPLIT, std::max<long>(1, ceil_div(512, (int)tiles)));
    int kchunk = ceil_div(ceil_div(h, nsp), 16) * 16;
    GemmArgsT<T> g{};
    g.m = w; g.n = m; g.k = h; g.A = Vq; g.lda = ldv; g.B = Zq; g.ldb = ldz; g.C = Wb; g.ldc = w;
    g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0; g.ndev = m_dev;
    if (Vt) {
      HSDM_LAUNCH(transpose_kernel<T>, dim3(ceil_div(h, 32), ceil_div(w, 32)), dim3(256), 0, s, h,
                  w, Vq, ldv, Vt);
      HSDM_TRY(hipGetLastError());
      g.A = Vt; g.lda = w; g.ta = 0;
    }
    HSDM_TRY(gemm_splitk_launch(g, kchunk, part, s));
    g = GemmArgsT<T>{};
    g.m = w; g.n = m; g.k = w; g.A = Tq; g.lda = W; g.B = Wb; g.ldb = w; g.C = W2; g.ldc = w;
    g.alpha = 1.0; g.beta = 0.0; g.flags = GF_KA_UPPER; g.ndev = m_dev;
    HSDM_TRY(gemm_launch(g, s));
    g = GemmArgsT<T>{};
    g.m = h; g.n = m; g.k = w; g.A = Vq; g.lda = ldv; g.B = W2; g.ldb = w; g.C = Zq; g.ldc = ldz;
    g.alpha = -1.0; g.beta = 1.0; g.ndev = m_dev;
    HSDM_TRY(gemm_launch(g, s));
  }
  return hipSuccess;
}

}  // namespace

hipError_t bt1_apply(int n, int B_, const double* Vst, long ldv, const double* T1, double* Z,
                     long ldz, int m, const int* m_dev, double* scratch, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (npanel_of(n, B_) == 0) return hipSuccess;
  Bt1Groups G_;
  HSDM_TRY(bt1_groups(n, B_, Vst, ldv, T1, m, scratch, G_, s));
  return bt1_groups_apply<double>(n, B_, G_, Vst, ldv, G_.Tall, Z, ldz, m, m_dev, G_.Wb, G_.W2,
                                  G_.part, G_.Vt, s);
}

size_t bt1_f32_scratch_floats(int n, int B_, int m) {
  const size_t W = (size_t)GP * B_;
  const size_t ngroup = ceil_div(npanel_of(n, B_), GP) + 1;
  return W * m * (2 + BT1_MAXSPLIT) + ngroup * W * W + 64;
}

hipError_t bt1_apply_f32(int n, int B_, const double* Vst, long ldv, const float* V32,
                         long ldv32, const double* T1, float* Z, long ldz, int m,
                         const int* m_dev, double* scratch, float* scratch32, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (npanel_of(n, B_) == 0) return hipSuccess;
  Bt1Groups G_;
  HSDM_TRY(bt1_groups(n, B_, Vst, ldv, T1, m, scratch, G_, s));
  const int W = G_.W;
  float* Wb = scratch32;
  float* W2 = Wb + (size_t)W * m;
  float* part = W2 + (size_t)W * m;
  float* Tall = part + (size_t)BT1_MAXSPLIT * W * m;
  HSDM_TRY(dev_convert(G_.Tall, W, Tall, W, W, G_.ngroup * W, s));
  return bt1_groups_apply<float>(n, B_, G_, V32, ldv32, Tall, Z, ldz, m, m_dev, Wb, W2, part,
                                 (float*)nullptr, s);
}
