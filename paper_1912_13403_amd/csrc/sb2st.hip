// Stage 2 of the two-stage tridiagonalization: band (half-bandwidth B) ->
// symmetric tridiagonal by bulge chasing.
//
// Sweep s removes column s below the subdiagonal.  Its task t owns the rows
// R_t = [s+1+tB, s+(t+1)B]:
//   - t = 0 first builds the reflector from column s (rows R_0);
//   - the current reflector is applied on both sides of the diagonal block
//     R_t x R_t and from the right to the block R_{t+1} x R_t below it, which
//     fills that block (the bulge);
//   - the next reflector is built from the first column of that block and
//     applied from the left to the rest of it; it is handed to task t+1.
// Task (s, t) touches only what tasks (s-1, t) and (s-1, t+1) wrote, so sweep
// s may run task t once sweep s-1 has finished task t+1: sweeps proceed as a
// pipeline, each two tasks behind its predecessor.
//
// One wavefront runs one sweep at a time (64 lanes; the two B x B blocks of
// a task live in registers, sums over lanes use DPP and permlane swaps).
// Workgroups of two wavefronts are launched cooperatively so that every
// wavefront is resident; consecutive sweeps run on consecutive wavefronts,
// so a workgroup holds two consecutive sweeps and the sweeps in flight (about
// n / 2B of them, each two tasks behind its predecessor) spread over many
// compute units, one or two per unit.  (Eight wavefronts per workgroup kept
// all sweeps in flight on a few compute units, whose memory pipelines then
// set the pace: 212 ms against 112 ms for n = 16384.)
//
// Every band load and store is an agent-scope relaxed atomic: written
// through to, and read from, the memory side shared by all XCDs.  No L2 then
// holds band data that another XCD would miss, or could write back over a
// newer value later, so a hand-off needs no L2 write-back or invalidation:
// the producer waits for its own stores to complete (s_waitcnt vmcnt(0)) and
// raises a counter (in LDS inside a workgroup, in global memory between
// workgroups), the consumer polls it and then loads.  Every wait is bounded
// and reports through the status word if it runs out.
//
// Storage: lower band storage AB[(r-c) + c*ldab], ldab = 2B (offsets up to
// 2B-1 hold the bulge).  Each reflector H_{s,t} (v, tau; v[0] = 1) is stored
// for the back-transformation in group (s / B, t): a 2B x B block whose
// column s % B holds v at rows (s % B) .. (s % B) + len - 1.
#include "hsdm_internal.h"
#include "hsdm_phases.h"

namespace {

constexpr int WPB = 2;  // wavefronts per workgroup
constexpr int DONE = 1 << 30;      // global counter of a finished sweep
constexpr int KROUND = 1 << 20;    // LDS counters: KROUND * round + tasks done
constexpr int KDONE = 1 << 19;     //   ... + KDONE once the sweep is finished

// Orders LDS accesses between the lanes of one wavefront: the LDS executes a
// wavefront's instructions in order, so a compiler barrier is enough (no wait
// on outstanding global memory operations).
HSDM_DEV void wave_sync() {
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

template <int CTRL>
HSDM_DEV double dpp(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

HSDM_DEV double first_lane(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

HSDM_DEV long uniform(long v) {
  const unsigned long long u = (unsigned long long)v;
  const unsigned lo = __builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return (long)(((unsigned long long)hi << 32) | lo);
}

HSDM_DEV double join(unsigned lo, unsigned hi) {
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// v + (the value of lane ^ 16): v_permlane16_swap of each 32-bit half gives
// the even rows' value and the odd rows' value (rows of 16 lanes) in every lane.
HSDM_DEV double xor16_sum(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
  const auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return join(pl[0], ph[0]) + join(pl[1], ph[1]);
}

// v + (the value of lane ^ 32), by v_permlane32_swap.
HSDM_DEV double xor32_sum(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
  const auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return join(pl[0], ph[0]) + join(pl[1], ph[1]);
}

// Sum over the 8 lanes 8I .. 8I+7 (lane xor 1, xor 2, then the mirror lane
// inside the half row, which lies in the other quad).
HSDM_DEV double sum8(double v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  return v;
}

// Sum over the 8 lanes J, J+8, .., J+56 (lane xor 8 by a rotation by 8
// inside rows of 16, then xor 16 and xor 32).
HSDM_DEV double sumI(double v) {
  v += dpp<0x128>(v);
  v = xor16_sum(v);
  return xor32_sum(v);
}

// The value of lane 8I in every lane 8I .. 8I+7: the first lane of each quad
// to the quad, then lanes 4..7 of each half row take lane 0's copy (row
// shift right by 4, written to banks 1 and 3 only).
HSDM_DEV double bcast8(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, 0x00, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x00, 0xF, 0xF, false);
  lo = __builtin_amdgcn_update_dpp(lo, lo, 0x114, 0xF, 0xA, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, 0x114, 0xF, 0xA, false);
  return join((unsigned)lo, (unsigned)hi);
}

// Hand-offs between the wavefronts of one workgroup: a counter in LDS.
HSDM_DEV void wait_lds(int* p, int target, DevStatusWord* st) {
  long spins = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
    if (++spins > (1L << 27)) {
      if ((threadIdx.x & 63) == 0) dev_set_status(st, DS_SYNC_TIMEOUT, 2);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  wave_sync();
}

// Band loads and stores: agent-scope relaxed atomics (sc1).
HSDM_DEV double band_ld(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

HSDM_DEV void band_st(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// All of this wave's memory operations have completed before what follows.
HSDM_DEV void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Sweep s waits for sweep s-1 on another workgroup: lane 0 polls the global
// counter with agent-scope relaxed loads (they miss the compute unit's
// cache); the band loads that follow are coherent by themselves, so a
// workgroup-scope fence (ordering only) ends the wait.
HSDM_DEV void wait_global(int* p, int target, DevStatusWord* st) {
  if ((threadIdx.x & 63) == 0) {
    long spins = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      ++spins;
      if (spins > (1L << 27) ||
          ((spins & 4095) == 0 &&
           __hip_atomic_load(&st->code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
        dev_set_status(st, DS_SYNC_TIMEOUT, 2);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  wave_sync();
}

// The wave's band stores are complete, then the counter is raised.
HSDM_DEV void publish_lds(int* p, int v) {
  wave_sync();
  stores_done();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

HSDM_DEV void publish_global(int* p, int v) {
  wave_sync();
  stores_done();
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reflector from x (x[0] = alpha, sig = sum of x[i]^2 over i >= 1):
// H = I - tau v v^T, v[0] = 1, H x = beta e_0 (LAPACK's dlarfg convention
// without the rescaling loop).
HSDM_DEV void make_reflector(double alpha, double sig, double& beta, double& tau, double& scal) {
  beta = alpha;
  tau = 0.0;
  scal = 0.0;
  if (sig > 0.0) {
    const double nrm = sqrt(alpha * alpha + sig);
    beta = (alpha >= 0.0) ? -nrm : nrm;
    tau = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
}

// A task works on two B x B blocks (B = 32): the diagonal block D (rows and
// columns R_t, held in full although only its lower triangle is stored) and
// the block K below it (rows R_{t+1}, columns R_t).  Lane l = 8 I + J holds
// the 16 elements (I + 8a, J + 8b), a, b < 4, of each block in registers, so
// that a product with a vector is 16 FMAs per lane plus a sum over the 8
// lanes of a row group (sum8) or of a column group (sumI), and the rank-one
// and rank-two updates need no data from other lanes.  The reflector v is
// kept in both index sets (rows I + 8a, columns J + 8b); one copy through LDS
// per task turns the row form of the next reflector into the column form.
// Workgroup wg of the nwg that chase the bulges of one band: wavefront w of
// the workgroup takes sweeps wg * WPB + w, then that plus nwg * WPB, and so on.
template <int B>
HSDM_DEV void sb2st_body(int n, int nsweep, double* AB, int ldab, double* V2, double* tau2,
                         const long* goff, int* progress, DevStatusWord* st, int wg, int nwg) {
  static_assert(B == 32, "8 x 8 lanes, 4 x 4 elements each");
  __shared__ double vl_all[WPB][B];
  __shared__ int lprog[WPB];
  const int lane = threadIdx.x & 63, wv_id = threadIdx.x >> 6;
  if (lane == 0) lprog[wv_id] = -1;
  __syncthreads();
  double* vl = vl_all[wv_id];
  const int gw = wg * WPB + wv_id, TW = nwg * WPB;
  const int I = lane >> 3, J = lane & 7;
  // Element (i, j), i >= j, of a block whose first row and column is r sits
  // at (i - j) + (r + j) LD = (r LD) + i + (LD - 1) j in the band storage.
  // With i = I + 8a, j = J + 8b that is a per-lane base (P for i >= j, Q for
  // the transposed position of i < j) plus a constant.
  constexpr int LD = 2 * B;
  const int P = I + (LD - 1) * J, Q = J + (LD - 1) * I, M = (I >= J) ? P : Q;
  auto offl = [&](int a, int b) { return P + 8 * a + 8 * (LD - 1) * b; };
  auto offd = [&](int a, int b) {
    return a > b ? P + 8 * a + 8 * (LD - 1) * b
                 : (a < b ? Q + 8 * b + 8 * (LD - 1) * a : M + 8 * LD * a);
  };

  for (int s = gw, round = 0; s < nsweep; s += TW, round++) {
    const int ntask = (n - 1 - s + B - 1) / B;
    // sweep s-1 runs on wavefront gw-1: in the same workgroup (LDS counter)
    // unless this is the workgroup's first wavefront (global counter)
    const bool first_wave = (wv_id == 0);
    const bool last_wave = (wv_id == WPB - 1);
    const int kbase = round * KROUND;
    double tau = 0.0;
    double vr[4], vc[4];  // current reflector at rows I + 8a and columns J + 8b
    const long g0 = uniform(goff[s / B]);
    for (int t = 0; t < ntask; t++) {
      if (s > 0) {
        if (first_wave)
          wait_global(progress + s - 1, t + 2, st);
        else
          wait_lds(&lprog[wv_id - 1], kbase + t + 2, st);
      }
      const int rs = s + 1 + t * B;
      const int len = min(B, n - rs);
      const int rs2 = rs + B;
      const int len2 = (rs2 < n) ? min(B, n - rs2) : 0;
      // every address below stays inside the band storage (B + 1 spare
      // columns); values outside the blocks are masked after the loads
      double* const blk = AB + (long)rs * LD;
      double d[4][4], k[4][4];
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) {
          d[a][b] = band_ld(blk + offd(a, b));
          k[a][b] = band_ld(blk + B + offl(a, b));
        }
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) {
          const int i = I + 8 * a, j = J + 8 * b;
          d[a][b] = (i < len && j < len) ? d[a][b] : 0.0;
          k[a][b] = (i < len2 && j < len) ? k[a][b] : 0.0;
        }
      if (t == 0) {
        // reflector from column s, rows s+1 .. s+len
        double xr[4], xc[4];
#pragma unroll
        for (int a = 0; a < 4; a++) {
          const int i = I + 8 * a, j = J + 8 * a;
          xr[a] = (i < len) ? band_ld(AB + (1 + i) + (long)s * LD) : 0.0;
          xc[a] = (j < len) ? band_ld(AB + (1 + j) + (long)s * LD) : 0.0;
        }
        const double alpha = first_lane(xr[0]);
        double ps = 0.0;
#pragma unroll
        for (int a = 0; a < 4; a++) ps += (I + 8 * a >= 1) ? xr[a] * xr[a] : 0.0;
        const double sig = first_lane(sumI(ps));
        double beta, scal;
        make_reflector(alpha, sig, beta, tau, scal);
#pragma unroll
        for (int a = 0; a < 4; a++) {
          const int i = I + 8 * a, j = J + 8 * a;
          vr[a] = (i == 0) ? 1.0 : xr[a] * scal;
          vc[a] = (j == 0) ? 1.0 : xc[a] * scal;
        }
        if (J == 0) {
#pragma unroll
          for (int a = 0; a < 4; a++) {
            const int i = I + 8 * a;
            vl[i] = vr[a];
            if (i < len) band_st(AB + (1 + i) + (long)s * LD, (i == 0) ? beta : 0.0);
          }
        }
        wave_sync();
      }
      // store H_{s,t} for the back-transformation (v is in LDS)
      {
        const int kk = s % B;
        const long gi = g0 + t;
        double* col = V2 + (gi * B + kk) * (long)(2 * B);
        const int r = lane - kk;
        col[lane] = (r >= 0 && r < len) ? vl[r] : 0.0;
        if (lane == 0) tau2[gi * B + kk] = tau;
      }
      // two-sided update of D: y = tau D v, w = y - (tau/2)(v.y) v,
      // D <- D - v w^T - w v^T (y and w in both index sets)
      {
        double yr[4], yc[4];
#pragma unroll
        for (int a = 0; a < 4; a++) {
          double p = 0.0;
#pragma unroll
          for (int b = 0; b < 4; b++) p += d[a][b] * vc[b];
          yr[a] = p;
        }
#pragma unroll
        for (int b = 0; b < 4; b++) {
          double p = 0.0;
#pragma unroll
          for (int a = 0; a < 4; a++) p += d[a][b] * vr[a];
          yc[b] = p;
        }
#pragma unroll
        for (int a = 0; a < 4; a++) yr[a] = tau * sum8(yr[a]);
#pragma unroll
        for (int b = 0; b < 4; b++) yc[b] = tau * sumI(yc[b]);
        double pv = 0.0;
#pragma unroll
        for (int a = 0; a < 4; a++) pv += vr[a] * yr[a];
        const double h = 0.5 * tau * sumI(pv);
#pragma unroll
        for (int a = 0; a < 4; a++) {
          yr[a] -= h * vr[a];
          yc[a] -= h * vc[a];
        }
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
          for (int b = 0; b < 4; b++) d[a][b] -= vr[a] * yc[b] + yr[a] * vc[b];
      }
      double tau_n = 0.0, vnr[4] = {0.0, 0.0, 0.0, 0.0}, vnc[4] = {0.0, 0.0, 0.0, 0.0};
      if (len2 > 0) {
        // right application to K: K <- K (I - tau v v^T)
#pragma unroll
        for (int a = 0; a < 4; a++) {
          double p = 0.0;
#pragma unroll
          for (int b = 0; b < 4; b++) p += k[a][b] * vc[b];
          const double z = tau * sum8(p);
#pragma unroll
          for (int b = 0; b < 4; b++) k[a][b] -= z * vc[b];
        }
        // next reflector from column 0 of K (lanes J = 0, b = 0)
        double xr[4];
#pragma unroll
        for (int a = 0; a < 4; a++) xr[a] = bcast8(k[a][0]);
        const double alpha = first_lane(xr[0]);
        double ps = 0.0;
#pragma unroll
        for (int a = 0; a < 4; a++) ps += (I + 8 * a >= 1) ? xr[a] * xr[a] : 0.0;
        const double sig = first_lane(sumI(ps));
        double beta, scal;
        make_reflector(alpha, sig, beta, tau_n, scal);
#pragma unroll
        for (int a = 0; a < 4; a++) vnr[a] = (I + 8 * a == 0) ? 1.0 : xr[a] * scal;
        if (J == 0) {
#pragma unroll
          for (int a = 0; a < 4; a++) vl[I + 8 * a] = vnr[a];
        }
        wave_sync();
#pragma unroll
        for (int b = 0; b < 4; b++) vnc[b] = vl[J + 8 * b];
        // left application to columns 1..: K <- (I - tau_n vn vn^T) K
#pragma unroll
        for (int b = 0; b < 4; b++) {
          double p = 0.0;
#pragma unroll
          for (int a = 0; a < 4; a++) p += vnr[a] * k[a][b];
          const double w = tau_n * sumI(p);
          const int j = J + 8 * b;
#pragma unroll
          for (int a = 0; a < 4; a++) {
            const int i = I + 8 * a;
            k[a][b] = (j == 0) ? ((i == 0) ? beta : 0.0) : k[a][b] - vnr[a] * w;
          }
        }
      }
      // write back the lower triangle of D and all of K
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) {
          const int i = I + 8 * a, j = J + 8 * b;
          if (i >= j && i < len) band_st(blk + offl(a, b), d[a][b]);
          if (i < len2 && j < len) band_st(blk + B + offl(a, b), k[a][b]);
        }
      tau = tau_n;
#pragma unroll
      for (int a = 0; a < 4; a++) {
        vr[a] = vnr[a];
        vc[a] = vnc[a];
      }
      publish_lds(&lprog[wv_id], kbase + t + 1);
      if (last_wave) publish_global(progress + s, t + 1);
    }
    publish_lds(&lprog[wv_id], kbase + KDONE);
    if (last_wave) publish_global(progress + s, DONE);
  }
}

template <int B>
__global__ __launch_bounds__(64 * WPB) void sb2st_kernel(int n, int nsweep, double* AB, int ldab,
                                                         double* V2, double* tau2,
                                                         const long* goff, int* progress,
                                                         DevStatusWord* st) {
  sb2st_body<B>(n, nsweep, AB, ldab, V2, tau2, goff, progress, st, blockIdx.x, gridDim.x);
}

// Several bands in one cooperative launch: workgroups wg0 .. wg0 + nwg - 1 of
// the grid chase the bulges of task p = wg_task[blockIdx.x], each task with
// its own band, reflector store, counters and status word.  All workgroups of
// the grid are resident together, as in the single-band launch.
template <int B>
__global__ __launch_bounds__(64 * WPB) void sb2st_group_kernel(const Sb2stTask* tasks,
                                                               const int* wg_task) {
  const int p = __builtin_amdgcn_readfirstlane(wg_task[blockIdx.x]);
  const Sb2stTask& q = tasks[p];
  sb2st_body<B>(q.n, q.nsweep, q.AB, 2 * B, q.V2, q.tau2, q.goff, q.progress, q.st,
                (int)blockIdx.x - q.wg0, q.nwg);
}

__global__ void extract_tridiag_kernel(int n, const double* AB, int ldab, double* d, double* e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  d[i] = AB[(long)i * ldab];
  if (i + 1 < n) e[i] = AB[1 + (long)i * ldab];
}

__global__ void fill_int_kernel(int* p, long n, int v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_dbl_kernel(double* p, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

}  // namespace

// Workgroups of kernel fn (one of the two chasing kernels) that can be
// resident together on the current device.
static hipError_t resident_wg(const void* fn, int& out) {
  int per_cu = 0, ncu = 0, dev = 0;
  HSDM_TRY(hipGetDevice(&dev));
  HSDM_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HSDM_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * WPB, 0));
  out = per_cu * ncu;
  return out > 0 ? hipSuccess : hipErrorInvalidConfiguration;
}

Sb2stLayout sb2st_layout(int n, int B) {
  Sb2stLayout L{};
  L.n = n;
  L.B = B;
  L.nsweep = n >= 3 ? n - 2 : 0;
  L.nblk = (L.nsweep + B - 1) / B;
  L.tmax = n >= 2 ? (n - 1 + B - 1) / B : 0;
  long g = 0;
  for (int sb = 0; sb < L.nblk; sb++) g += (n - 1 - sb * B + B - 1) / B;
  L.ngroups = g;
  L.v2_doubles = g * 2L * B * B;
  return L;
}

void sb2st_group_offsets(const Sb2stLayout& L, long* offs) {
  long g = 0;
  for (int sb = 0; sb < L.nblk; sb++) {
    offs[sb] = g;
    g += (L.n - 1 - sb * L.B + L.B - 1) / L.B;
  }
  offs[L.nblk] = g;
}

hipError_t sb2st_prepare(const Sb2stLayout& L, double* V2, double* tau2, int* progress,
                         hipStream_t s) {
  if (L.nsweep <= 0) return hipSuccess;
  HSDM_LAUNCH(fill_dbl_kernel, dim3(4096), dim3(256), 0, s, V2, L.v2_doubles);
  HSDM_TRY(hipGetLastError());
  HSDM_LAUNCH(fill_dbl_kernel, dim3(1024), dim3(256), 0, s, tau2, L.ngroups * L.B);
  HSDM_TRY(hipGetLastError());
  HSDM_LAUNCH(fill_int_kernel, dim3(ceil_div(L.nsweep, 256)), dim3(256), 0, s, progress,
                     (long)L.nsweep, 0);
  return hipGetLastError();
}

hipError_t sb2st_finish(const Sb2stLayout& L, const double* AB, int ldab, double* d, double* e,
                        hipStream_t s) {
  HSDM_LAUNCH(extract_tridiag_kernel, dim3(ceil_div(L.n, 256)), dim3(256), 0, s, L.n, AB,
                     ldab, d, e);
  return hipGetLastError();
}

// Algorithmic work of one band: about 6 B n^2 flops; HBM bytes that the
// reduction must move: the band in ((B + 1) n doubles), the stage-2
// reflectors (B per group, B long) and their scalars out, d and e out.  The
// band blocks each task rewrites stay on chip in the ideal schedule and are
// not counted.
double sb2st_algo_flops(const Sb2stLayout& L) { return 6.0 * L.B * (double)L.n * L.n; }
double sb2st_algo_bytes(const Sb2stLayout& L) {
  return 8.0 * ((L.B + 1.0) * L.n + (double)L.ngroups * L.B * L.B + (double)L.ngroups * L.B +
                2.0 * L.n);
}

int sb2st_group_nwg(const Sb2stLayout& L) {
  if (L.nsweep <= 0) return 0;
  // A sweep trails its predecessor by two tasks, so the wavefront that
  // finished sweep s (about (n - s) / B tasks) is needed again for sweep
  // s + TW no earlier than 2 TW tasks later: TW >= n / 2B wavefronts keep the
  // pipeline from waiting for a free wavefront.
  int need = ceil_div(ceil_div(L.n, 2 * L.B), WPB) + 1;
  if (need > SB2ST_MAX_WG) need = SB2ST_MAX_WG;
  const int all = ceil_div(L.nsweep, WPB);
  return need < all ? need : all;
}

hipError_t sb2st_group_launch(const Sb2stTask* d_tasks, const int* d_wg_task, int total_wg,
                              double flops, double bytes, hipStream_t s) {
  if (total_wg <= 0) return hipSuccess;
  if (total_wg > SB2ST_MAX_WG) return hipErrorInvalidValue;
  void* args[] = {(void*)&d_tasks, (void*)&d_wg_task};
  const void* fn = (const void*)sb2st_group_kernel<32>;
  int cap = 0;
  HSDM_TRY(resident_wg(fn, cap));
  if (total_wg > cap) return hipErrorInvalidValue;
  return coop_launch("sb2st_group_kernel<32>", flops, bytes, true, true, fn, dim3(total_wg),
                     dim3(64 * WPB), args, s);
}

hipError_t sb2st_run(const Sb2stLayout& L, double* AB, int ldab, double* d, double* e, double* V2,
                     double* tau2, const long* d_goff, int* progress, DevStatusWord* st,
                     hipStream_t s) {
  const int n = L.n;
  if (L.B != 32 || ldab != 2 * L.B) return hipErrorInvalidValue;
  if (L.nsweep > 0) {
    HSDM_LAUNCH(fill_dbl_kernel, dim3(4096), dim3(256), 0, s, V2, L.v2_doubles);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(fill_dbl_kernel, dim3(1024), dim3(256), 0, s, tau2, L.ngroups * L.B);
    HSDM_TRY(hipGetLastError());
    HSDM_LAUNCH(fill_int_kernel, dim3(ceil_div(L.nsweep, 256)), dim3(256), 0, s, progress,
                       (long)L.nsweep, 0);
    HSDM_TRY(hipGetLastError());
    int nsweep = L.nsweep;
    const void* fn = (const void*)sb2st_kernel<32>;
    int nwg = ceil_div(nsweep, WPB), cap = 0;
    HSDM_TRY(resident_wg(fn, cap));
    if (nwg > cap) nwg = cap;
    // (sweep s and s-1 share a workgroup iff s is not the first sweep of its
    // wavefront group; TW = nwg * WPB keeps that true for every round)
    void* args[] = {(void*)&n, (void*)&nsweep, (void*)&AB, (void*)&ldab, (void*)&V2,
                    (void*)&tau2, (void*)&d_goff, (void*)&progress, (void*)&st};
    HSDM_TRY(coop_launch("sb2st_kernel<32>", sb2st_algo_flops(L), sb2st_algo_bytes(L), true, true,
                         fn, dim3(nwg), dim3(64 * WPB), args, s));
  }
  HSDM_LAUNCH(extract_tridiag_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, AB, ldab,
                     d, e);
  return hipGetLastError();
}
