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
// One wavefront runs one sweep at a time (64 lanes; the B x B blocks live in
// LDS); workgroups of 8 wavefronts are launched cooperatively so that every
// wavefront is resident.  Consecutive sweeps run on consecutive wavefronts:
// inside a workgroup the hand-off is a progress counter in LDS, between
// workgroups a counter in global memory with agent-scope release/acquire;
// every wait is bounded and reports through the status word if it runs out.
// Sums over the rows of a block use DPP and LDS swizzle moves.
//
// Storage: lower band storage AB[(r-c) + c*ldab], ldab = 2B (offsets up to
// 2B-1 hold the bulge).  Each reflector H_{s,t} (v, tau; v[0] = 1) is stored
// for the back-transformation in group (s / B, t): a 2B x B block whose
// column s % B holds v at rows (s % B) .. (s % B) + len - 1.
#include "hsdm_internal.h"
#include "hsdm_phases.h"

namespace {

constexpr int WPB = 8;  // wavefronts per workgroup
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

template <int PAT>
HSDM_DEV double swz(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)u, PAT);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(unsigned)(u >> 32), PAT);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

HSDM_DEV double first_lane(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum of a value that is zero outside lanes 0..31, returned in every lane:
// lane xor 1 and xor 2 (quad permutations), rotations by 4 and 8 inside rows
// of 16, lane xor 16 (swizzle, bit-mask mode), then lane 0's total.
HSDM_DEV double wsum(double v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x124>(v);
  v += dpp<0x128>(v);
  v += swz<0x401F>(v);
  return first_lane(v);
}

// v + (the value of lane ^ 32): v_permlane32_swap of each 32-bit half gives
// the lower lanes' value and the upper lanes' value in every lane.
HSDM_DEV double hsum(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
  const auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double a = __builtin_bit_cast(double, ((unsigned long long)(unsigned)ph[0] << 32) | (unsigned)pl[0]);
  const double b = __builtin_bit_cast(double, ((unsigned long long)(unsigned)ph[1] << 32) | (unsigned)pl[1]);
  return a + b;
}

// Sweep s waits for sweep s-1.  Consecutive sweeps run on the wavefronts of
// one workgroup except across workgroup boundaries, so the hand-off uses
// workgroup scope (no cache maintenance: the wavefronts share the CU's
// caches) when both sweeps are in the same workgroup, agent scope otherwise.
HSDM_DEV void wait_ge(int* p, int target, bool agent, DevStatusWord* st) {
  // poll with relaxed loads; one acquire fence once the counter is reached
  if ((threadIdx.x & 63) == 0) {
    long spins = 0;
    for (;;) {
      const int v = agent ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                          : __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (v >= target) break;
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
  if (agent)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  else
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  wave_sync();
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

HSDM_DEV void publish_lds(int* p, int v) {
  wave_sync();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

HSDM_DEV void publish(int* p, int v, bool agent) {
  wave_sync();
  if ((threadIdx.x & 63) == 0) {
    if (agent)
      __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    else
      __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

template <int B>
__global__ __launch_bounds__(64 * WPB) void sb2st_kernel(int n, int nsweep, double* AB, int ldab,
                                                         double* V2, double* tau2,
                                                         const long* goff, int* progress,
                                                         DevStatusWord* st) {
  static_assert(2 * B == 64, "one lane per row of a 2B-row group column");
  __shared__ double Dl_all[WPB][B][B + 1];
  __shared__ double Bl_all[WPB][B][B + 1];
  __shared__ double vc_all[WPB][B], vn_all[WPB][B], wv_all[WPB][B];
  __shared__ int lprog[WPB];
  const int lane = threadIdx.x & 63, wv_id = threadIdx.x >> 6;
  if (lane == 0) lprog[wv_id] = -1;
  __syncthreads();
  double(*Dl)[B + 1] = Dl_all[wv_id];
  double(*Bl)[B + 1] = Bl_all[wv_id];
  double* vc = vc_all[wv_id];
  double* vn = vn_all[wv_id];
  double* wk = wv_all[wv_id];
  const int gw = blockIdx.x * WPB + wv_id, TW = gridDim.x * WPB;
  const int li = lane % B, hf = lane / B;  // row index and column half (B/2 columns each)
  constexpr int HB = B / 2;

  for (int s = gw, round = 0; s < nsweep; s += TW, round++) {
    const int ntask = (n - 1 - s + B - 1) / B;
    // sweep s-1 runs on wavefront gw-1: in the same workgroup (LDS counter)
    // unless this is the workgroup's first wavefront (global counter)
    const bool first_wave = (wv_id == 0);
    const bool last_wave = (wv_id == WPB - 1);
    const int kbase = round * KROUND;
    double tau = 0.0;
    const long g0 = goff[s / B];
    for (int t = 0; t < ntask; t++) {
      if (s > 0) {
        if (first_wave)
          wait_ge(progress + s - 1, t + 2, true, st);
        else
          wait_lds(&lprog[wv_id - 1], kbase + t + 2, st);
      }
      const int rs = s + 1 + t * B;
      const int len = min(B, n - rs);
      const int rs2 = rs + B;
      const int len2 = (rs2 < n) ? min(B, n - rs2) : 0;
      // load the diagonal block (symmetrized) and the block below: all loads
      // are issued before the first use through one base pointer per lane
      // (the band storage has B + 1 spare columns, so every address is inside
      // it; invalid values are masked)
      {
        double dv[HB], bv[HB];
        const double* col = AB + (long)(rs + hf * HB) * ldab + (li - hf * HB);
#pragma unroll
        for (int q = 0; q < HB; q++) {
          dv[q] = col[(long)q * (ldab - 1)];
          bv[q] = col[(long)q * (ldab - 1) + B];
        }
#pragma unroll
        for (int q = 0; q < HB; q++) {
          const int j = hf * HB + q;
          dv[q] = (li < len && j < len && li >= j) ? dv[q] : 0.0;
          bv[q] = (li < len2 && j < len) ? bv[q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < HB; q++) {
          const int j = hf * HB + q;
          Bl[li][j] = bv[q];
          if (li >= j) {
            Dl[li][j] = dv[q];
            Dl[j][li] = dv[q];
          }
        }
      }
      if (t == 0) {
        // reflector from column s, rows s+1 .. s+len
        const double x = (lane < len) ? AB[(1 + lane) + (long)s * ldab] : 0.0;
        const double alpha = first_lane(x);
        const double sig = wsum((lane >= 1 && lane < len) ? x * x : 0.0);
        double beta = alpha, scal = 0.0;
        tau = 0.0;
        if (sig > 0.0) {
          const double nrm = sqrt(alpha * alpha + sig);
          beta = (alpha >= 0.0) ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
        if (lane < B) vc[lane] = (lane == 0) ? 1.0 : ((lane < len) ? x * scal : 0.0);
        if (lane < len) AB[(1 + lane) + (long)s * ldab] = (lane == 0) ? beta : 0.0;
      } else {
        if (lane < B) vc[lane] = vn[lane];
      }
      wave_sync();
      // store H_{s,t} for the back-transformation
      {
        const int k = s % B;
        const long gi = g0 + t;
        double* col = V2 + (gi * B + k) * (long)(2 * B);
        const int r = lane - k;
        col[lane] = (r >= 0 && r < len) ? vc[r] : 0.0;
        if (lane == 0) tau2[gi * B + k] = tau;
      }
      // two-sided update of the diagonal block: y = tau D v, w = y - (tau/2)(v.y) v
      {
        double p = 0.0;
        for (int q = 0; q < HB; q++) {
          const int j = hf * HB + q;
          p += Dl[li][j] * vc[j];
        }
        const double y = tau * hsum(p);
        const double vy = wsum(hf == 0 ? vc[li] * y : 0.0);
        const double w = y - 0.5 * tau * vy * vc[li];
        if (hf == 0) wk[li] = w;
        wave_sync();
        const double vi = vc[li];
        for (int q = 0; q < HB; q++) {
          const int j = hf * HB + q;
          Dl[li][j] -= vi * wk[j] + w * vc[j];
        }
      }
      double tau_n = 0.0;
      if (len2 > 0) {
        // right application to the block below: Bk <- Bk (I - tau v v^T)
        double p = 0.0;
        for (int q = 0; q < HB; q++) {
          const int j = hf * HB + q;
          p += Bl[li][j] * vc[j];
        }
        const double z = tau * hsum(p);
        for (int q = 0; q < HB; q++) {
          const int j = hf * HB + q;
          Bl[li][j] -= z * vc[j];
        }
        wave_sync();
        // next reflector from the first column of the block
        const double x = (lane < len2) ? Bl[lane][0] : 0.0;
        const double alpha = first_lane(x);
        const double sig = wsum((lane >= 1 && lane < len2) ? x * x : 0.0);
        double beta = alpha, scal = 0.0;
        if (sig > 0.0) {
          const double nrm = sqrt(alpha * alpha + sig);
          beta = (alpha >= 0.0) ? -nrm : nrm;
          tau_n = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
        if (lane < B) vn[lane] = (lane == 0) ? 1.0 : ((lane < len2) ? x * scal : 0.0);
        wave_sync();
        // left application to columns 1..: w_j = tau_n sum_r vn_r Bk[r][j]
        // (lane owns column li, rows of its half)
        double pc = 0.0;
        for (int q = 0; q < HB; q++) {
          const int r = hf * HB + q;
          pc += vn[r] * Bl[r][li];
        }
        const double wj = tau_n * hsum(pc);
        wave_sync();
        if (li >= 1) {
          for (int q = 0; q < HB; q++) {
            const int r = hf * HB + q;
            Bl[r][li] -= vn[r] * wj;
          }
        } else {
          for (int q = 0; q < HB; q++) {
            const int r = hf * HB + q;
            Bl[r][0] = (r == 0) ? beta : 0.0;
          }
        }
        wave_sync();
      }
      // write back: all LDS values first, then the stores (column j of the
      // band: rows li of both blocks are consecutive)
      {
        double dv[HB], bv[HB];
#pragma unroll
        for (int q = 0; q < HB; q++) {
          const int j = hf * HB + q;
          dv[q] = Dl[li][j];
          bv[q] = Bl[li][j];
        }
        // element (rs + li, rs + j) of D sits at (li - j) + (rs + j) ldab
        double* col = AB + (long)(rs + hf * HB) * ldab + (li - hf * HB);
#pragma unroll
        for (int q = 0; q < HB; q++) {
          const int j = hf * HB + q;
          double* cj = col + (long)q * (ldab - 1);
          if (li < len && j < len && li >= j) cj[0] = dv[q];
          if (li < len2 && j < len) cj[B] = bv[q];
        }
      }
      tau = tau_n;
      publish_lds(&lprog[wv_id], kbase + t + 1);
      if (last_wave) publish(progress + s, t + 1, true);
    }
    publish_lds(&lprog[wv_id], kbase + KDONE);
    if (last_wave) publish(progress + s, DONE, true);
  }
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

hipError_t sb2st_run(const Sb2stLayout& L, double* AB, int ldab, double* d, double* e, double* V2,
                     double* tau2, const long* d_goff, int* progress, DevStatusWord* st,
                     hipStream_t s) {
  const int n = L.n;
  if (L.B != 32 || ldab != 2 * L.B) return hipErrorInvalidValue;
  if (L.nsweep > 0) {
    hipLaunchKernelGGL(fill_dbl_kernel, dim3(4096), dim3(256), 0, s, V2, L.v2_doubles);
    HSDM_TRY(hipGetLastError());
    hipLaunchKernelGGL(fill_dbl_kernel, dim3(1024), dim3(256), 0, s, tau2, L.ngroups * L.B);
    HSDM_TRY(hipGetLastError());
    hipLaunchKernelGGL(fill_int_kernel, dim3(ceil_div(L.nsweep, 256)), dim3(256), 0, s, progress,
                       (long)L.nsweep, 0);
    HSDM_TRY(hipGetLastError());
    int nsweep = L.nsweep;
    int nwg = ceil_div(nsweep, WPB);
    if (nwg > 256) nwg = 256;
    // (sweep s and s-1 share a workgroup iff s is not the first sweep of its
    // wavefront group; TW = nwg * WPB keeps that true for every round)
    void* args[] = {(void*)&n, (void*)&nsweep, (void*)&AB, (void*)&ldab, (void*)&V2,
                    (void*)&tau2, (void*)&d_goff, (void*)&progress, (void*)&st};
    // algorithmic: about 6 B n^2 flops; each task reads and writes the lower
    // half of its diagonal block and the block below (24 B^2 bytes), n^2 / 2B tasks
    const double nn = (double)n * n;
    kt_begin("sb2st_kernel<32>", 6.0 * L.B * nn, 12.0 * L.B * nn, 0, s);
    HSDM_TRY(hipLaunchCooperativeKernel((const void*)sb2st_kernel<32>, dim3(nwg), dim3(64 * WPB),
                                        args, 0, s));
    kt_end(s);
  }
  hipLaunchKernelGGL(extract_tridiag_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, AB, ldab,
                     d, e);
  return hipGetLastError();
}
