// C ABI of libhsdm: handle, argument checks, workspace, and the phase driver
// of the dense H, S -> eigenpairs / density-matrix path.  Every phase is a
// kernel of this library; the host only enqueues work on the caller's stream
// and reads back the status word and the scalar results at the end.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hsdm.h"
#include "hsdm_internal.h"
#include "hsdm_phases.h"
#include "hsdm_util.h"

namespace {

constexpr int BAND = 32;
constexpr int NPHASE = 10;
constexpr int NLANE = 8;  // worker streams of the multi-task solves (at most)
const char* kPhaseNames[NPHASE] = {"cholesky_inverse",     "standard_form",
                                   "full_to_band",         "band_to_tridiagonal",
                                   "divide_conquer",       "backtransform_stage2",
                                   "backtransform_stage1", "refinement",
                                   "backtransform_cholesky", "density"};
constexpr int MAX_REFINE_STEPS = 8;
// the refinement stops after a step whose largest correction is at most this
// (the vectors' error is then of the order of its square)
constexpr double REFINE_TOL = 1e-6;

__global__ void reset_status_kernel(DevStatusWord* st, OccOut* occ) {
  if (threadIdx.x == 0) {
    st->code = 0;
    st->detail = 0;
    occ->mu = 0.0;
    occ->band_energy = 0.0;
    occ->sum_f = 0.0;
    occ->m = 0;
    occ->iters = 0;
  }
}

__global__ void set_int_kernel(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void eye_kernel(double* Z, long ldz, int n) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * n) return;
  const int i = (int)(idx % n), j = (int)(idx / n);
  Z[i + (long)j * ldz] = (i == j) ? 1.0 : 0.0;
}

__global__ void copy_vec_kernel(const double* a, double* b, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// Everything a recorded density-matrix solve depends on: the caller's
// buffers and settings, whether the factor of S was cached (the recorded
// work differs), and the workspace it was recorded against.
struct GraphKey {
  int n, ldh, lds, ldd, lde;
  const double *H, *S;
  double *D, *E;
  double ne, kT, fmax, fcut, deg_tol;
  bool cached;
  void* ws;
  bool operator==(const GraphKey& o) const {
    return n == o.n && ldh == o.ldh && lds == o.lds && ldd == o.ldd && lde == o.lde &&
           H == o.H && S == o.S && D == o.D && E == o.E && ne == o.ne && kT == o.kT &&
           fmax == o.fmax && fcut == o.fcut && deg_tol == o.deg_tol && cached == o.cached &&
           ws == o.ws;
  }
};

struct SolveGraph {
  GraphKey key;
  hipGraphExec_t exec;
  long last_use;
};
constexpr size_t MAX_GRAPHS = 4;

struct Pinned {
  DevStatusWord st;
  OccOut occ;
  double rec[2 * MAX_REFINE_STEPS];  // refinement record of the last refined solve
};

}  // namespace

struct hsdm_ctx {
  int device = 0;
  double fmax = 2.0;
  double fcut_rel = 1e-16;
  double deg_tol = -1.0;
  bool timing = false;
  bool ktiming = false;
  bool kt_every = false;  // every launch timed: no worker streams
  int nlane = 4;          // worker streams used by multi-task solves
  long n_states = 0;      // eigenvectors formed by the eigenpair solves (0: all)
  bool concurrent = false;  // solves may overlap other handles' on the device
  int precision = 0;        // 0: FP64 throughout; 1: the refined form (real pencils)
  int refine_steps = 8;     // most refinement steps of the refined form
  // workspace of the refined form (grown on demand)
  void* rws_raw = nullptr;
  size_t rws_cap = 0;
  float *A32 = nullptr, *V32 = nullptr, *Z32 = nullptr, *bt1f = nullptr;
  void *f32_scr = nullptr, *ref_scr = nullptr;
  double* rrec = nullptr;
  int last_refine = 0;      // steps of the last solve (0: FP64 form)
  // solves recorded as HIP graphs (HSDM_KEY_GRAPH): replayed on the handle's
  // own stream when a call repeats a recorded one's buffers and settings
  bool graph_mode = false;
  std::vector<SolveGraph> graphs;
  long graph_clock = 0;
  hipStream_t gstream = nullptr;
  hipEvent_t gev[2] = {};
  int last_graph = 0;       // 0: eager, 1: recorded and run, 2: replayed
  int last_mref = 0;        // columns refined by the last solve
  KTimer* kt = nullptr;
  std::string err;
  int detail = 0;
  // workspace
  int ws_n = 0;
  bool borrowed = false;  // workspace carved from the library's static scratch (never freed)
  void* ws_raw = nullptr;  // the one device allocation holding the workspace (not borrowed)
  size_t ws_cap = 0;       // its size in bytes
  std::vector<long> goff_host;  // group offsets of the carved size (uploaded with it)
  double* ws = nullptr;
  int* iws = nullptr;
  long* d_goff = nullptr;
  DevStatusWord* st = nullptr;
  OccOut* occ = nullptr;
  Pinned* host = nullptr;
  StedcPlan* plan = nullptr;
  Sb2stLayout lay{};
  // carved pointers
  double *Lbuf, *Linv, *Abuf, *Vst, *Zbuf, *Cbuf, *T1, *tau1, *AB, *sy_scr, *dvec, *evec, *lam,
      *fvec, *V2, *tau2, *F2, *dc_scr, *bt1_scr, *colsum, *hnorm;
  int *dc_iscr, *progress;
  // per-task contexts of the multi-task solves (workspace and S factor each),
  // picked by S identity, then least recently used
  std::vector<hsdm_ctx*> subs;
  long last_use = 0;
  long use_clock = 0;
  std::vector<OccTask> h_tasks;
  OccTask* d_tasks = nullptr;
  int d_tasks_cap = 0;
  std::vector<int> tag_m;  // occupied-state count of each task of the last batch
  Sy2sbGroupHost sy_host;   // panel QR schedule of the last multi-task reduction
  std::vector<Sy2sbArgs> sy_args;
  void* d_qr = nullptr;
  size_t d_qr_bytes = 0;
  std::vector<Bt2Task> h_bt2;  // stage-2 back-transform descriptors of the last multi-task solve
  std::vector<int> h_bt2map;
  void* d_bt2 = nullptr;
  size_t d_bt2_bytes = 0;
  std::vector<Sb2stTask> h_sb;
  std::vector<int> h_wgmap;
  void* d_sb = nullptr;  // Sb2stTask[nprob] then the workgroup -> task map
  size_t d_sb_bytes = 0;
  hsdm_ctx* na = nullptr;        // context of the allocation-free solve (static scratch)
  // embedded Hermitian pencils: R(H), R(S), D_R, E_R (2n x 2n each)
  int cws_n = 0;
  double* cws = nullptr;
  double *HR, *SR, *DR, *ER;
  // worker streams of the multi-task solves (created on first use, default
  // priority): the tasks' independent phases run spread over them, ordered
  // after the caller's stream by lane_ev[NLANE] and joined back through
  // lane_ev[k]; lane k > 0 embeds Hermitian pencils in lane_buf[k]'s buffers
  // (lane 0 in the handle's own)
  hipStream_t lane_s[NLANE] = {};
  hipEvent_t lane_ev[NLANE + 1] = {};
  hsdm_ctx* lane_buf[NLANE] = {};
  // cached factor of S, keyed by the content of the caller's S (size, real
  // or complex, 64-bit hash of the lower triangle), never by its address: a
  // buffer freed and reused for another S must not find the old factor
  int s_n = 0;
  bool s_cplx = false;
  unsigned long long s_hash = 0;
  bool s_valid = false;
  // content hashes of the S matrices of a call (device, then pinned host)
  unsigned long long* d_hash = nullptr;
  unsigned long long* h_hash = nullptr;
  int hash_cap = 0;
  // phase timing
  hipEvent_t ev[NPHASE + 1] = {};
  double phase_ms[NPHASE] = {};
  bool phase_done[NPHASE] = {};
  // algorithmic work of the last single solve's phases (timing on)
  double phase_flops[NPHASE] = {};
  int last_kind = 0;          // 1: density-matrix solve, 2: eigenpair solve
  int last_n = 0, last_ns = 0;
  bool last_factored = false;
};

namespace {

int fail_dev(hsdm_ctx* h, hipError_t e, const char* where) {
  h->err = std::string(where) + ": " + hipGetErrorString(e);
  return HSDM_DEVICE_ERROR;
}

#define DEV_TRY(h, x)                                \
  do {                                               \
    hipError_t _e = (x);                             \
    if (_e != hipSuccess) return fail_dev(h, _e, #x); \
  } while (0)

void free_cws(hsdm_ctx* h) {
  if (h->cws) (void)hipFree(h->cws);
  h->cws = nullptr;
  h->cws_n = 0;
}

// Workspace of the Hermitian route for complex sizes up to n (the real
// workspace is that of size 2n); a size-n' problem uses it with leading
// dimension 2n'.  Zero-filled once, by a kernel on stream s (the caller's
// stream, ahead of the work that uses the buffers: a null-stream memset is
// not ordered with non-blocking streams), so the upper triangles of R(H)
// and R(S), which nothing writes, hold zeros.
int ensure_cws(hsdm_ctx* h, int n, hipStream_t s) {
  if (h->cws_n >= n && h->cws) return HSDM_OK;
  free_cws(h);
  const size_t q = (size_t)4 * n * n;
  hipError_t e = hipMalloc(&h->cws, 4 * q * sizeof(double));
  if (e != hipSuccess) {
    h->cws = nullptr;
    return fail_dev(h, e, "workspace allocation");
  }
  // 4 buffers of (2n)^2 doubles: a 2n x 8n column-major block
  e = dev_fill(h->cws, 2L * n, 2 * n, 8 * n, 0.0, s);
  if (e != hipSuccess) {
    free_cws(h);
    return fail_dev(h, e, "workspace clear");
  }
  h->HR = h->cws;
  h->SR = h->cws + q;
  h->DR = h->cws + 2 * q;
  h->ER = h->cws + 3 * q;
  h->cws_n = n;
  return HSDM_OK;
}

void free_lanes(hsdm_ctx* h) {
  if (h->lane_s[0]) (void)hipDeviceSynchronize();
  for (int k = 0; k < NLANE; k++) {
    if (h->lane_s[k]) (void)hipStreamDestroy(h->lane_s[k]);
    h->lane_s[k] = nullptr;
    if (h->lane_buf[k]) {
      free_cws(h->lane_buf[k]);
      delete h->lane_buf[k];
      h->lane_buf[k] = nullptr;
    }
  }
  for (int k = 0; k <= NLANE; k++) {
    if (h->lane_ev[k]) (void)hipEventDestroy(h->lane_ev[k]);
    h->lane_ev[k] = nullptr;
  }
}

int ensure_lanes(hsdm_ctx* h) {
  if (h->lane_s[0]) return HSDM_OK;
  for (int k = 0; k < NLANE; k++) {
    hipError_t e = hipStreamCreateWithFlags(&h->lane_s[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->lane_ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
      free_lanes(h);
      return fail_dev(h, e, "worker stream creation");
    }
  }
  hipError_t e = hipEventCreateWithFlags(&h->lane_ev[NLANE], hipEventDisableTiming);
  if (e != hipSuccess) {
    free_lanes(h);
    return fail_dev(h, e, "worker stream creation");
  }
  return HSDM_OK;
}

// Embedding buffers of lane k for complex sizes up to n.
hsdm_ctx* lane_cws(hsdm_ctx* h, int k) { return k == 0 ? h : h->lane_buf[k]; }
int ensure_lane_cws(hsdm_ctx* h, int k, int n, hipStream_t s) {
  if (n <= 0) return HSDM_OK;
  if (k > 0 && !h->lane_buf[k]) h->lane_buf[k] = new hsdm_ctx();
  hsdm_ctx* b = lane_cws(h, k);
  const int r = ensure_cws(b, n, s);
  if (r && b != h) h->err = b->err;
  return r;
}

// The lanes start after the work queued so far on s; s continues after all
// the work queued on the lanes.
hipError_t lanes_fork(hsdm_ctx* h, hipStream_t s, int nl) {
  HSDM_TRY(hipEventRecord(h->lane_ev[NLANE], s));
  for (int k = 0; k < nl; k++) HSDM_TRY(hipStreamWaitEvent(h->lane_s[k], h->lane_ev[NLANE], 0));
  return hipSuccess;
}
hipError_t lanes_join(hsdm_ctx* h, hipStream_t s, int nl) {
  for (int k = 0; k < nl; k++) {
    HSDM_TRY(hipEventRecord(h->lane_ev[k], h->lane_s[k]));
    HSDM_TRY(hipStreamWaitEvent(s, h->lane_ev[k], 0));
  }
  return hipSuccess;
}

// Forks the first nl lanes off s (nl = 0: none) and joins them back; a
// return between fork and join (an error) still waits for the lanes' work
// before the call returns.
struct Lanes {
  hsdm_ctx* h;
  hipStream_t s;
  int nl;
  bool forked = false;
  hipError_t fork() {
    if (nl == 0) return hipSuccess;
    forked = true;
    return lanes_fork(h, s, nl);
  }
  hipError_t join() {
    if (!forked) return hipSuccess;
    forked = false;
    return lanes_join(h, s, nl);
  }
  ~Lanes() {
    if (!forked) return;
    for (int k = 0; k < nl; k++) (void)hipStreamSynchronize(h->lane_s[k]);
    (void)hipStreamSynchronize(s);
  }
};

void free_graphs(hsdm_ctx* h) {
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
}

void free_ws(hsdm_ctx* h) {
  free_graphs(h);  // recorded against this workspace
  if (!h->borrowed && h->ws_raw) (void)hipFree(h->ws_raw);
  h->ws_raw = nullptr;
  h->ws_cap = 0;
  stedc_plan_destroy(h->plan);
  h->ws = nullptr;
  h->iws = nullptr;
  h->d_goff = nullptr;
  h->plan = nullptr;
  h->ws_n = 0;
  h->s_valid = false;
}

struct WsLayout {
  size_t oL, oLi, oA, oV, oZ, oC, oT1, otau1, oAB, osy, od, oe, olam, of, oV2, otau2, oF2, odc,
      obt1, ocs, ohn, total, ints;
};

WsLayout ws_layout(int n) {
  WsLayout w{};
  const size_t nn = (size_t)n * n;
  const Sb2stLayout L = sb2st_layout(n, BAND);
  const int npanel = (n > BAND) ? ceil_div(n - 1, BAND) : 0;
  size_t off = 0;
  auto take = [&](size_t cnt) {
    size_t o = off;
    off += (cnt + 31) & ~(size_t)31;  // 256-byte aligned pieces
    return o;
  };
  w.oL = take(nn); w.oLi = take(nn); w.oA = take(nn); w.oV = take(nn); w.oZ = take(nn);
  w.oC = take(nn);
  w.oT1 = take((size_t)(npanel + 1) * BAND * BAND); w.otau1 = take(n + 1);
  w.oAB = take((size_t)2 * BAND * (n + BAND + 1)); w.osy = take(sy2sb_scratch_doubles(n, BAND));
  w.od = take(n); w.oe = take(n); w.olam = take(n); w.of = take(n);
  w.oV2 = take(L.v2_doubles + 1); w.otau2 = take((size_t)L.ngroups * BAND + 1);
  w.oF2 = take(bt2_pack_doubles(L) + 1);
  w.odc = take(stedc_scratch_doubles(n)); w.obt1 = take(bt1_scratch_doubles(n, BAND, n));
  w.ocs = take(n); w.ohn = take(1);
  w.total = off;
  w.ints = stedc_iscratch_ints(n) + (size_t)n + 128;
  return w;
}


// Points the workspace pointers of h into w (WsLayout(n).total doubles) and
// iws (WsLayout(n).ints ints).
void carve_ws(hsdm_ctx* h, int n, double* w, int* iws) {
  const WsLayout wl = ws_layout(n);
  h->ws = w;
  h->iws = iws;
  h->Lbuf = w + wl.oL; h->Linv = w + wl.oLi; h->Abuf = w + wl.oA; h->Vst = w + wl.oV;
  h->Zbuf = w + wl.oZ; h->Cbuf = w + wl.oC; h->T1 = w + wl.oT1; h->tau1 = w + wl.otau1;
  h->AB = w + wl.oAB; h->sy_scr = w + wl.osy; h->dvec = w + wl.od; h->evec = w + wl.oe;
  h->lam = w + wl.olam; h->fvec = w + wl.of; h->V2 = w + wl.oV2; h->tau2 = w + wl.otau2;
  h->F2 = w + wl.oF2; h->dc_scr = w + wl.odc; h->bt1_scr = w + wl.obt1; h->colsum = w + wl.ocs;
  h->hnorm = w + wl.ohn;
  h->dc_iscr = iws;
  h->progress = iws + stedc_iscratch_ints(n);
  h->lay = sb2st_layout(n, BAND);
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device bytes of the workspace of a solve of size n, as one block: the
// workspace doubles and ints, the group offsets of the stage-2 reflectors
// and the divide-and-conquer plan's tables.
size_t ws_block_bytes(int n) {
  const WsLayout wl = ws_layout(n);
  const Sb2stLayout L = sb2st_layout(n, BAND);
  return up256(wl.total * sizeof(double)) + up256(wl.ints * sizeof(int)) +
         up256(sizeof(long) * (L.nblk + 1)) + stedc_plan_device_bytes(n);
}

// Device bytes of the workspace of a real solve of size n.
double ws_bytes(int n) { return (double)ws_block_bytes(n); }

// Points every workspace pointer of h into the block at base (ws_block_bytes(n)
// bytes) for size n and queues the upload of its tables on stream s.  The
// factor of S that the block held for another size is gone.
int carve_block(hsdm_ctx* h, int n, void* base, hipStream_t s) {
  stedc_plan_destroy(h->plan);
  h->plan = nullptr;
  h->ws_n = 0;
  h->s_valid = false;
  const WsLayout wl = ws_layout(n);
  const Sb2stLayout L = sb2st_layout(n, BAND);
  char* b = (char*)base;
  double* w = (double*)b;
  b += up256(wl.total * sizeof(double));
  int* iw = (int*)b;
  b += up256(wl.ints * sizeof(int));
  carve_ws(h, n, w, iw);
  h->d_goff = (long*)b;
  b += up256(sizeof(long) * (L.nblk + 1));
  h->plan = stedc_plan_create_in(n, b);
  if (!h->plan) {
    h->err = "divide-and-conquer plan creation failed";
    return HSDM_DEVICE_ERROR;
  }
  h->goff_host.assign(L.nblk + 1, 0);
  sb2st_group_offsets(L, h->goff_host.data());
  DEV_TRY(h, hipMemcpyAsync(h->d_goff, h->goff_host.data(), sizeof(long) * h->goff_host.size(),
                            hipMemcpyHostToDevice, s));
  DEV_TRY(h, stedc_plan_upload(h->plan, s));
  h->ws_n = n;
  return HSDM_OK;
}

// The workspace for size n.  The block only grows: a smaller size is carved
// from the block in hand, so that solves of varying sizes do not free and
// allocate device memory (a free waits for the whole device, other streams
// included).
int ensure_ws(hsdm_ctx* h, int n, hipStream_t s) {
  if (h->ws_n == n && h->ws) return HSDM_OK;
  const size_t need = ws_block_bytes(n);
  if (!h->ws_raw || h->ws_cap < need) {
    free_ws(h);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) return fail_dev(h, e, "workspace allocation");
    h->ws_raw = p;
    h->ws_cap = need;
  }
  return carve_block(h, n, h->ws_raw, s);
}

// The refined form's workspace: A, the reflectors and the eigenvectors in
// FP32 (n x n each), the FP32 reduction's and back-transform's scratch, the
// refinement's blocks and its record.
int ensure_rws(hsdm_ctx* h, int n, hipStream_t s) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t nn = (size_t)n * n;
  const size_t b32 = al(nn * sizeof(float));
  const size_t bf = al(sy2sb_f32_scratch_bytes(n, BAND));
  const size_t bb = al(bt1_f32_scratch_floats(n, BAND, n) * sizeof(float));
  const size_t br = al(refine_scratch_bytes(n, n));
  const size_t need = 3 * b32 + bf + bb + br + al(2 * MAX_REFINE_STEPS * sizeof(double));
  if (h->rws_cap < need) {
    if (h->rws_raw) {
      DEV_TRY(h, hipStreamSynchronize(s));
      (void)hipFree(h->rws_raw);
      h->rws_raw = nullptr;
      h->rws_cap = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) return fail_dev(h, e, "refined-form workspace allocation");
    h->rws_raw = p;
    h->rws_cap = need;
  }
  char* p = (char*)h->rws_raw;
  h->A32 = (float*)p; p += b32;
  h->V32 = (float*)p; p += b32;
  h->Z32 = (float*)p; p += b32;
  h->f32_scr = p; p += bf;
  h->bt1f = (float*)p; p += bb;
  h->ref_scr = p; p += br;
  h->rrec = (double*)p;
  return HSDM_OK;
}

// ---- the allocation-free density-matrix solve --------------------------------
// Its workspace lives in `scratch`, a static device array of the library:
// every GPU the library runs on holds one copy until the process ends, and
// every call of hsdm_solve_dm_real_noalloc on that GPU uses it (calls that
// overlap on one GPU race).  Host code never names the array except in
// hipGetSymbolAddress: the device address of each GPU's copy is taken once
// per device at hsdm_init and kept in scratch_dev[].
constexpr size_t NOALLOC_BYTES = (size_t)56 << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex scratch_mu;
void* scratch_dev[64] = {};

// With `device` current: the address of its copy of the scratch array.
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[device]) {
    void* p = nullptr;
    HSDM_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return hipErrorInvalidSymbol;
    scratch_dev[device] = p;
  }
  *out = scratch_dev[device];
  return hipSuccess;
}


void mark(hsdm_ctx* h, int phase, hipStream_t s) {
  if (h->timing) {
    (void)hipEventRecord(h->ev[phase], s);
    if (phase > 0) h->phase_done[phase - 1] = true;
  }
}

// Algorithmic flops of each phase of the last single solve (the counts of the
// method, not of this implementation's extra work): Cholesky n^3/3 (when S
// was factored), standard form n^3, full -> band 4n^3/3, band ->
// tridiagonal 6 B n^2, divide and conquer the merge products at their sizes
// after deflation (read back from the device), the back-transforms 2 n^2 m,
// 2 n^2 m and n^2 m, D and E n^2 m each, with m the vectors formed.
void phase_work(hsdm_ctx* h) {
  for (int p = 0; p < NPHASE; p++) h->phase_flops[p] = 0.0;
  if (!h->last_kind || h->last_n <= 0) return;
  const double n = h->last_n;
  const double m = h->last_kind == 1 ? (double)h->host->occ.m : (double)h->last_ns;
  h->phase_flops[0] = h->last_factored ? n * n * n / 3.0 : 0.0;
  h->phase_flops[1] = n * n * n;
  h->phase_flops[2] = 4.0 * n * n * n / 3.0;
  h->phase_flops[3] = sb2st_algo_flops(h->lay);
  h->phase_flops[4] = h->plan ? stedc_last_flops(h->plan) : 0.0;
  // the refined form transforms every vector back and refines mref of them:
  // per step 6 n^2 mref (A X, X^T X, X^T A X) and 2 n^2 mref (X E), the
  // first step 2 n^2 (n - mref) more for the Rayleigh quotients of the rest
  const double mb = h->last_refine ? n : m;
  h->phase_flops[5] = 2.0 * n * n * mb;
  h->phase_flops[6] = 2.0 * n * n * mb;
  if (h->last_refine) {
    const double mr = h->last_mref;
    h->phase_flops[7] = h->last_refine * 8.0 * n * n * mr + 2.0 * n * n * (n - mr);
  }
  h->phase_flops[8] = n * n * m;
  h->phase_flops[9] = h->last_kind == 1 ? 2.0 * n * n * m : 0.0;
}

int finish(hsdm_ctx* h, hipStream_t s) {
  DEV_TRY(h, hipMemcpyAsync(&h->host->st, h->st, sizeof(DevStatusWord), hipMemcpyDeviceToHost, s));
  DEV_TRY(h, hipMemcpyAsync(&h->host->occ, h->occ, sizeof(OccOut), hipMemcpyDeviceToHost, s));
  DEV_TRY(h, hipStreamSynchronize(s));
  if (h->ktiming) {
    kt_collect(h->kt, h->host->occ.m, h->tag_m.empty() ? nullptr : h->tag_m.data(),
               (int)h->tag_m.size());
    kt_activate(nullptr);
  }
  if (h->timing) {
    for (int p = 0; p < NPHASE; p++) {
      h->phase_ms[p] = 0.0;
      if (!h->phase_done[p]) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, h->ev[p], h->ev[p + 1]) == hipSuccess) h->phase_ms[p] = ms;
    }
    phase_work(h);
  }
  const int code = h->host->st.code;
  h->detail = h->host->st.detail;
  switch (code) {
    case DS_OK: return HSDM_OK;
    case DS_NOT_SPD:
      h->s_valid = false;
      h->err = "S is not positive definite (column " + std::to_string(h->detail) + ")";
      return HSDM_NOT_SPD;
    case DS_NO_CONVERGE:
      h->err = std::string("eigenvalue iteration did not converge (") +
               (h->detail == 1 ? "leaf QL" : "secular equation") + ")";
      return HSDM_NO_CONVERGE;
    case DS_MU_FAIL: h->err = "chemical potential search failed"; return HSDM_MU_FAIL;
    default:
      h->s_valid = false;
      h->err = "inter-workgroup wait timed out";
      return HSDM_SYNC_TIMEOUT;
  }
}

bool bad_ld(int ld, int n) { return ld < (n > 1 ? n : 1); }

// Identity of the caller's S for the factor cache: its size, whether it is
// complex, and the content hash of its lower triangle (the part the solvers
// read).
struct SKey {
  int n;
  bool cplx;
  unsigned long long hash;
};

bool s_cached(const hsdm_ctx* h, const SKey& k) {
  return h->s_valid && h->s_n == k.n && h->s_cplx == k.cplx && h->s_hash == k.hash;
}

// Content hashes of cnt matrices S[p] (n[p] x n[p], leading dimension
// lds[p], complex if cplx[p]) into out[p], with one synchronization of s.
int s_hashes(hsdm_ctx* h, int cnt, const void* const* S, const int* n, const int* lds,
             const int* cplx, unsigned long long* out, hipStream_t s) {
  if (cnt <= 0) return HSDM_OK;
  if (h->hash_cap < cnt) {
    if (h->d_hash) (void)hipFree(h->d_hash);
    if (h->h_hash) (void)hipHostFree(h->h_hash);
    h->d_hash = nullptr;
    h->h_hash = nullptr;
    h->hash_cap = 0;
    DEV_TRY(h, hipMalloc(&h->d_hash, sizeof(unsigned long long) * cnt));
    DEV_TRY(h, hipHostMalloc((void**)&h->h_hash, sizeof(unsigned long long) * cnt,
                             hipHostMallocDefault));
    h->hash_cap = cnt;
  }
  DEV_TRY(h, dev_hash_clear(h->d_hash, cnt, s));
  for (int p = 0; p < cnt; p++)
    DEV_TRY(h, dev_hash_lower(S[p], lds[p], n[p], cplx[p], h->d_hash + p, s));
  DEV_TRY(h, hipMemcpyAsync(h->h_hash, h->d_hash, sizeof(unsigned long long) * cnt,
                            hipMemcpyDeviceToHost, s));
  DEV_TRY(h, hipStreamSynchronize(s));
  for (int p = 0; p < cnt; p++) out[p] = h->h_hash[p];
  return HSDM_OK;
}

// The cache key of one S.
int s_key(hsdm_ctx* h, const void* S, int n, int lds, bool cplx, SKey& key, hipStream_t s) {
  const int c = cplx ? 1 : 0;
  key = SKey{n, cplx, 0ull};
  return s_hashes(h, 1, &S, &n, &lds, &c, &key.hash, s);
}

// Cholesky + inverse of the real symmetric S (n x n, lower) into the cache,
// skipped when the cache holds the factor of the S that `key` names.
int factor_s(hsdm_ctx* h, int n, const double* S, int lds, const SKey& key, hipStream_t s) {
  h->last_factored = false;
  if (s_cached(h, key)) return HSDM_OK;
  h->last_factored = true;
  DEV_TRY(h, dev_copy(S, lds, h->Lbuf, n, n, n, s));
  DEV_TRY(h, dev_fill(h->Linv, n, n, n, 0.0, s));
  DEV_TRY(h, chol_inv(n, h->Lbuf, n, h->Linv, n, h->Abuf, n, h->st, s));
  h->s_n = key.n;
  h->s_cplx = key.cplx;
  h->s_hash = key.hash;
  h->s_valid = true;
  return HSDM_OK;
}

// A = Linv H Linv^T (lower).  Zbuf and Vst serve as scratch.
int standard_form(hsdm_ctx* h, int n, const double* H, int ldh, const double* Li, int ldli,
                  double* A, int lda, hipStream_t s) {
  DEV_TRY(h, dev_sym_full(H, ldh, h->Zbuf, n, n, s));
  GemmArgs g{};
  g.m = n; g.n = n; g.k = n; g.A = Li; g.lda = ldli; g.B = h->Zbuf; g.ldb = n; g.C = h->Vst;
  g.ldc = n; g.alpha = 1.0; g.beta = 0.0; g.flags = GF_KA_LOWER;
  DEV_TRY(h, gemm_launch(g, s));
  g = GemmArgs{};
  g.m = n; g.n = n; g.k = n; g.A = h->Vst; g.lda = n; g.B = Li; g.ldb = ldli; g.C = A; g.ldc = lda;
  g.alpha = 1.0; g.beta = 0.0; g.ta = 0; g.tb = 1;
  g.flags = GF_KB_UPPER | GF_C_LOWER_TILES | GF_C_LOWER_ONLY;
  DEV_TRY(h, gemm_launch(g, s));
  return HSDM_OK;
}

// Two-stage reduction of h->Abuf (lower) to (dvec, evec); reflectors kept.
int reduce(hsdm_ctx* h, int n, hipStream_t s, int phase_band) {
  DEV_TRY(h, bt1_zero_fill(n, BAND, h->Vst, n, s));
  DEV_TRY(h, sy2sb_run(n, BAND, h->Abuf, n, h->Vst, n, h->tau1, h->T1, h->AB, 2 * BAND, h->sy_scr,
                       h->st, s));
  mark(h, phase_band, s);
  DEV_TRY(h, sb2st_run(h->lay, h->AB, 2 * BAND, h->dvec, h->evec, h->V2, h->tau2, h->d_goff,
                       h->progress, h->st, s));
  return HSDM_OK;
}

// The refined form's two-stage reduction: h->Abuf (lower, FP64) stays as it
// is; its FP32 copy is reduced with FP32 trailing updates, the band chased in
// FP64.
int reduce_f32(hsdm_ctx* h, int n, hipStream_t s, int phase_band) {
  DEV_TRY(h, dev_convert(h->Abuf, n, h->A32, n, n, n, s));
  DEV_TRY(h, bt1_zero_fill(n, BAND, h->Vst, n, s));
  DEV_TRY(h, sy2sb_f32_run(n, BAND, h->A32, n, h->Vst, n, h->V32, n, h->tau1, h->T1, h->AB,
                           2 * BAND, h->f32_scr, h->st, s));
  mark(h, phase_band, s);
  DEV_TRY(h, sb2st_run(h->lay, h->AB, 2 * BAND, h->dvec, h->evec, h->V2, h->tau2, h->d_goff,
                       h->progress, h->st, s));
  return HSDM_OK;
}

// The refined form after the tridiagonal eigensolve (every vector, FP64):
// both back-transforms of all n columns (stage 2 in FP64, stage 1 in FP32),
// then `steps` refinement steps of the first mref columns against the FP64
// standard-form matrix.  lam holds the eigenvalues on entry and the
// refined ones (Rayleigh quotients) on exit; the vectors are in h->Zbuf.
int refine_vectors(hsdm_ctx* h, int n, int mref, double* lam, hipStream_t s) {
  DEV_TRY(h, bt2_prepare(h->lay, h->V2, h->tau2, h->F2, s));
  DEV_TRY(h, bt2_apply(h->lay, h->F2, h->d_goff, h->Zbuf, n, n, nullptr, h->progress, h->st, s));
  mark(h, 6, s);
  DEV_TRY(h, dev_convert(h->Zbuf, n, h->Z32, n, n, n, s));
  DEV_TRY(h, bt1_apply_f32(n, BAND, h->Vst, n, h->V32, n, h->T1, h->Z32, n, n, nullptr,
                           h->bt1_scr, h->bt1f, s));
  DEV_TRY(h, dev_convert(h->Z32, n, h->Zbuf, n, n, n, s));
  mark(h, 7, s);
  int done = 0;
  DEV_TRY(h, refine_run(n, mref, h->Abuf, n, h->Zbuf, n, h->Z32, n, h->Cbuf, n, lam,
                        h->refine_steps, REFINE_TOL, h->ref_scr, h->rrec, h->host->rec, &done,
                        s));
  h->last_refine = done;
  h->last_mref = mref;
  return HSDM_OK;
}

struct OccHook {
  hsdm_ctx* h;
  int n;
  double ne, kT;
};

hipError_t occ_hook(void* ctx, const double* lam, hipStream_t s) {
  OccHook* o = (OccHook*)ctx;
  hsdm_ctx* h = o->h;
  const bool auto_tol = h->deg_tol < 0.0;
  return occupations_launch(o->n, lam, h->fmax, o->ne, o->kT, auto_tol ? 0.0 : h->deg_tol,
                            auto_tol ? h->hnorm : nullptr, h->fcut_rel * h->fmax, h->fvec, h->occ,
                            h->st, s);
}

// Kernel timing for the duration of one solve (finish() folds the records).
struct KtScope {
  explicit KtScope(hsdm_ctx* h) {
    if (h->ktiming) {
      kt_reset(h->kt);
      kt_activate(h->kt);
    }
    coop_set_shared(h->concurrent);
  }
  ~KtScope() {
    kt_activate(nullptr);
    kt_set_tag(-1);
    coop_set_shared(false);
  }
};

// The cooperative-launch mode of a handle for the duration of one call.
struct CoopScope {
  explicit CoopScope(const hsdm_ctx* h) { coop_set_shared(h->concurrent); }
  ~CoopScope() { coop_set_shared(false); }
};

}  // namespace

// probe.hip: the device's sustained FP64 matrix-core rate (iters rounds per
// wavefront) and HBM copy bandwidth (two buffers of `bytes`), each timed on
// its second launch: out[0] = TFLOP/s or GB/s (bytes read + written), out[1]
// = ms, out[2] = flops or bytes.
hipError_t probe_fp64_mfma(int iters, double* out, hipStream_t s);
hipError_t probe_hbm_copy(double bytes, double* out, hipStream_t s);

extern "C" {

int hsdm_version(void) { return 100; }

int hsdm_init(hsdm_handle* out, int device) {
  if (!out) return -1;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return HSDM_DEVICE_ERROR;
  if (device < 0 || device >= ndev) return -2;
  hsdm_ctx* h = new hsdm_ctx();
  h->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete h;
    return HSDM_DEVICE_ERROR;
  }
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(DevStatusWord) + sizeof(OccOut) + 64) != hipSuccess) {
    delete h;
    return HSDM_DEVICE_ERROR;
  }
  h->st = (DevStatusWord*)p;
  h->occ = (OccOut*)((char*)p + 32);
  if (hipHostMalloc((void**)&h->host, sizeof(Pinned), hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(p);
    delete h;
    return HSDM_DEVICE_ERROR;
  }
  for (int i = 0; i <= NPHASE; i++) (void)hipEventCreate(&h->ev[i]);
  h->kt = kt_create();
  void* scr = nullptr;
  if (scratch_address(device, &scr) != hipSuccess) {
    hsdm_finalize(h);
    return HSDM_DEVICE_ERROR;
  }
  *out = h;
  return HSDM_OK;
}

int hsdm_finalize(hsdm_handle h) {
  if (!h) return -1;
  (void)hipSetDevice(h->device);
  for (hsdm_ctx* c : h->subs) hsdm_finalize(c);
  h->subs.clear();
  if (h->na) {
    free_ws(h->na);  // the plan object only: the workspace is the static scratch
    delete h->na;
    h->na = nullptr;
  }
  free_lanes(h);
  if (h->d_tasks) (void)hipFree(h->d_tasks);
  if (h->d_sb) (void)hipFree(h->d_sb);
  if (h->d_qr) (void)hipFree(h->d_qr);
  if (h->d_bt2) (void)hipFree(h->d_bt2);
  free_ws(h);
  free_cws(h);
  if (h->rws_raw) (void)hipFree(h->rws_raw);
  if (h->gstream) (void)hipStreamDestroy(h->gstream);
  for (auto& e : h->gev)
    if (e) (void)hipEventDestroy(e);
  if (h->st) (void)hipFree(h->st);
  if (h->host) (void)hipHostFree(h->host);
  if (h->d_hash) (void)hipFree(h->d_hash);
  if (h->h_hash) (void)hipHostFree(h->h_hash);
  for (int i = 0; i <= NPHASE; i++)
    if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
  kt_destroy(h->kt);
  delete h;
  return HSDM_OK;
}

int hsdm_reinit(hsdm_handle h) {
  if (!h) return -1;
  for (hsdm_ctx* c : h->subs) hsdm_reinit(c);
  h->s_valid = false;
  return HSDM_OK;
}

int hsdm_set_real(hsdm_handle h, int key, double v) {
  if (!h) return -1;
  switch (key) {
    case HSDM_KEY_FMAX:
      if (!(v > 0.0) || !std::isfinite(v)) return -3;
      h->fmax = v;
      return HSDM_OK;
    case HSDM_KEY_FCUT:
      if (!(v >= 0.0) || !(v < 1.0)) return -3;
      h->fcut_rel = v;
      return HSDM_OK;
    case HSDM_KEY_DEG_TOL:
      if (std::isnan(v)) return -3;
      h->deg_tol = v;
      return HSDM_OK;
    default: return -2;
  }
}

int hsdm_set_int(hsdm_handle h, int key, long v) {
  if (!h) return -1;
  if (key == HSDM_KEY_TIMING) {
    if (v < 0 || v > 3) return -3;
    h->timing = (v != 0);
    h->ktiming = (v >= 2);
    h->kt_every = (v == 2);
    kt_set_whole_only(h->kt, v == 3);
    return HSDM_OK;
  }
  if (key == HSDM_KEY_STREAMS) {
    if (v < 1 || v > NLANE) return -3;
    h->nlane = (int)v;
    return HSDM_OK;
  }
  if (key == HSDM_KEY_N_STATES) {
    if (v < 0) return -3;
    h->n_states = v;
    return HSDM_OK;
  }
  if (key == HSDM_KEY_CONCURRENT) {
    if (v != 0 && v != 1) return -3;
    h->concurrent = (v == 1);
    return HSDM_OK;
  }
  if (key == HSDM_KEY_PRECISION) {
    if (v != 0 && v != 1) return -3;
    h->precision = (int)v;
    return HSDM_OK;
  }
  if (key == HSDM_KEY_GRAPH) {
    if (v != 0 && v != 1) return -3;
    h->graph_mode = (v == 1);
    if (!h->graph_mode) free_graphs(h);
    return HSDM_OK;
  }
  if (key == HSDM_KEY_AUTOTUNE) {
    if (v != 0 && v != 1) return -3;
    gemm_tuning(v == 1);
    return HSDM_OK;
  }
  if (key == HSDM_KEY_REFINE_STEPS) {
    if (v < 1 || v > MAX_REFINE_STEPS) return -3;
    h->refine_steps = (int)v;
    return HSDM_OK;
  }
  return -2;
}

const char* hsdm_status_string(int status) {
  switch (status) {
    case HSDM_OK: return "ok";
    case HSDM_NOT_SPD: return "S is not positive definite";
    case HSDM_NO_CONVERGE: return "eigenvalue iteration did not converge";
    case HSDM_MU_FAIL: return "chemical potential search failed";
    case HSDM_DEVICE_ERROR: return "device error";
    case HSDM_SYNC_TIMEOUT: return "inter-workgroup wait timed out";
    default: return status < 0 ? "invalid argument" : "unknown status";
  }
}

const char* hsdm_last_error(hsdm_handle h) { return h ? h->err.c_str() : "null handle"; }
int hsdm_status_detail(hsdm_handle h) { return h ? h->detail : 0; }

int hsdm_phase_times(hsdm_handle h, double* times, int cap) {
  if (!h || !times) return 0;
  int k = cap < NPHASE ? cap : NPHASE;
  for (int i = 0; i < k; i++) times[i] = h->phase_ms[i];
  return k;
}

int hsdm_last_graph(hsdm_handle h) { return h ? h->last_graph : -1; }

int hsdm_tune_entries(void) { return gemm_tune_count(); }

int hsdm_tune_clear(void) {
  gemm_tune_clear();
  return HSDM_OK;
}

int hsdm_tune_save(const char* path) {
  if (!path) return -1;
  return gemm_tune_save(path) ? HSDM_OK : HSDM_DEVICE_ERROR;
}

int hsdm_tune_load(const char* path) {
  if (!path) return -1;
  const int r = gemm_tune_load(path);
  return r < 0 ? (r == -1 ? -2 : -3) : r;
}

int hsdm_refine_history(hsdm_handle h, double* out, int cap) {
  if (!h) return -1;
  if (cap < 0 || (cap > 0 && !out)) return -3;
  const int k = std::min(cap / 2, h->last_refine);
  for (int i = 0; i < 2 * k; i++) out[i] = h->host->rec[i];
  return h->last_refine;
}

const char* hsdm_phase_name(int i) { return (i >= 0 && i < NPHASE) ? kPhaseNames[i] : ""; }

int hsdm_phase_flops(hsdm_handle h, double* flops, int cap) {
  if (!h || !flops) return 0;
  int k = cap < NPHASE ? cap : NPHASE;
  for (int i = 0; i < k; i++) flops[i] = h->phase_flops[i];
  return k;
}

int hsdm_kernel_count(hsdm_handle h) { return h ? kt_count(h->kt) : 0; }

int hsdm_timing_kernel(hsdm_handle h, const char* name) {
  if (!h) return -1;
  kt_set_only(h->kt, name);
  return HSDM_OK;
}

const char* hsdm_kernel_stat(hsdm_handle h, int i, double* out) {
  if (!h) return nullptr;
  return kt_stat(h->kt, i, out);
}

int hsdm_dgemm(hsdm_handle h, char transa, char transb, int m, int n, int k, double alpha,
               const double* A, int lda, const double* B, int ldb, double beta, double* C,
               int ldc, void* stream) {
  if (!h) return -1;
  const int ta = (transa == 'T' || transa == 't') ? 1 : ((transa == 'N' || transa == 'n') ? 0 : -1);
  const int tb = (transb == 'T' || transb == 't') ? 1 : ((transb == 'N' || transb == 'n') ? 0 : -1);
  if (ta < 0) return -2;
  if (tb < 0) return -3;
  if (m < 0) return -4;
  if (n < 0) return -5;
  if (k < 0) return -6;
  if (m > 0 && k > 0 && !A) return -8;
  if (lda < (ta ? (k > 1 ? k : 1) : (m > 1 ? m : 1))) return -9;
  if (n > 0 && k > 0 && !B) return -10;
  if (ldb < (tb ? (n > 1 ? n : 1) : (k > 1 ? k : 1))) return -11;
  if (m > 0 && n > 0 && !C) return -13;
  if (ldc < (m > 1 ? m : 1)) return -14;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  GemmArgs g{};
  g.m = m; g.n = n; g.k = k; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta; g.ta = ta; g.tb = tb;
  DEV_TRY(h, gemm_launch(g, s));
  DEV_TRY(h, hipStreamSynchronize(s));
  return HSDM_OK;
}

int hsdm_probe(hsdm_handle h, int which, double size, double* out, void* stream) {
  if (!h) return -1;
  if (which != 0 && which != 1) return -2;
  if (!(size >= (which == 0 ? 1.0 : 16.0)) || size > (which == 0 ? 1e7 : 64e9)) return -3;
  if (!out) return -4;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  if (which == 0)
    DEV_TRY(h, probe_fp64_mfma((int)size, out, s));
  else
    DEV_TRY(h, probe_hbm_copy(size, out, s));
  return HSDM_OK;
}

int hsdm_cholesky_inverse(hsdm_handle h, int n, const double* S, int lds, double* L, int ldl,
                          double* Linv, int ldli, void* stream) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!S) return -3;
  if (bad_ld(lds, n)) return -4;
  if (!L) return -5;
  if (bad_ld(ldl, n)) return -6;
  if (!Linv) return -7;
  if (bad_ld(ldli, n)) return -8;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  int r = ensure_ws(h, n, s);
  if (r) return r;
  HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, s, h->st, h->occ);
  DEV_TRY(h, hipGetLastError());
  DEV_TRY(h, dev_copy(S, lds, L, ldl, n, n, s));
  DEV_TRY(h, dev_fill(Linv, ldli, n, n, 0.0, s));
  DEV_TRY(h, chol_inv(n, L, ldl, Linv, ldli, h->Abuf, n, h->st, s));
  return finish(h, s);
}

int hsdm_standard_form(hsdm_handle h, int n, const double* H, int ldh, const double* Linv,
                       int ldli, double* A, int lda, void* stream) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!H) return -3;
  if (bad_ld(ldh, n)) return -4;
  if (!Linv) return -5;
  if (bad_ld(ldli, n)) return -6;
  if (!A) return -7;
  if (bad_ld(lda, n)) return -8;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  int r = ensure_ws(h, n, s);
  if (r) return r;
  HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, s, h->st, h->occ);
  DEV_TRY(h, hipGetLastError());
  r = standard_form(h, n, H, ldh, Linv, ldli, A, lda, s);
  if (r) return r;
  return finish(h, s);
}

int hsdm_tridiagonalize(hsdm_handle h, int n, const double* A, int lda, double* d, double* e,
                        double* Q, int ldq, void* stream) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!A) return -3;
  if (bad_ld(lda, n)) return -4;
  if (!d) return -5;
  if (n > 1 && !e) return -6;
  if (Q && bad_ld(ldq, n)) return -8;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  int r = ensure_ws(h, n, s);
  if (r) return r;
  HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, s, h->st, h->occ);
  DEV_TRY(h, hipGetLastError());
  DEV_TRY(h, dev_copy(A, lda, h->Abuf, n, n, n, s));
  CoopScope cs(h);
  r = reduce(h, n, s, 0);
  if (r) return r;
  HSDM_LAUNCH(copy_vec_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, h->dvec, d, n);
  DEV_TRY(h, hipGetLastError());
  if (n > 1) {
    HSDM_LAUNCH(copy_vec_kernel, dim3(ceil_div(n - 1, 256)), dim3(256), 0, s, h->evec, e,
                       n - 1);
    DEV_TRY(h, hipGetLastError());
  }
  if (Q) {
    const long tot = (long)n * n;
    HSDM_LAUNCH(eye_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Q,
                       (long)ldq, n);
    DEV_TRY(h, hipGetLastError());
    DEV_TRY(h, bt2_prepare(h->lay, h->V2, h->tau2, h->F2, s));
    DEV_TRY(h, bt2_apply(h->lay, h->F2, h->d_goff, Q, ldq, n, nullptr, h->progress, h->st, s));
    DEV_TRY(h, bt1_apply(n, BAND, h->Vst, n, h->T1, Q, ldq, n, nullptr, h->bt1_scr, s));
  }
  return finish(h, s);
}

int hsdm_tridiag_eigh(hsdm_handle h, int n, const double* d, const double* e, double* w, double* Z,
                      int ldz, void* stream) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!d) return -3;
  if (n > 1 && !e) return -4;
  if (!w) return -5;
  if (!Z) return -6;
  if (bad_ld(ldz, n)) return -7;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  int r = ensure_ws(h, n, s);
  if (r) return r;
  HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, s, h->st, h->occ);
  DEV_TRY(h, hipGetLastError());
  DEV_TRY(h, stedc_run(h->plan, d, e, w, Z, ldz, h->dc_scr, h->dc_iscr, nullptr, nullptr, nullptr,
                       h->st, s));
  return finish(h, s);
}

int hsdm_occupations(hsdm_handle h, int n, const double* eval, double ne, double kT,
                     double deg_tol, double* f, double* mu, double* band_energy, int* n_occ,
                     void* stream) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!eval) return -3;
  if (!(ne >= 0.0) || ne > h->fmax * n) return -4;
  if (!(kT >= 0.0) || !std::isfinite(kT)) return -5;
  if (!(deg_tol >= 0.0)) return -6;
  if (!f) return -7;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, s, h->st, h->occ);
  DEV_TRY(h, hipGetLastError());
  DEV_TRY(h, occupations_launch(n, eval, h->fmax, ne, kT, deg_tol, nullptr, h->fcut_rel * h->fmax,
                                f, h->occ, h->st, s));
  int r = finish(h, s);
  if (mu) *mu = h->host->occ.mu;
  if (band_energy) *band_energy = h->host->occ.band_energy;
  if (n_occ) *n_occ = h->host->occ.m;
  return r;
}

int hsdm_density(hsdm_handle h, int n, int m, const double* C, int ldc, const double* f,
                 const double* eval, double* D, int ldd, double* E, int lde, void* stream) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (m < 0 || m > n) return -3;
  if (m > 0 && !C) return -4;
  if (bad_ld(ldc, n)) return -5;
  if (m > 0 && !f) return -6;
  if (m > 0 && E && !eval) return -7;
  if (!D) return -8;
  if (bad_ld(ldd, n)) return -9;
  if (E && bad_ld(lde, n)) return -11;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, s, h->st, h->occ);
  DEV_TRY(h, hipGetLastError());
  DEV_TRY(h, density_launch(n, m, C, ldc, f, eval, D, ldd, E, lde, nullptr, s));
  return finish(h, s);
}

// Density-matrix solve of the real pencil (H, S) of size n into D, E (both
// triangles) and h->lam (eigenvalues), with the S factor cached under `key`.
// The caller has checked the arguments and sized the workspace; the status
// words are read by finish().
static int dm_core(hsdm_ctx* h, int n, const double* H, int ldh, const double* S, int lds,
                   const SKey& key, double ne, double kT, double* D, int ldd, double* E, int lde,
                   hipStream_t s) {
  int r;
  for (int p = 0; p < NPHASE; p++) h->phase_done[p] = false;
  h->last_kind = 1;
  h->last_n = n;
  h->last_refine = 0;
  const bool refined = h->precision == 1;
  if (refined && (r = ensure_rws(h, n, s))) return r;
  HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, s, h->st, h->occ);
  DEV_TRY(h, hipGetLastError());
  mark(h, 0, s);
  if ((r = factor_s(h, n, S, lds, key, s))) return r;
  mark(h, 1, s);
  if (h->deg_tol < 0.0) DEV_TRY(h, dev_norm1_sym(H, ldh, n, h->colsum, h->hnorm, s));
  if ((r = standard_form(h, n, H, ldh, h->Linv, n, h->Abuf, n, s))) return r;
  mark(h, 2, s);
  if ((r = refined ? reduce_f32(h, n, s, 3) : reduce(h, n, s, 3))) return r;
  mark(h, 4, s);
  OccHook hook{h, n, ne, kT};
  const int* m_dev = &h->occ->m;
  if (refined) {
    // every vector: the refinement corrects the wanted ones with all others
    DEV_TRY(h, stedc_run(h->plan, h->dvec, h->evec, h->lam, h->Zbuf, n, h->dc_scr, h->dc_iscr,
                         nullptr, nullptr, nullptr, h->st, s));
    DEV_TRY(h, occ_hook(&hook, h->lam, s));
    mark(h, 5, s);
    // the wanted count at the unrefined eigenvalues, with a margin for the
    // states the refinement moves across the occupation cut
    DEV_TRY(h, hipMemcpyAsync(&h->host->occ, h->occ, sizeof(OccOut), hipMemcpyDeviceToHost, s));
    DEV_TRY(h, hipStreamSynchronize(s));
    const int m0 = h->host->occ.m;
    const int mref = std::min(n, m0 + std::max(32, m0 / 32));
    if ((r = refine_vectors(h, n, mref, h->lam, s))) return r;
    DEV_TRY(h, occ_hook(&hook, h->lam, s));
  } else {
    DEV_TRY(h, stedc_run(h->plan, h->dvec, h->evec, h->lam, h->Zbuf, n, h->dc_scr, h->dc_iscr,
                         m_dev, occ_hook, &hook, h->st, s));
    mark(h, 5, s);
    DEV_TRY(h, bt2_prepare(h->lay, h->V2, h->tau2, h->F2, s));
    DEV_TRY(h, bt2_apply(h->lay, h->F2, h->d_goff, h->Zbuf, n, n, m_dev, h->progress, h->st, s));
    mark(h, 6, s);
    DEV_TRY(h, bt1_apply(n, BAND, h->Vst, n, h->T1, h->Zbuf, n, n, m_dev, h->bt1_scr, s));
    mark(h, 7, s);
  }
  mark(h, 8, s);
  GemmArgs g{};
  g.m = n; g.n = n; g.k = n; g.A = h->Linv; g.lda = n; g.B = h->Zbuf; g.ldb = n; g.C = h->Cbuf;
  g.ldc = n; g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0; g.flags = GF_KA_UPPER;
  g.ndev = m_dev;
  DEV_TRY(h, gemm_launch(g, s));
  mark(h, 9, s);
  DEV_TRY(h, density_launch(n, n, h->Cbuf, n, h->fvec, h->lam, D, ldd, E, lde, m_dev, s));
  mark(h, 10, s);
  return HSDM_OK;
}

// Eigenpairs of the real pencil (H, S) of size n: all eigenvalues into eval,
// the eigenvectors of the lowest ns into C (C^T S C = I); the S factor cached
// under `key`.  With ns < n the final divide-and-conquer merge forms only
// those ns vectors (a device count in the handle's occupation record, which
// this solve does not otherwise use) and the back-transforms take ns columns.
static int ev_core(hsdm_ctx* h, int n, const double* H, int ldh, const double* S, int lds,
                   const SKey& key, double* eval, double* C, int ldc, int ns, hipStream_t s,
                   bool refined = false) {
  int r;
  for (int p = 0; p < NPHASE; p++) h->phase_done[p] = false;
  h->last_kind = 2;
  h->last_n = n;
  h->last_ns = ns;
  h->last_refine = 0;
  if (refined && (r = ensure_rws(h, n, s))) return r;
  if (refined) {
    HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, s, h->st, h->occ);
    DEV_TRY(h, hipGetLastError());
    mark(h, 0, s);
    if ((r = factor_s(h, n, S, lds, key, s))) return r;
    mark(h, 1, s);
    if ((r = standard_form(h, n, H, ldh, h->Linv, n, h->Abuf, n, s))) return r;
    mark(h, 2, s);
    if ((r = reduce_f32(h, n, s, 3))) return r;
    mark(h, 4, s);
    DEV_TRY(h, stedc_run(h->plan, h->dvec, h->evec, eval, h->Zbuf, n, h->dc_scr, h->dc_iscr,
                         nullptr, nullptr, nullptr, h->st, s));
    mark(h, 5, s);
    if ((r = refine_vectors(h, n, ns, eval, s))) return r;
    mark(h, 8, s);
    GemmArgs g{};
    g.m = n; g.n = ns; g.k = n; g.A = h->Linv; g.lda = n; g.B = h->Zbuf; g.ldb = n; g.C = C;
    g.ldc = ldc; g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0; g.flags = GF_KA_UPPER;
    DEV_TRY(h, gemm_launch(g, s));
    mark(h, 9, s);
    mark(h, 10, s);
    return HSDM_OK;
  }
  HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, s, h->st, h->occ);
  DEV_TRY(h, hipGetLastError());
  const int* m_dev = nullptr;
  if (ns < n) {
    HSDM_LAUNCH(set_int_kernel, dim3(1), dim3(64), 0, s, &h->occ->m, ns);
    DEV_TRY(h, hipGetLastError());
    m_dev = &h->occ->m;
  }
  mark(h, 0, s);
  if ((r = factor_s(h, n, S, lds, key, s))) return r;
  mark(h, 1, s);
  if ((r = standard_form(h, n, H, ldh, h->Linv, n, h->Abuf, n, s))) return r;
  mark(h, 2, s);
  if ((r = reduce(h, n, s, 3))) return r;
  mark(h, 4, s);
  DEV_TRY(h, stedc_run(h->plan, h->dvec, h->evec, eval, h->Zbuf, n, h->dc_scr, h->dc_iscr,
                       m_dev, nullptr, nullptr, h->st, s));
  mark(h, 5, s);
  if (ns > 0) {
    DEV_TRY(h, bt2_prepare(h->lay, h->V2, h->tau2, h->F2, s));
    DEV_TRY(h, bt2_apply(h->lay, h->F2, h->d_goff, h->Zbuf, n, ns, nullptr, h->progress, h->st,
                         s));
  }
  mark(h, 6, s);
  if (ns > 0) DEV_TRY(h, bt1_apply(n, BAND, h->Vst, n, h->T1, h->Zbuf, n, ns, nullptr, h->bt1_scr, s));
  mark(h, 7, s);
  mark(h, 8, s);
  if (ns > 0) {
    GemmArgs g{};
    g.m = n; g.n = ns; g.k = n; g.A = h->Linv; g.lda = n; g.B = h->Zbuf; g.ldb = n; g.C = C;
    g.ldc = ldc; g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0; g.flags = GF_KA_UPPER;
    DEV_TRY(h, gemm_launch(g, s));
  }
  mark(h, 9, s);
  mark(h, 10, s);
  return HSDM_OK;
}

static int check_hs(hsdm_handle h, int n, const double* H, int ldh, const double* S, int lds) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!H) return -3;
  if (bad_ld(ldh, n)) return -4;
  if (!S) return -5;
  if (bad_ld(lds, n)) return -6;
  return 0;
}

int hsdm_solve_ev_real(hsdm_handle h, int n, const double* H, int ldh, const double* S, int lds,
                       double* eval, double* C, int ldc, void* stream) {
  int a = check_hs(h, n, H, ldh, S, lds);
  if (a) return a;
  if (!eval) return -7;
  if (!C) return -8;
  if (bad_ld(ldc, n)) return -9;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  int r = ensure_ws(h, n, s);
  if (r) return r;
  SKey key;
  if ((r = s_key(h, S, n, lds, false, key, s))) return r;
  KtScope kts(h);
  const int ns = (h->n_states > 0 && h->n_states < n) ? (int)h->n_states : n;
  if ((r = ev_core(h, n, H, ldh, S, lds, key, eval, C, ldc, ns, s, h->precision == 1))) return r;
  return finish(h, s);
}

int hsdm_solve_ev_complex(hsdm_handle h, int n, const void* H, int ldh, const void* S, int lds,
                          double* eval, void* C, int ldc, void* stream) {
  if (!h) return -1;
  if (n < 1 || n > (1 << 29)) return -2;
  if (!H) return -3;
  if (bad_ld(ldh, n)) return -4;
  if (!S) return -5;
  if (bad_ld(lds, n)) return -6;
  if (!eval) return -7;
  if (!C) return -8;
  if (bad_ld(ldc, n)) return -9;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  const int n2 = 2 * n;
  int r = ensure_ws(h, n2, s);
  if (r) return r;
  if ((r = ensure_cws(h, n, s))) return r;
  SKey key;
  if ((r = s_key(h, S, n, lds, true, key, s))) return r;
  KtScope kts(h);
  if (!s_cached(h, key)) DEV_TRY(h, herm_embed(n, S, lds, h->SR, n2, s));
  DEV_TRY(h, herm_embed(n, H, ldh, h->HR, n2, s));
  // real eigenpairs of the embedded pencil (each eigenvalue twice) into lam,
  // DR; every real vector is formed (a degenerate cluster at the n_states
  // boundary needs all of its 2k candidates), the first ns pairs kept
  const int ns = (h->n_states > 0 && h->n_states < n) ? (int)h->n_states : n;
  if ((r = ev_core(h, n2, h->HR, n2, h->SR, n2, key, h->lam, h->DR, n2, n2, s))) return r;
  DEV_TRY(h, herm_pair_eval(n, h->lam, eval, s));
  DEV_TRY(h, herm_extract_pairs(n, ns, h->DR, n2, C, ldc, s));
  if ((r = finish(h, s))) return r;
  // A complex eigenvalue of multiplicity k has 2k real eigenvectors spanning
  // a k-dimensional complex space; one vector per real pair may then be
  // dependent.  For such clusters the complex basis is rebuilt from all 2k
  // candidates u_j = x_j + i y_j with their complex S-inner products
  // <u_i, u_j> = delta_ij - i M_ij, M = Q_c^T R(S) J Q_c.
  std::vector<double> lam2(n2);
  DEV_TRY(h, hipMemcpy(lam2.data(), h->lam, sizeof(double) * n2, hipMemcpyDeviceToHost));
  double scale = 1.0;
  for (double v : lam2) scale = std::max(scale, std::fabs(v));
  const double tol = 1e-10 * scale;
  bool sr_fresh = false;
  for (int l0 = 0; l0 < ns;) {
    int l1 = l0 + 1;
    while (l1 < n && 0.5 * (lam2[2 * l1] + lam2[2 * l1 + 1]) -
                         0.5 * (lam2[2 * l1 - 2] + lam2[2 * l1 - 1]) <= tol)
      l1++;
    const int k = l1 - l0, k2 = 2 * k;
    if (k > 1) {
      if (!sr_fresh) {
        // R(S) again: the buffer may hold another S when the factor was cached
        DEV_TRY(h, herm_embed(n, S, lds, h->SR, n2, s));
        sr_fresh = true;
      }
      const double* Qc = h->DR + (long)(2 * l0) * n2;
      double* JQ = h->HR;    // 2n x k2 (k2 <= 2n: each fits a 2n x 2n buffer)
      double* P = h->ER;     // 2n x k2
      double* M = h->Cbuf;   // k2 x k2 (free after the eigenvectors are formed)
      double* cf = h->Zbuf;  // k2 x k complex
      DEV_TRY(h, herm_jmul(n, k2, Qc, n2, JQ, n2, s));
      GemmArgs g{};
      g.m = n2; g.n = k2; g.k = n2; g.A = h->SR; g.lda = n2; g.B = JQ; g.ldb = n2; g.C = P;
      g.ldc = n2; g.alpha = 1.0; g.beta = 0.0; g.flags = GF_A_SYM_LOWER;
      DEV_TRY(h, gemm_launch(g, s));
      g = GemmArgs{};
      g.m = k2; g.n = k2; g.k = n2; g.A = Qc; g.lda = n2; g.B = P; g.ldb = n2; g.C = M;
      g.ldc = k2; g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0;
      DEV_TRY(h, gemm_launch(g, s));
      std::vector<double> Mh((size_t)k2 * k2);
      DEV_TRY(h, hipMemcpyAsync(Mh.data(), M, sizeof(double) * k2 * k2, hipMemcpyDeviceToHost, s));
      DEV_TRY(h, hipStreamSynchronize(s));
      // <u_i, u_j> = r_i^T R(S) r_j - i r_i^T R(S) J r_j (J r is the real form
      // of i u, and Re <u, i v> = -Im <u, v>), so the Gram matrix is G = I - i M.
      // Its pivoted Cholesky (rank k) picks k independent candidates u_piv;
      // W = U_piv L^{-H} is S-orthonormal.
      using cd = std::complex<double>;
      auto G = [&](int i, int j) { return cd(i == j ? 1.0 : 0.0, -Mh[i + (size_t)j * k2]); };
      std::vector<int> piv(k2);
      for (int j = 0; j < k2; j++) piv[j] = j;
      std::vector<double> d(k2, 1.0);
      std::vector<cd> L((size_t)k2 * k, 0.0);  // L[row j (candidate), col a]
      for (int a = 0; a < k; a++) {
        int best = a;
        for (int j = a + 1; j < k2; j++)
          if (d[piv[j]] > d[piv[best]]) best = j;
        std::swap(piv[a], piv[best]);
        const int pa = piv[a];
        if (!(d[pa] > 1e-3)) {
          h->err = "complex eigenvector basis of a degenerate cluster could not be formed";
          return HSDM_NO_CONVERGE;
        }
        const double lpp = std::sqrt(d[pa]);
        L[pa + (size_t)a * k2] = lpp;
        for (int j = a + 1; j < k2; j++) {
          const int pj = piv[j];
          cd v = G(pj, pa);
          for (int b = 0; b < a; b++) v -= L[pj + (size_t)b * k2] * std::conj(L[pa + (size_t)b * k2]);
          v /= lpp;
          L[pj + (size_t)a * k2] = v;
          d[pj] -= std::norm(v);
        }
      }
      // coefficients: column a of L11^{-H} placed at the selected candidates
      // (L11[a][b] = L[piv[a]][b], lower triangular); solve L11^H X = I
      std::vector<cd> X((size_t)k * k, 0.0);
      for (int c = 0; c < k; c++) {
        for (int r = k - 1; r >= 0; r--) {
          cd v = (r == c) ? cd(1.0) : cd(0.0);
          for (int q = r + 1; q < k; q++) v -= std::conj(L[piv[q] + (size_t)r * k2]) * X[q + (size_t)c * k];
          X[r + (size_t)c * k] = v / std::conj(L[piv[r] + (size_t)r * k2]);
        }
      }
      std::vector<cd> coef((size_t)k2 * k, 0.0);
      for (int c = 0; c < k; c++)
        for (int r = 0; r < k; r++) coef[piv[r] + (size_t)c * k2] = X[r + (size_t)c * k];
      DEV_TRY(h, hipMemcpyAsync(cf, coef.data(), sizeof(double) * 2 * k2 * k,
                                hipMemcpyHostToDevice, s));
      // columns past ns are not the caller's: the cluster's first ns - l0 only
      DEV_TRY(h, herm_combine(n, k2, std::min(k, ns - l0), Qc, n2, cf,
                              (char*)C + (size_t)l0 * ldc * 16, ldc, s));
      DEV_TRY(h, hipStreamSynchronize(s));
    }
    l0 = l1;
  }
  return HSDM_OK;
}

// The density-matrix solve as a HIP graph: the first call with a given key
// records dm_core's launches on the handle's stream (nothing runs while
// recording) and instantiates them; that call and every later one with the
// same key launch the graph on the handle's stream, ordered after the
// caller's stream by an event and joined back into it.  The host state that
// dm_core sets while recording (the cached factor's identity, the solve's
// kind and size) is set again for a replay.
static int dm_graph(hsdm_ctx* h, int n, const double* H, int ldh, const double* S, int lds,
                    const SKey& key, double ne, double kT, double* D, int ldd, double* E,
                    int lde, hipStream_t s) {
  if (!h->gstream) {
    DEV_TRY(h, hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
    for (auto& e : h->gev) DEV_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  const GraphKey gk{n, ldh, lds, ldd, E ? lde : 0, H, S, D, E, ne, kT, h->fmax,
                    h->fcut_rel, h->deg_tol, s_cached(h, key), h->ws_raw};
  SolveGraph* g = nullptr;
  for (auto& x : h->graphs)
    if (x.key == gk) g = &x;
  if (!g) {
    if (h->graphs.size() >= MAX_GRAPHS) {
      auto lru = std::min_element(h->graphs.begin(), h->graphs.end(),
                                  [](const SolveGraph& a, const SolveGraph& b) {
                                    return a.last_use < b.last_use;
                                  });
      (void)hipGraphExecDestroy(lru->exec);
      h->graphs.erase(lru);
    }
    DEV_TRY(h, hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
    const int r = dm_core(h, n, H, ldh, S, lds, key, ne, kT, D, ldd, E, lde, h->gstream);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->gstream, &graph);
    if (r) {
      if (graph) (void)hipGraphDestroy(graph);
      h->s_valid = false;  // the factor was never computed
      return r;
    }
    if (ec != hipSuccess) h->s_valid = false;
    DEV_TRY(h, ec);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) h->s_valid = false;
    DEV_TRY(h, ei);
    h->graphs.push_back(SolveGraph{gk, exec, 0});
    g = &h->graphs.back();
    h->last_graph = 1;
  } else {
    for (int p = 0; p < NPHASE; p++) h->phase_done[p] = false;
    h->last_kind = 1;
    h->last_n = n;
    h->last_refine = 0;
    h->last_factored = !gk.cached;
    if (!gk.cached) {
      h->s_n = key.n;
      h->s_cplx = key.cplx;
      h->s_hash = key.hash;
      h->s_valid = true;
    }
    h->last_graph = 2;
  }
  g->last_use = ++h->graph_clock;
  DEV_TRY(h, hipEventRecord(h->gev[0], s));
  DEV_TRY(h, hipStreamWaitEvent(h->gstream, h->gev[0], 0));
  DEV_TRY(h, hipGraphLaunch(g->exec, h->gstream));
  DEV_TRY(h, hipEventRecord(h->gev[1], h->gstream));
  DEV_TRY(h, hipStreamWaitEvent(s, h->gev[1], 0));
  return HSDM_OK;
}

int hsdm_solve_dm_real(hsdm_handle h, int n, const double* H, int ldh, const double* S, int lds,
                       double ne, double kT, double* D, int ldd, double* E, int lde, double* eval,
                       double* band_energy, double* mu, void* stream) {
  int a = check_hs(h, n, H, ldh, S, lds);
  if (a) return a;
  if (!(ne >= 0.0) || !std::isfinite(ne) || ne > h->fmax * n) return -7;
  if (!(kT >= 0.0) || !std::isfinite(kT)) return -8;
  if (!D) return -9;
  if (bad_ld(ldd, n)) return -10;
  if (E && bad_ld(lde, n)) return -12;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  int r = ensure_ws(h, n, s);
  if (r) return r;
  SKey key;
  if ((r = s_key(h, S, n, lds, false, key, s))) return r;
  h->last_graph = 0;
  if (h->graph_mode && !h->timing && !h->ktiming && !h->concurrent && h->precision == 0 &&
      !gemm_tuning_on()) {
    r = dm_graph(h, n, H, ldh, S, lds, key, ne, kT, D, ldd, E, lde, s);
  } else {
    KtScope kts(h);
    r = dm_core(h, n, H, ldh, S, lds, key, ne, kT, D, ldd, E, lde, s);
  }
  if (eval && r == HSDM_OK) {
    HSDM_LAUNCH(copy_vec_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, h->lam, eval, n);
    DEV_TRY(h, hipGetLastError());
  }
  if (r == HSDM_OK) r = finish(h, s);
  if (mu) *mu = h->host->occ.mu;
  if (band_energy) *band_energy = h->host->occ.band_energy;
  return r;
}

int hsdm_solve_dm_real_noalloc(hsdm_handle h, int n, const double* H, int ldh, const double* S,
                               int lds, double ne, double kT, double* D, int ldd, double* E,
                               int lde, double* eval, double* band_energy, double* mu,
                               void* stream) {
  int a = check_hs(h, n, H, ldh, S, lds);
  if (a) return a;
  if (!(ne >= 0.0) || !std::isfinite(ne) || ne > h->fmax * n) return -7;
  if (!(kT >= 0.0) || !std::isfinite(kT)) return -8;
  if (!D) return -9;
  if (bad_ld(ldd, n)) return -10;
  if (E && bad_ld(lde, n)) return -12;
  if (n > HSDM_NOALLOC_MAX_N) {
    h->err = "hsdm_solve_dm_real_noalloc: n = " + std::to_string(n) + " exceeds the maximum " +
             std::to_string(HSDM_NOALLOC_MAX_N) + " of the static scratch";
    return -2;
  }
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  void* scr = nullptr;
  DEV_TRY(h, scratch_address(h->device, &scr));  // taken at hsdm_init: no allocation here
  if (ws_block_bytes(n) > NOALLOC_BYTES) {
    h->err = "hsdm_solve_dm_real_noalloc: the static scratch is too small for n = " +
             std::to_string(n);
    return HSDM_DEVICE_ERROR;
  }
  // the context of the allocation-free solves: host object only, its device
  // pointers carved from the scratch (its tables uploaded again on every
  // call: another call on this GPU may have used the scratch since); status
  // words and pinned results are the handle's own
  if (!h->na) {
    h->na = new hsdm_ctx();
    h->na->borrowed = true;
    h->na->device = h->device;
  }
  hsdm_ctx* c = h->na;
  c->err.clear();
  {
    const int r0 = carve_block(c, n, scr, s);
    if (r0) {
      h->err = c->err;
      return r0;
    }
  }
  c->st = h->st;
  c->occ = h->occ;
  c->host = h->host;
  c->fmax = h->fmax;
  c->fcut_rel = h->fcut_rel;
  c->deg_tol = h->deg_tol;
  c->timing = false;
  c->ktiming = false;
  c->s_valid = false;  // the scratch is shared: S is always factored
  CoopScope cs(h);
  int r = dm_core(c, n, H, ldh, S, lds, SKey{n, false, 0ull}, ne, kT, D, ldd, E, lde, s);
  c->s_valid = false;
  if (eval && r == HSDM_OK) {
    HSDM_LAUNCH(copy_vec_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, c->lam, eval, n);
    DEV_TRY(h, hipGetLastError());
  }
  if (r == HSDM_OK) r = finish(c, s);
  if (r != HSDM_OK) {
    if (!c->err.empty()) h->err = c->err;
    h->detail = c->detail;
  }
  if (mu) *mu = h->host->occ.mu;
  if (band_energy) *band_energy = h->host->occ.band_energy;
  return r;
}

int hsdm_solve_dm_complex(hsdm_handle h, int n, const void* H, int ldh, const void* S, int lds,
                          double ne, double kT, void* D, int ldd, void* E, int lde, double* eval,
                          double* band_energy, double* mu, void* stream) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!H) return -3;
  if (bad_ld(ldh, n)) return -4;
  if (!S) return -5;
  if (bad_ld(lds, n)) return -6;
  if (!(ne >= 0.0) || !std::isfinite(ne) || ne > h->fmax * n) return -7;
  if (!(kT >= 0.0) || !std::isfinite(kT)) return -8;
  if (!D) return -9;
  if (bad_ld(ldd, n)) return -10;
  if (E && bad_ld(lde, n)) return -12;
  if (n > (1 << 30) / 2) return -2;
  h->err.clear();
  hipStream_t s = (hipStream_t)stream;
  DEV_TRY(h, hipSetDevice(h->device));
  const int n2 = 2 * n;
  int r = ensure_ws(h, n2, s);
  if (r) return r;
  if ((r = ensure_cws(h, n, s))) return r;
  SKey key;
  if ((r = s_key(h, S, n, lds, true, key, s))) return r;
  KtScope kts(h);
  if (!s_cached(h, key)) DEV_TRY(h, herm_embed(n, S, lds, h->SR, n2, s));
  DEV_TRY(h, herm_embed(n, H, ldh, h->HR, n2, s));
  r = dm_core(h, n2, h->HR, n2, h->SR, n2, key, 2.0 * ne, kT, h->DR, n2, E ? h->ER : nullptr, n2,
              s);
  if (r == HSDM_OK) {
    DEV_TRY(h, herm_extract(n, h->DR, n2, D, ldd, s));
    if (E) DEV_TRY(h, herm_extract(n, h->ER, n2, E, lde, s));
    if (eval) DEV_TRY(h, herm_pair_eval(n, h->lam, eval, s));
    r = finish(h, s);
  }
  if (mu) *mu = h->host->occ.mu;
  if (band_energy) *band_energy = 0.5 * h->host->occ.band_energy;
  return r;
}

}  // extern "C"

namespace {

// One task of a multi-task solve.
struct TaskSpec {
  int cplx, n;
  const void *H, *S;
  int ldh, lds;
  void *D, *E;
  int ldd, lde;
  double w;             // weight in a shared electron count
  double ne, kT, fmax;  // own electron count and occupations (independent tasks)
};

// Task contexts for the tasks of one call: first a context that holds the
// factor of the task's S, then the least recently used of the others
// (created as needed).
int pick_contexts(hsdm_ctx* h, int nt, const TaskSpec* T, const std::vector<SKey>& keys,
                  std::vector<hsdm_ctx*>& ctx) {
  ctx.assign(nt, nullptr);
  std::vector<char> used(h->subs.size(), 0);
  for (int p = 0; p < nt; p++) {
    const SKey& key = keys[p];
    for (size_t i = 0; i < h->subs.size(); i++)
      if (!used[i] && s_cached(h->subs[i], key)) {
        used[i] = 1;
        ctx[p] = h->subs[i];
        break;
      }
  }
  for (int p = 0; p < nt; p++) {
    if (ctx[p]) continue;
    long best = -1;
    for (size_t i = 0; i < h->subs.size(); i++)
      if (!used[i] && (best < 0 || h->subs[i]->last_use < h->subs[best]->last_use)) best = (long)i;
    if (best < 0) {
      hsdm_ctx* c = nullptr;
      const int r = hsdm_init(&c, h->device);
      if (r) {
        h->err = "task context allocation failed";
        return r;
      }
      h->subs.push_back(c);
      used.push_back(0);
      best = (long)h->subs.size() - 1;
    }
    used[best] = 1;
    ctx[p] = h->subs[best];
  }
  for (int p = 0; p < nt; p++) ctx[p]->last_use = ++h->use_clock;
  return HSDM_OK;
}

// The tasks' path: A1-A6 for each task, the bands of all tasks in shared
// cooperative launches, then the occupations (one chemical potential for all
// tasks when `shared`, Eq. (16); else each task's own), then A8-A12 for
// each task.  Outputs on the host: the shared mu and weighted band energy,
// and each task's mu and band energy.
int solve_tasks(hsdm_ctx* h, int nt, const TaskSpec* T, bool shared, double ne, double kT,
                double* eb_total, double* mu_shared, double* eb_each, double* mu_each,
                hipStream_t s) {
  int r;
  std::vector<SKey> keys(nt);
  {
    std::vector<const void*> sp(nt);
    std::vector<int> sn(nt), sl(nt), sc(nt);
    std::vector<unsigned long long> hv(nt);
    for (int p = 0; p < nt; p++) {
      sp[p] = T[p].S;
      sn[p] = T[p].n;
      sl[p] = T[p].lds;
      sc[p] = T[p].cplx;
    }
    if ((r = s_hashes(h, nt, sp.data(), sn.data(), sl.data(), sc.data(), hv.data(), s))) return r;
    for (int p = 0; p < nt; p++) keys[p] = SKey{T[p].n, T[p].cplx != 0, hv[p]};
  }
  std::vector<hsdm_ctx*> ctx;
  if ((r = pick_contexts(h, nt, T, keys, ctx))) return r;
  if (h->d_tasks_cap < nt) {
    if (h->d_tasks) (void)hipFree(h->d_tasks);
    h->d_tasks = nullptr;
    h->d_tasks_cap = 0;
    DEV_TRY(h, hipMalloc(&h->d_tasks, sizeof(OccTask) * nt));
    h->d_tasks_cap = nt;
  }
  // Tasks that share an S (the same caller buffer, size and leading
  // dimension, e.g. the spin channels of one k-point) use the factor of the
  // first of them.  The tasks' independent phases run on the worker streams
  // when there are several tasks (and not every launch is timed): each group
  // of tasks sharing an S on one lane, groups placed largest first on the
  // least loaded lane.
  std::vector<int> src(nt), lane(nt, 0);
  for (int p = 0; p < nt; p++) {
    src[p] = p;
    for (int q = 0; q < p; q++)
      if (src[q] == q && T[q].S == T[p].S && T[q].n == T[p].n && T[q].lds == T[p].lds &&
          T[q].cplx == T[p].cplx) {
        src[p] = q;
        break;
      }
  }
  const bool use_lanes = nt > 1 && !h->kt_every;
  const int nl = use_lanes ? h->nlane : 0;
  std::vector<std::vector<int>> order(use_lanes ? nl : 1);  // tasks of each lane, in order
  if (use_lanes) {
    if ((r = ensure_lanes(h))) return r;
    std::vector<int> groups;
    std::vector<double> work(nt, 0.0);
    for (int p = 0; p < nt; p++) {
      const double nr = T[p].cplx ? 2.0 * T[p].n : (double)T[p].n;
      work[src[p]] += nr * nr * nr;
      if (src[p] == p) groups.push_back(p);
    }
    std::stable_sort(groups.begin(), groups.end(),
                     [&](int x, int y) { return work[x] > work[y]; });
    double load[NLANE] = {};
    for (int g : groups) {
      const int k = (int)(std::min_element(load, load + nl) - load);
      load[k] += work[g];
      for (int p = g; p < nt; p++)
        if (src[p] == g) {
          lane[p] = k;
          order[k].push_back(p);
        }
    }
  } else {
    for (int p = 0; p < nt; p++) order[0].push_back(p);
  }
  // issue order: the lanes' task lists interleaved, so that every lane has
  // work queued early
  std::vector<int> issue;
  for (size_t i = 0;; i++) {
    bool any = false;
    for (auto& o : order)
      if (i < o.size()) {
        issue.push_back(o[i]);
        any = true;
      }
    if (!any) break;
  }
  auto stream_of = [&](int p) { return use_lanes ? h->lane_s[lane[p]] : s; };
  for (size_t k = 0; k < order.size(); k++) {
    int nk = 0;
    for (int p : order[k])
      if (T[p].cplx) nk = std::max(nk, T[p].n);
    if ((r = ensure_lane_cws(h, (int)k, nk, s))) return r;
  }
  for (int p = 0; p < nt; p++) {
    hsdm_ctx* c = ctx[p];
    c->err.clear();
    if ((r = ensure_ws(c, T[p].cplx ? 2 * T[p].n : T[p].n, s))) {
      h->err = c->err;
      return r;
    }
  }
  // The refined form (HSDM_KEY_PRECISION = 1): every task's FP32 reduction
  // and, after the occupations, its refinement run one task after another
  // on s (their bulge chasing, panel QRs and stage-2 back-transform need
  // their workgroups placed together, so they do not share the device), in
  // one workspace of the handle sized for the largest task; each task keeps
  // its FP64 reflectors, eigenvectors and standard-form matrix in its own.
  const bool refined = h->precision == 1;
  if (refined) {
    int nmax = 0;
    for (int p = 0; p < nt; p++) nmax = std::max(nmax, T[p].cplx ? 2 * T[p].n : T[p].n);
    if ((r = ensure_rws(h, nmax, s))) return r;
    for (int p = 0; p < nt; p++) {
      hsdm_ctx* c = ctx[p];
      c->A32 = h->A32; c->V32 = h->V32; c->Z32 = h->Z32; c->f32_scr = h->f32_scr;
      c->bt1f = h->bt1f; c->ref_scr = h->ref_scr; c->rrec = h->rrec;
      c->refine_steps = h->refine_steps;
    }
  }
  KtScope kts(h);
  Lanes lanes{h, s, nl};
  for (int p = 0; p < NPHASE; p++) h->phase_done[p] = false;
  h->last_kind = 0;
  h->h_tasks.assign(nt, OccTask{});
  DEV_TRY(h, lanes.fork());
  // 1. every task: factor, standard form
  for (int p : issue) {
    hsdm_ctx* c = ctx[p];
    hsdm_ctx* L = lane_cws(h, use_lanes ? lane[p] : 0);
    const hipStream_t ls = stream_of(p);
    const TaskSpec& t = T[p];
    c->fmax = shared ? h->fmax : t.fmax;
    c->fcut_rel = h->fcut_rel;
    c->deg_tol = h->deg_tol;
    c->timing = false;
    c->ktiming = false;
    const int nr = t.cplx ? 2 * t.n : t.n;
    const SKey& key = keys[p];
    const bool own = src[p] == p;
    const double *Hr = (const double*)t.H, *Sr = (const double*)t.S;
    int ldhr = t.ldh, ldsr = t.lds;
    if (t.cplx) {
      if (own && !s_cached(c, key)) DEV_TRY(h, herm_embed(t.n, t.S, t.lds, L->SR, nr, ls));
      DEV_TRY(h, herm_embed(t.n, t.H, t.ldh, L->HR, nr, ls));
      Hr = L->HR;
      Sr = L->SR;
      ldhr = ldsr = nr;
    }
    HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, ls, c->st, c->occ);
    DEV_TRY(h, hipGetLastError());
    if (own && (r = factor_s(c, nr, Sr, ldsr, key, ls))) return r;
    if (c->deg_tol < 0.0) DEV_TRY(h, dev_norm1_sym(Hr, ldhr, nr, c->colsum, c->hnorm, ls));
    if ((r = standard_form(c, nr, Hr, ldhr, ctx[src[p]]->Linv, nr, c->Abuf, nr, ls))) return r;
    DEV_TRY(h, bt1_zero_fill(nr, BAND, c->Vst, nr, ls));
    h->h_tasks[p] = OccTask{c->lam, c->fvec, c->occ, c->deg_tol < 0.0 ? c->hnorm : nullptr, nr,
                            t.w};
  }
  DEV_TRY(h, lanes.join());
  if (refined) {
    // every task on s: FP32 reduction with FP64 panels, bulge chasing,
    // every eigenpair of the tridiagonal (the refinement corrects the
    // wanted vectors with all the others)
    for (int p : issue) {
      hsdm_ctx* c = ctx[p];
      const TaskSpec& t = T[p];
      const int nr = t.cplx ? 2 * t.n : t.n;
      if ((r = reduce_f32(c, nr, s, 3))) {
        h->err = c->err;
        return r;
      }
      DEV_TRY(h, stedc_run(c->plan, c->dvec, c->evec, c->lam, c->Zbuf, nr, c->dc_scr,
                           c->dc_iscr, nullptr, nullptr, nullptr, c->st, s));
      if (!shared) {
        OccHook hook{c, nr, t.cplx ? 2.0 * t.ne : t.ne, t.kT};
        DEV_TRY(h, occ_hook(&hook, c->lam, s));
      }
    }
  }
  // full -> band of all tasks, pair step by pair step, the panel QRs of a
  // step in shared cooperative launches
  if (!refined) {
    h->sy_args.resize(nt);
    for (int p = 0; p < nt; p++) {
      hsdm_ctx* c = ctx[p];
      const int nr = T[p].cplx ? 2 * T[p].n : T[p].n;
      h->sy_args[p] = Sy2sbArgs{nr, c->Abuf, nr, c->Vst, nr, c->tau1, c->T1, c->AB, 2 * BAND,
                                c->sy_scr, c->st};
    }
    const size_t need = sy2sb_group_bytes(nt, h->sy_args.data(), BAND, h->sy_host);
    if (h->d_qr_bytes < need) {
      if (h->d_qr) (void)hipFree(h->d_qr);
      h->d_qr = nullptr;
      h->d_qr_bytes = 0;
      DEV_TRY(h, hipMalloc(&h->d_qr, need));
      h->d_qr_bytes = need;
    }
    DEV_TRY(h, sy2sb_run_group(nt, h->sy_args.data(), BAND, h->sy_host, h->d_qr, s));
    for (int p = 0; p < nt; p++) {
      hsdm_ctx* c = ctx[p];
      DEV_TRY(h, sb2st_prepare(c->lay, c->V2, c->tau2, c->progress, s));
    }
  }
  // 2. bulge chasing of all bands, as many per cooperative launch as fit:
  //    each band alone is latency-bound and fills a small part of the device.
  //    A launch lasts as long as its largest band, so the bands go into the
  //    launches largest first.
  if (!refined) {
    h->h_sb.assign(nt, Sb2stTask{});
    h->h_wgmap.clear();
    std::vector<int> by_size(nt);
    for (int p = 0; p < nt; p++) by_size[p] = p;
    std::stable_sort(by_size.begin(), by_size.end(),
                     [&](int x, int y) { return ctx[x]->lay.n > ctx[y]->lay.n; });
    std::vector<int> first(1, 0);  // first entry of by_size in each launch
    std::vector<double> fl(1, 0.0), by(1, 0.0);
    int in_launch = 0;
    for (int i = 0; i < nt; i++) {
      const int p = by_size[i];
      hsdm_ctx* c = ctx[p];
      const int w = sb2st_group_nwg(c->lay);
      if (w > 0 && in_launch + w > SB2ST_MAX_WG) {
        first.push_back(i);
        fl.push_back(0.0);
        by.push_back(0.0);
        in_launch = 0;
      }
      h->h_sb[p] = Sb2stTask{c->AB, c->V2, c->tau2, c->d_goff, c->progress, c->st, c->lay.n,
                             c->lay.nsweep, in_launch, w};
      for (int q = 0; q < w; q++) h->h_wgmap.push_back(p);
      in_launch += w;
      fl.back() += sb2st_algo_flops(c->lay);
      by.back() += sb2st_algo_bytes(c->lay);
    }
    first.push_back(nt);
    const size_t tb = sizeof(Sb2stTask) * nt;
    const size_t need = tb + sizeof(int) * (h->h_wgmap.size() + 1);
    if (h->d_sb_bytes < need) {
      if (h->d_sb) (void)hipFree(h->d_sb);
      h->d_sb = nullptr;
      h->d_sb_bytes = 0;
      DEV_TRY(h, hipMalloc(&h->d_sb, need));
      h->d_sb_bytes = need;
    }
    Sb2stTask* d_sb = (Sb2stTask*)h->d_sb;
    int* d_map = (int*)((char*)h->d_sb + tb);
    DEV_TRY(h, hipMemcpyAsync(d_sb, h->h_sb.data(), tb, hipMemcpyHostToDevice, s));
    if (!h->h_wgmap.empty())
      DEV_TRY(h, hipMemcpyAsync(d_map, h->h_wgmap.data(), sizeof(int) * h->h_wgmap.size(),
                                hipMemcpyHostToDevice, s));
    int off = 0;
    for (size_t g = 0; g + 1 < first.size(); g++) {
      int cnt = 0;
      for (int i = first[g]; i < first[g + 1]; i++) cnt += h->h_sb[by_size[i]].nwg;
      DEV_TRY(h, sb2st_group_launch(d_sb, d_map + off, cnt, fl[g], by[g], s));
      off += cnt;
    }
  }
  // 3. every task: eigenpairs of the tridiagonal (all of them when the
  //    occupations are shared: they are not known yet)
  DEV_TRY(h, lanes.fork());
  for (int p : issue) {
    if (refined) break;
    hsdm_ctx* c = ctx[p];
    const hipStream_t ls = stream_of(p);
    const TaskSpec& t = T[p];
    const int nr = t.cplx ? 2 * t.n : t.n;
    DEV_TRY(h, sb2st_finish(c->lay, c->AB, 2 * BAND, c->dvec, c->evec, ls));
    if (shared) {
      DEV_TRY(h, stedc_run(c->plan, c->dvec, c->evec, c->lam, c->Zbuf, nr, c->dc_scr,
                           c->dc_iscr, nullptr, nullptr, nullptr, c->st, ls));
    } else {
      OccHook hook{c, nr, t.cplx ? 2.0 * t.ne : t.ne, t.kT};
      DEV_TRY(h, stedc_run(c->plan, c->dvec, c->evec, c->lam, c->Zbuf, nr, c->dc_scr,
                           c->dc_iscr, &c->occ->m, occ_hook, &hook, c->st, ls));
    }
  }
  DEV_TRY(h, lanes.join());
  // 4. one chemical potential for all tasks (Eq. (16))
  HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, s, h->st, h->occ);
  DEV_TRY(h, hipGetLastError());
  if (shared) {
    DEV_TRY(h, hipMemcpyAsync(h->d_tasks, h->h_tasks.data(), sizeof(OccTask) * nt,
                              hipMemcpyHostToDevice, s));
    DEV_TRY(h, occupations_joint_launch(nt, h->d_tasks, h->fmax, ne, kT, h->deg_tol,
                                        h->fcut_rel * h->fmax, h->occ, h->st, s));
  }
  if (refined) {
    // the wanted count of each task at the unrefined eigenvalues, with a
    // margin for the states the refinement moves across the occupation
    // cut; the refinement of those vectors (both back-transforms of every
    // vector first); the occupations again at the refined eigenvalues
    for (int p = 0; p < nt; p++)
      DEV_TRY(h, hipMemcpyAsync(&ctx[p]->host->occ, ctx[p]->occ, sizeof(OccOut),
                                hipMemcpyDeviceToHost, s));
    DEV_TRY(h, hipStreamSynchronize(s));
    for (int p : issue) {
      hsdm_ctx* c = ctx[p];
      const TaskSpec& t = T[p];
      const int nr = t.cplx ? 2 * t.n : t.n;
      const int m0 = c->host->occ.m;
      const int mref = std::min(nr, m0 + std::max(32, m0 / 32));
      // the FP32 reflectors of stage 1 (the shared workspace held another
      // task's meanwhile): the FP64 ones rounded, as the reduction made them
      DEV_TRY(h, dev_convert(c->Vst, nr, c->V32, nr, nr, nr, s));
      if ((r = refine_vectors(c, nr, mref, c->lam, s))) {
        h->err = c->err;
        return r;
      }
      if (!shared) {
        OccHook hook{c, nr, t.cplx ? 2.0 * t.ne : t.ne, t.kT};
        DEV_TRY(h, occ_hook(&hook, c->lam, s));
      }
    }
    if (shared) {
      HSDM_LAUNCH(reset_status_kernel, dim3(1), dim3(64), 0, s, h->st, h->occ);
      DEV_TRY(h, hipGetLastError());
      DEV_TRY(h, occupations_joint_launch(nt, h->d_tasks, h->fmax, ne, kT, h->deg_tol,
                                          h->fcut_rel * h->fmax, h->occ, h->st, s));
    }
  }
  // 5. stage-2 back-transform of all tasks' occupied vectors in one launch
  // (the refined form has transformed every vector back already)
  h->h_bt2.resize(nt);
  for (int p = 0; p < nt && !refined; p++) {
    hsdm_ctx* c = ctx[p];
    const int nr = T[p].cplx ? 2 * T[p].n : T[p].n;
    DEV_TRY(h, bt2_prepare(c->lay, c->V2, c->tau2, c->F2, s));
    h->h_bt2[p] = bt2_task(c->lay, c->F2, c->d_goff, c->Zbuf, nr, nr, &c->occ->m, c->progress,
                           c->st);
  }
  if (!refined) {
    const size_t need = sizeof(Bt2Task) * (nt + 1) +
                        sizeof(int) * (bt2_group_map_ints(nt, h->h_bt2.data()) + 1);
    if (h->d_bt2_bytes < need) {
      if (h->d_bt2) (void)hipFree(h->d_bt2);
      h->d_bt2 = nullptr;
      h->d_bt2_bytes = 0;
      DEV_TRY(h, hipMalloc(&h->d_bt2, need));
      h->d_bt2_bytes = need;
    }
    Bt2Task* d_t = (Bt2Task*)h->d_bt2;
    int* d_m = (int*)((char*)h->d_bt2 + sizeof(Bt2Task) * (nt + 1));
    DEV_TRY(h, bt2_group_apply(nt, h->h_bt2.data(), h->h_bt2map, d_t, d_m, s));
  }
  // 6. every task: the other back-transforms, D and E
  DEV_TRY(h, lanes.fork());
  for (int p : issue) {
    kt_set_tag(p);
    hsdm_ctx* c = ctx[p];
    hsdm_ctx* L = lane_cws(h, use_lanes ? lane[p] : 0);
    const hipStream_t ls = stream_of(p);
    const TaskSpec& t = T[p];
    const int nr = t.cplx ? 2 * t.n : t.n;
    const int* m_dev = &c->occ->m;
    if (!refined)
      DEV_TRY(h, bt1_apply(nr, BAND, c->Vst, nr, c->T1, c->Zbuf, nr, nr, m_dev, c->bt1_scr, ls));
    GemmArgs g{};
    g.m = nr; g.n = nr; g.k = nr; g.A = ctx[src[p]]->Linv; g.lda = nr; g.B = c->Zbuf; g.ldb = nr;
    g.C = c->Cbuf; g.ldc = nr; g.alpha = 1.0; g.beta = 0.0; g.ta = 1; g.tb = 0;
    g.flags = GF_KA_UPPER; g.ndev = m_dev;
    DEV_TRY(h, gemm_launch(g, ls));
    if (t.cplx) {
      DEV_TRY(h, density_launch(nr, nr, c->Cbuf, nr, c->fvec, c->lam, L->DR, nr,
                                t.E ? L->ER : nullptr, nr, m_dev, ls));
      DEV_TRY(h, herm_extract(t.n, L->DR, nr, t.D, t.ldd, ls));
      if (t.E) DEV_TRY(h, herm_extract(t.n, L->ER, nr, t.E, t.lde, ls));
    } else {
      DEV_TRY(h, density_launch(nr, nr, c->Cbuf, nr, c->fvec, c->lam, (double*)t.D, t.ldd,
                                (double*)t.E, t.E ? t.lde : nr, m_dev, ls));
    }
  }
  DEV_TRY(h, lanes.join());
  kt_set_tag(-1);
  // status of every task, then of the shared occupations
  h->tag_m.assign(nt, 0);
  double bt2_work = 0.0;
  for (int p = 0; p < nt; p++) {
    hsdm_ctx* c = ctx[p];
    if ((r = finish(c, s))) {
      h->detail = c->detail;
      h->err = "task " + std::to_string(p) + ": " + c->err;
      h->tag_m.clear();
      return r;
    }
    h->tag_m[p] = c->host->occ.m;
    bt2_work += bt2_flops(c->lay, c->host->occ.m);
    const double half = T[p].cplx ? 0.5 : 1.0;
    if (eb_each) eb_each[p] = half * c->host->occ.band_energy;
    if (mu_each) mu_each[p] = c->host->occ.mu;
  }
  kt_set_last_work("bt2_group_kernel", bt2_work, 0.0);
  r = finish(h, s);
  h->tag_m.clear();
  if (mu_shared) *mu_shared = h->host->occ.mu;
  if (eb_total) *eb_total = h->host->occ.band_energy;
  return r;
}

double ctx_bytes(const hsdm_ctx* c) {
  double b = (c->ws_raw && !c->borrowed) ? (double)c->ws_cap : 0.0;
  if (c->cws) b += 16.0 * 8.0 * (double)c->cws_n * c->cws_n;
  if (c->rws_raw) b += (double)c->rws_cap;  // the refined form's workspace
  return b;
}

}  // namespace

extern "C" {

int hsdm_solve_dm_batch(hsdm_handle h, int nprob, int is_complex, const int* n,
                        const void* const* H, const int* ldh, const void* const* S,
                        const int* lds, const double* weight, double ne, double kT,
                        void* const* D, const int* ldd, void* const* E, const int* lde,
                        double* band_energy, double* mu, void* stream) {
  if (!h) return -1;
  if (nprob < 1) return -2;
  if (is_complex != 0 && is_complex != 1) return -3;
  if (!n || !H || !ldh || !S || !lds || !D || !ldd || (E && !lde)) return -4;
  double cap = 0.0;
  std::vector<TaskSpec> T(nprob);
  for (int p = 0; p < nprob; p++) {
    if (n[p] < 1 || (is_complex && n[p] > (1 << 29))) return -4;
    if (!H[p]) return -5;
    if (bad_ld(ldh[p], n[p])) return -6;
    if (!S[p]) return -7;
    if (bad_ld(lds[p], n[p])) return -8;
    const double w = weight ? weight[p] : 1.0;
    if (!(w > 0.0) || !std::isfinite(w)) return -9;
    if (!D[p]) return -12;
    if (bad_ld(ldd[p], n[p])) return -13;
    if (E && E[p] && bad_ld(lde[p], n[p])) return -15;
    cap += w * n[p];
    T[p] = TaskSpec{is_complex, n[p], H[p], S[p], ldh[p], lds[p], D[p], E ? E[p] : nullptr,
                    ldd[p], E ? lde[p] : n[p], w, 0.0, 0.0, h->fmax};
  }
  if (!(ne >= 0.0) || !std::isfinite(ne) || ne > h->fmax * cap * (1.0 + 1e-15)) return -10;
  if (!(kT >= 0.0) || !std::isfinite(kT)) return -11;
  h->err.clear();
  DEV_TRY(h, hipSetDevice(h->device));
  double eb = 0.0, m = 0.0;
  const int r = solve_tasks(h, nprob, T.data(), true, is_complex ? 2.0 * ne : ne, kT, &eb, &m,
                            nullptr, nullptr, (hipStream_t)stream);
  if (mu) *mu = m;
  if (band_energy) *band_energy = (is_complex ? 0.5 : 1.0) * eb;
  return r;
}

int hsdm_solve_dm_group(hsdm_handle h, int nprob, const int* is_complex, const int* n,
                        const void* const* H, const int* ldh, const void* const* S,
                        const int* lds, const double* n_electrons, const double* kT,
                        const double* f_max, void* const* D, const int* ldd, void* const* E,
                        const int* lde, double* band_energy, double* mu, void* stream) {
  if (!h) return -1;
  if (nprob < 1) return -2;
  if (!is_complex || !n || !H || !ldh || !S || !lds || !n_electrons || !kT || !D || !ldd ||
      (E && !lde))
    return -3;
  std::vector<TaskSpec> T(nprob);
  for (int p = 0; p < nprob; p++) {
    if (is_complex[p] != 0 && is_complex[p] != 1) return -3;
    if (n[p] < 1 || (is_complex[p] && n[p] > (1 << 29))) return -4;
    if (!H[p]) return -5;
    if (bad_ld(ldh[p], n[p])) return -6;
    if (!S[p]) return -7;
    if (bad_ld(lds[p], n[p])) return -8;
    const double fm = f_max ? f_max[p] : h->fmax;
    if (!(fm > 0.0) || !std::isfinite(fm)) return -11;
    if (!(n_electrons[p] >= 0.0) || !std::isfinite(n_electrons[p]) || n_electrons[p] > fm * n[p])
      return -9;
    if (!(kT[p] >= 0.0) || !std::isfinite(kT[p])) return -10;
    if (!D[p]) return -12;
    if (bad_ld(ldd[p], n[p])) return -13;
    if (E && E[p] && bad_ld(lde[p], n[p])) return -15;
    T[p] = TaskSpec{is_complex[p], n[p], H[p], S[p], ldh[p], lds[p], D[p],
                    E ? E[p] : nullptr, ldd[p], E ? lde[p] : n[p], 1.0, n_electrons[p], kT[p], fm};
  }
  h->err.clear();
  DEV_TRY(h, hipSetDevice(h->device));
  return solve_tasks(h, nprob, T.data(), false, 0.0, 0.0, nullptr, nullptr, band_energy, mu,
                     (hipStream_t)stream);
}

double hsdm_task_bytes(int n, int is_complex) {
  if (n < 1) return 0.0;
  const int nr = is_complex ? 2 * n : n;
  return ws_bytes(nr) + (is_complex ? 16.0 * 8.0 * (double)n * n : 0.0);
}

double hsdm_workspace_bytes(hsdm_handle h) {
  if (!h) return 0.0;
  double b = ctx_bytes(h);
  for (const hsdm_ctx* c : h->subs) b += ctx_bytes(c);
  for (const hsdm_ctx* c : h->lane_buf)
    if (c) b += ctx_bytes(c);
  return b;
}

int hsdm_release_tasks(hsdm_handle h, double keep_bytes) {
  if (!h) return -1;
  if (!(keep_bytes >= 0.0)) return -2;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  auto tasks_bytes = [&]() {
    double b = h->cws ? 16.0 * 8.0 * (double)h->cws_n * h->cws_n : 0.0;
    for (const hsdm_ctx* c : h->subs) b += ctx_bytes(c);
    for (const hsdm_ctx* c : h->lane_buf)
      if (c) b += ctx_bytes(c);
    return b;
  };
  // the worker lanes' embedding buffers first (rebuilt by the next call
  // that needs them), then task contexts, least recently used first
  for (int k = NLANE - 1; k > 0 && tasks_bytes() > keep_bytes; k--)
    if (h->lane_buf[k]) free_cws(h->lane_buf[k]);
  while (!h->subs.empty() && tasks_bytes() > keep_bytes) {
    size_t lru = 0;
    for (size_t i = 1; i < h->subs.size(); i++)
      if (h->subs[i]->last_use < h->subs[lru]->last_use) lru = i;
    hsdm_finalize(h->subs[lru]);
    h->subs.erase(h->subs.begin() + (long)lru);
  }
  if (h->subs.empty() && tasks_bytes() > keep_bytes) free_cws(h);
  return HSDM_OK;
}

}  // extern "C"
