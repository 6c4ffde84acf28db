// Host launchers of the reduction, tridiagonal and back-transformation phases.
#pragma once
#include <vector>
#include "hsdm_internal.h"

// gemm.hip -- X = A Y for a symmetric A (lower triangle stored), n <= 32
// columns: g describes the first pass (GF_A_TRIL, m = k; C = g.C, alpha 1,
// beta 0); both passes run split over K in one launch, their partials
// (ceil(k / kchunk) m x n slices each) in part1 and part2, then one reduction
// writes C.  The roundings are those of the two passes reduced one after
// the other.
hipError_t gemm_sym_pair_launch(const GemmArgs& g, int kchunk, double* part1, double* part2,
                                hipStream_t s);
hipError_t gemm_sym_pair_launch(const GemmArgsF& g, int kchunk, float* part1, float* part2,
                                hipStream_t s);

// sy2sb.hip -- full -> band (half-bandwidth B).  A (lower triangle) is
// overwritten; Vst receives the explicit panel reflectors (n x n, lower
// trapezoid), tau1 the scalars, T1 one B x B triangular factor per panel, AB
// the band in band storage (ldab >= 2B rows per column, rows > B zeroed).
size_t sy2sb_scratch_doubles(int n, int B);
// The refined form's reduction: A (lower triangle) in FP32 with FP32
// trailing updates; the panel QRs in FP64 into Vst, tau1, T1 as above; V32
// (n x n, ld ldv32) receives the FP32 roundings of the reflectors; AB the
// band in FP64.  scratch: sy2sb_f32_scratch_bytes(n, B) bytes.
size_t sy2sb_f32_scratch_bytes(int n, int B);
hipError_t sy2sb_f32_run(int n, int B, float* A, long lda, double* Vst, long ldv, float* V32,
                         long ldv32, double* tau1, double* T1, double* AB, int ldab,
                         void* scratch, DevStatusWord* st, hipStream_t s);
hipError_t sy2sb_run(int n, int B, double* A, long lda, double* Vst, long ldv, double* tau1,
                     double* T1, double* AB, int ldab, double* scratch, DevStatusWord* st,
                     hipStream_t s);

// The same for several matrices at once: the tasks advance one panel pair
// per round, and every step of a round runs in shared launches over the
// tasks (each task's panel QR and tall-skinny products alone fill few
// compute units); only the trailing rank-2B / rank-4B updates stay one
// launch per task.  The host vectors are the caller's (kept until the stream
// has run the work); d_buf is device memory of sy2sb_group_bytes(...) bytes.
struct Sy2sbArgs {
  int n;
  double* A;
  long lda;
  double* Vst;
  long ldv;
  double* tau1;
  double* T1;
  double* AB;
  int ldab;
  double* scratch;
  DevStatusWord* st;
};
struct PanelQrTask {
  double *P, *V, *tau, *T, *part, *prow, *gpart;
  DevStatusWord* st;
  long ldp, ldv, span;
  int h, g0, G, pad;
};
// out (B x B, leading dimension ldo) = U^T W for h x B operands, from G
// per-workgroup partial sums in part; b0: the item's first workgroup
struct AtbGroupItem {
  const double* U;
  const double* W;
  double* part;
  double* out;
  long ldu, ldw, ldo;
  int h, G, b0, pad;
};
// dst (m x n, leading dimension ldd) = src (leading dimension lds)
struct CopyGroupItem {
  const double* src;
  double* dst;
  long lds, ldd;
  int m, n;
};
struct Sy2sbGroupHost {
  std::vector<PanelQrTask> desc;
  std::vector<int> wgmap;
  std::vector<GemmGroupItem> gemm;  // grouped tall-skinny products of every round
  std::vector<int> gemmmap;
  std::vector<AtbGroupItem> atb;
  std::vector<int> atbmap;
  std::vector<CopyGroupItem> copy;
};
size_t sy2sb_group_bytes(int nt, const Sy2sbArgs* t, int B, Sy2sbGroupHost& host);
hipError_t sy2sb_run_group(int nt, const Sy2sbArgs* t, int B, Sy2sbGroupHost& host, void* d_buf,
                           hipStream_t s);

// sb2st.hip -- band -> tridiagonal by bulge chasing.  ldab must be 2B and AB
// must have B + 1 spare columns after the n used ones.  AB is overwritten;
// d (n) and e (n-1) receive the tridiagonal; the stage-2 reflectors are
// stored group-wise in V2 (see sb2st_layout) with their scalars in tau2.
struct Sb2stLayout {
  int n, B;
  int nsweep;       // sweeps that create reflectors
  int nblk;         // sweep blocks of B sweeps
  int tmax;         // max tasks per sweep
  long ngroups;     // groups (sweep block, task)
  long v2_doubles;  // size of V2 (2B x B per group)
};
Sb2stLayout sb2st_layout(int n, int B);
// group offset table: first group index of each sweep block (nblk + 1 entries)
void sb2st_group_offsets(const Sb2stLayout& L, long* offs);
hipError_t sb2st_run(const Sb2stLayout& L, double* AB, int ldab, double* d, double* e, double* V2,
                     double* tau2, const long* d_goff, int* progress, DevStatusWord* st,
                     hipStream_t s);
// The same, split for several bands chased in one cooperative launch:
// sb2st_prepare (clears the reflector store and the sweep counters) for each
// band, one sb2st_group_launch over bands whose workgroup counts
// (sb2st_group_nwg each) add up to at most SB2ST_MAX_WG, then sb2st_finish
// (reads d and e off the band) for each.  d_tasks and d_wg_task are device
// arrays: one Sb2stTask per band and the task index of each workgroup.
constexpr int SB2ST_MAX_WG = 1024;  // four 2-wavefront workgroups per compute unit
struct Sb2stTask {
  double* AB;  // ldab = 2B
  double* V2;
  double* tau2;
  const long* goff;
  int* progress;
  DevStatusWord* st;
  int n, nsweep, wg0, nwg;
};
hipError_t sb2st_prepare(const Sb2stLayout& L, double* V2, double* tau2, int* progress,
                         hipStream_t s);
hipError_t sb2st_finish(const Sb2stLayout& L, const double* AB, int ldab, double* d, double* e,
                        hipStream_t s);
int sb2st_group_nwg(const Sb2stLayout& L);
// algorithmic flops and HBM bytes of one band's reduction (timer records)
double sb2st_algo_flops(const Sb2stLayout& L);
double sb2st_algo_bytes(const Sb2stLayout& L);
hipError_t sb2st_group_launch(const Sb2stTask* d_tasks, const int* d_wg_task, int total_wg,
                              double flops, double bytes, hipStream_t s);

// bt.hip -- back-transformations.
// Z (n x m) <- Q2 Z.  bt2_prepare forms the T factor of every group and packs
// V, T into matrix-core operand order (bt2_pack_doubles doubles); bt2_apply
// applies all groups, one workgroup per strip of 16 columns of Z.
size_t bt2_pack_doubles(const Sb2stLayout& L);
hipError_t bt2_prepare(const Sb2stLayout& L, const double* V2, const double* tau2, double* F2,
                       hipStream_t s);
// iscratch: ceil(m / 16) ints of device scratch (cleared here).
hipError_t bt2_apply(const Sb2stLayout& L, const double* F2, const long* d_goff, double* Z,
                     long ldz, int m, const int* m_dev, int* iscratch, DevStatusWord* st,
                     hipStream_t s);
// Several Z's in one launch (one task each): bt2_task describes a task like
// bt2_apply's arguments (m: host bound of the device count); bt2_group_apply
// clears every task's counters and launches all their strips together.
// tasks and hmap are the caller's host arrays (kept until the stream has run
// the work); d_tasks holds nt descriptors, d_map bt2_group_map_ints ints
// (two per workgroup).
constexpr int NSPLIT = 8;
struct SplitRanges {
  int hi[NSPLIT];  // range k covers sweep blocks lo[k] .. hi[k] (hi[k] = lo[k-1] - 1)
  int lo[NSPLIT];
};
struct Bt2Task {
  SplitRanges R;
  const double* F2;
  const long* goff;
  double* Z;
  long ldz;
  const int* m_dev;
  int* done;
  DevStatusWord* st;
  int n, nblk, nstrip, m, b0, pad;  // b0: first workgroup of the task's share (informative)
};
Bt2Task bt2_task(const Sb2stLayout& L, const double* F2, const long* d_goff, double* Z,
                 long ldz, int m, const int* m_dev, int* iscratch, DevStatusWord* st);
size_t bt2_group_map_ints(int nt, const Bt2Task* tasks);
// algorithmic flops of Z <- Q2 Z for m columns
double bt2_flops(const Sb2stLayout& L, int m);
hipError_t bt2_group_apply(int nt, Bt2Task* tasks, std::vector<int>& hmap, Bt2Task* d_tasks,
                           int* d_map, hipStream_t s);
// Z (n x m) <- Q1 Z, the stage-1 panel reflectors (I - V T V^T), applied in
// groups of 16 panels, last group first.  Vst must hold zeros above each
// panel's first reflector row (bt1_zero_fill, before the reduction).
size_t bt1_scratch_doubles(int n, int B, int m);
hipError_t bt1_zero_fill(int n, int B, double* Vst, long ldv, hipStream_t s);
hipError_t bt1_apply(int n, int B, const double* Vst, long ldv, const double* T1, double* Z,
                     long ldz, int m, const int* m_dev, double* scratch, hipStream_t s);
// The same with the group products in FP32 on the matrix cores (the
// refined form): the groups' T are formed in FP64 from Vst and T1 (scratch
// as above), then applied with the FP32 reflectors V32 (ld ldv32) to the
// FP32 Z; scratch32: bt1_f32_scratch_floats(n, B, m) floats.
size_t bt1_f32_scratch_floats(int n, int B, int m);
hipError_t bt1_apply_f32(int n, int B, const double* Vst, long ldv, const float* V32,
                         long ldv32, const double* T1, float* Z, long ldz, int m,
                         const int* m_dev, double* scratch, float* scratch32, hipStream_t s);

// stedc.hip -- all eigenvalues (ascending) and eigenvectors of a symmetric
// tridiagonal by divide and conquer.  When m_dev is given, only the first
// *m_dev eigenvectors of the final merge are formed (the occupations are
// evaluated between the final eigenvalues and the final vectors through the
// callback).
struct StedcPlan;
// A plan's device arrays live in caller-provided device memory of
// stedc_plan_device_bytes(n) bytes (256-byte aligned, part of the solve's
// workspace); stedc_plan_upload copies its tables there on stream s (the
// plan's host tables stay alive with the plan).  A plan allocates and frees
// no device memory.
size_t stedc_plan_device_bytes(int n);
StedcPlan* stedc_plan_create_in(int n, void* dev);
hipError_t stedc_plan_upload(StedcPlan* p, hipStream_t s);
// Flops of the merge products of the last stedc_run on this plan (2 m n k
// per product, from the sizes the device wrote after deflation); reads the
// device descriptors, so the run's stream must have been synchronized.
double stedc_last_flops(const StedcPlan* p);
void stedc_plan_destroy(StedcPlan* p);
size_t stedc_scratch_doubles(int n);
size_t stedc_iscratch_ints(int n);
typedef hipError_t (*StedcEigvalHook)(void* ctx, const double* lam, hipStream_t s);
hipError_t stedc_run(StedcPlan* p, const double* d, const double* e, double* lam, double* Z,
                     long ldz, double* scratch, int* iscratch, const int* m_dev,
                     StedcEigvalHook hook, void* hook_ctx, DevStatusWord* st, hipStream_t s);

// herm.hip -- Hermitian pencils through the real embedding
// R(A) = [[Re A, -Im A], [Im A, Re A]] (2n x 2n).  A and X are interleaved
// complex (double2), column-major, leading dimensions in complex elements.
// herm_embed writes the lower triangle of R(A) from the lower triangle of A;
// herm_extract reads X = R[:n, :n] + i R[n:, :n]; herm_pair_eval averages the
// embedded pencil's eigenvalue pairs (2l, 2l + 1) into eval[l].
hipError_t herm_embed(int n, const void* A, long lda, double* R, long ldr, hipStream_t s);
hipError_t herm_extract(int n, const double* R, long ldr, void* X, long ldx, hipStream_t s);
hipError_t herm_pair_eval(int n, const double* lam2, double* eval, hipStream_t s);
// Eigenvectors: herm_extract_pairs reads X[:, l] = x + i y from real column 2l
// ([x; y]) for l < m; herm_jmul forms J Q = [-Q_y; Q_x] for k2 columns (J: the real form
// of multiplication by i); herm_combine forms X[:, a] = sum_j (x_j + i y_j) c[j, a]
// for a complex k2 x k coefficient matrix c (device, interleaved).
hipError_t herm_extract_pairs(int n, int m, const double* R, long ldr, void* X, long ldx,
                              hipStream_t s);
hipError_t herm_jmul(int n, int k2, const double* Q, long ldq, double* JQ, long ldj,
                     hipStream_t s);
hipError_t herm_combine(int n, int k2, int k, const double* Q, long ldq, const void* c, void* X,
                        long ldx, hipStream_t s);

// refine.hip -- eigenpair refinement of the refined form (Ogita-Aishima
// iterative refinement): steps on the first m columns of X (n x n, the
// eigenvectors of the symmetric A, lower triangle stored, within FP32
// rounding; X32 its FP32 copy, kept in step), every column taking part in
// the corrections, until the largest correction is at most tol or after
// max_steps.  lam receives the Rayleigh quotients (all n; the first m
// refined in every step); Y (n x n) is scratch; rec (device) and host_rec
// (pinned host) receive rec[2k] = delta and rec[2k+1] = max |e_ij| of step
// k; *steps_done the steps run (the stream is synchronized after each).
// scratch: refine_scratch_bytes(n, m).
size_t refine_scratch_bytes(int n, int m);
hipError_t refine_run(int n, int m, const double* A, long lda, double* X, long ldx, float* X32,
                      long ldx32, double* Y, long ldy, double* lam, int max_steps, double tol,
                      void* scratch, double* rec, double* host_rec, int* steps_done,
                      hipStream_t s);
