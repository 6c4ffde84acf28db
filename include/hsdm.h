/*
 * hsdm.h -- C ABI of libhsdm: the dense path from a Hamiltonian H and an
 * overlap S to eigenpairs and density matrices on one AMD Instinct MI355X
 * (gfx950), in FP64.
 *
 * The problem is the generalized eigenproblem  H C = S C eps  (Eq. (3) of the
 * ELSI 2.x paper, arXiv:1912.13403) with H symmetric and S symmetric positive
 * definite, followed by the density matrix  p_ij = sum_l f_l c_il c_jl
 * (Eq. (4)) and the energy-weighted density matrix
 * q_ij = sum_l eps_l f_l c_il c_jl (Eq. (17)), the occupations f_l and the
 * chemical potential coming from the eigenvalues and the electron count
 * (Sec. 2.6, normalization of Eq. (16) for one unit task).
 *
 * Conventions shared by every call
 *   - Matrices are column-major FP64 in DEVICE memory of the handle's device:
 *     element (i, j) of X with leading dimension ldx is X[i + j*ldx], and
 *     ldx >= n.  Vectors of length n are device arrays unless stated.
 *   - Only the LOWER triangle of H and S is read; inputs are never modified.
 *   - Outputs D, E are written in full (both triangles); eigenvectors are
 *     columns in ascending eigenvalue order, normalized so that C^T S C = I.
 *   - The caller owns every buffer passed in; the handle owns its workspace
 *     and the cached factor of S.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it in order; every call that returns a status other
 *     than an argument error synchronizes that stream before returning.
 *   - One handle must not be used by two host threads at once; different
 *     handles are independent.
 *   - Return value: HSDM_OK, a negative number -k if argument k (1-based,
 *     the handle counting as argument 1) is invalid, or a positive status
 *     below.  After a non-zero status the outputs are undefined.  The library
 *     never aborts.
 */
#ifndef HSDM_H
#define HSDM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsdm_ctx *hsdm_handle;

enum hsdm_status {
  HSDM_OK = 0,
  HSDM_NOT_SPD = 1,        /* S is not positive definite; hsdm_status_detail = failing column (1-based) */
  HSDM_NO_CONVERGE = 2,    /* an eigenvalue iteration did not converge */
  HSDM_MU_FAIL = 3,        /* chemical potential search failed (non-finite eigenvalues) */
  HSDM_DEVICE_ERROR = 4,   /* HIP error or out of device memory; see hsdm_last_error */
  HSDM_SYNC_TIMEOUT = 5    /* a bounded inter-workgroup wait ran out (device overloaded) */
};

/* Keys of hsdm_set_real / hsdm_set_int. */
enum hsdm_key {
  HSDM_KEY_FMAX = 1,       /* real: maximum occupation per state (2 spin-degenerate, 1 per spin channel); default 2 */
  HSDM_KEY_FCUT = 2,       /* real: states with f <= fcut * fmax get no eigenvector (f is below it); default 1e-16 */
  HSDM_KEY_DEG_TOL = 3,    /* real: kT = 0 degeneracy window; < 0 selects 1e-12 * ||H||_1 (default) */
  HSDM_KEY_TIMING = 4      /* int: 1 records per-phase times (hsdm_phase_times); 2 also times every
                              launch of the main kernels of a solve (hsdm_kernel_stat; multi-task
                              solves then keep every launch on the caller's stream, so that no
                              launch's time includes another's); 3 times only the kernels
                              launched once per solve (no event overhead on the many small
                              launches); 0 off (default) */
  , HSDM_KEY_STREAMS = 5   /* int: worker streams of the multi-task solves, 1 ... 8 (default 4);
                              they run side by side only as far as the HIP runtime gives the
                              process hardware queues (GPU_MAX_HW_QUEUES) */
  , HSDM_KEY_CONCURRENT = 7 /* int: 1 = this handle's solves may run at the same time as other
                              handles' solves on the same GPU (other host threads and streams,
                              e.g. the slots of a serving loop).  No workgroup of such a solve
                              then waits for another workgroup while other solves share the
                              device: the panel QR runs as one launch per column and the stage-2
                              back-transform as independent strips; a kernel whose workgroups
                              must all be resident (the bulge chasing, grouped panel QRs) waits
                              for the device to drain and runs with no other launch submitted
                              until it ends.  Results are bitwise those of a handle with the
                              key 0.  0 (default): for a handle that has the device to itself */
  , HSDM_KEY_N_STATES = 6  /* int: number of eigenvectors the eigenpair solves form, the lowest
                              ones (the paper's n_states: its dense runs compute only part of
                              the eigenvectors, Sec. 3); 0 or >= n: all (default 0).  C then
                              holds n_states columns; every eigenvalue is still returned */
  , HSDM_KEY_PRECISION = 8 /* int: arithmetic of hsdm_solve_ev_real, hsdm_solve_dm_real,
                              hsdm_solve_dm_complex (on its real embedding) and the multi-task
                              hsdm_solve_dm_batch and hsdm_solve_dm_group.  0 (default): FP64
                              throughout.  1: the
                              refined form -- the full -> band reduction's trailing updates and
                              the stage-1 back-transform in FP32 on the matrix cores, every
                              eigenvector formed, then at most HSDM_KEY_REFINE_STEPS steps of FP64
                              eigenpair refinement (Ogita-Aishima iterative refinement against
                              the FP64 standard-form matrix) of the wanted ones: the lowest
                              n_states for the eigenpair solve, the states occupied above the
                              cut (with a margin) for the density-matrix solve; Cholesky,
                              standard form, the tridiagonal eigensolve, occupations and D, E
                              stay FP64.  The refinement stops after the first step whose
                              largest correction is at most 1e-6 (the error left is of the
                              order of its square; a pair of eigenvalues too close to resolve in
                              a step counts with the correction it would need at that step's
                              separation), later steps correcting only the vectors still above
                              it.  In a multi-task solve every task's reduction, eigensolve
                              and refinement run one task after another on the caller's stream,
                              the wanted vectors chosen at the shared (batch) or own (group)
                              occupations of the unrefined eigenvalues, the occupations taken
                              again at the refined ones.  hsdm_solve_ev_complex and the
                              allocation-free solve always run the FP64 form */
  , HSDM_KEY_REFINE_STEPS = 9 /* int: most refinement steps of the refined form, 1 ... 8
                              (default 8) */
  , HSDM_KEY_GRAPH = 11    /* int: 1 = hsdm_solve_dm_real (FP64 form, timing off, not
                              concurrent, autotuner off) records its device work as a HIP graph
                              on the first call with a given set of buffers (H, S, D, E and
                              their leading dimensions), n, n_electrons, kT, settings and state
                              of the cached factor of S, and replays that graph on later such
                              calls -- the repeat-size solves of an SCF loop, which pass the
                              same buffers with new contents.  The graph runs on a stream of
                              the handle, ordered after the caller's stream and joined back into
                              it.  At most 4 graphs are kept per handle (least recently used
                              dropped); they are dropped when the workspace is reallocated or
                              the key is set to 0 (default) */
  , HSDM_KEY_AUTOTUNE = 10 /* int, process-wide (any handle sets it): 1 = the GEMM tile
                              autotuner is on -- the first product of each class not yet in the
                              tile table (element type, transposes, operand form, lower output,
                              bit lengths of m, n, k) runs the candidate tiles on its own
                              operands, C saved and restored around each run, and the fastest
                              enters the table; that solve is slower (it synchronizes and
                              allocates), later ones use the table.  Tiles never change a
                              result: every tile sums each element's products over k in the
                              same order.  0 (default): products use the table where it has
                              their class, else the built-in rule */
};

/* Create a handle bound to HIP device `device` (~ elsi_init, Sec. 2.1). */
int hsdm_init(hsdm_handle *h, int device);
/* Release the handle and its device workspace (~ elsi_finalize). */
int hsdm_finalize(hsdm_handle h);
/* Forget the cached factor of S (~ elsi_reinit, Sec. 2.7: a new geometry
 * brings a new overlap matrix; everything else is kept).  The factor is
 * cached by the CONTENT of S: its size, real or complex, and a 64-bit hash of
 * its lower triangle computed on the device at every call (one read of the
 * lower triangle and one synchronization of the stream).  A solve whose S
 * has the content of the cached one reuses the factor, whatever buffer holds
 * it; any other S is factored anew, so a freed buffer reused for another S
 * never finds a stale factor.  reinit drops the factor outright. */
int hsdm_reinit(hsdm_handle h);
/* Solver settings (~ the elsi_set_* routines of the API of Sec. 2.1, which
 * configure a handle between elsi_init and the solves).  hsdm_set_real takes
 * HSDM_KEY_FMAX, HSDM_KEY_FCUT, HSDM_KEY_DEG_TOL; hsdm_set_int takes
 * HSDM_KEY_TIMING, HSDM_KEY_STREAMS, HSDM_KEY_N_STATES, HSDM_KEY_CONCURRENT,
 * HSDM_KEY_PRECISION, HSDM_KEY_REFINE_STEPS, HSDM_KEY_AUTOTUNE, HSDM_KEY_GRAPH.
 * Returns HSDM_OK,
 * -1 (null handle), -2 (unknown key for this call) or -3 (value out of the
 * key's range; the setting is left unchanged).  Settings apply to the solves
 * that follow and are kept across hsdm_reinit. */
int hsdm_set_real(hsdm_handle h, int key, double value);
int hsdm_set_int(hsdm_handle h, int key, long value);

/* All eigenpairs of H C = S C eps (Eq. (3)).
 *   eval[n]        device, ascending eigenvalues (out), all n
 *   C[ldc * ns]    device, eigenvectors (out) of the lowest ns = n_states
 *                  eigenvalues (HSDM_KEY_N_STATES; all n by default),
 *                  C^T S C = I; only those ns vectors are formed
 * Path: Cholesky S = L L^T with L^{-1} (cached), A = L^{-1} H L^{-T},
 * full-to-band, band-to-tridiagonal, divide and conquer, back-transforms. */
int hsdm_solve_ev_real(hsdm_handle h, int n, const double *H, int ldh, const double *S, int lds,
                       double *eval, double *C, int ldc, void *stream);

/* Density matrices from H, S and the electron count (Eqs. (3), (4), (17),
 * Sec. 2.6).  kT > 0: Fermi-Dirac occupations with mu from bisection on
 * sum_l f_l = n_electrons; kT = 0: step occupations, degenerate states at the
 * Fermi level sharing the remainder equally.
 *   D[ldd * n]      device, density matrix (out)
 *   E[lde * n]      device, energy-weighted density matrix (out), nullable
 *   eval[n]         device, ascending eigenvalues (out), nullable
 *   band_energy     HOST, sum_l f_l eps_l = Tr(D H) (out), nullable
 *   mu              HOST, chemical potential (out), nullable
 * Only eigenvectors of states with f_l > fcut * fmax are formed. */
int hsdm_solve_dm_real(hsdm_handle h, int n, const double *H, int ldh, const double *S, int lds,
                       double n_electrons, double kT, double *D, int ldd, double *E, int lde,
                       double *eval, double *band_energy, double *mu, void *stream);

/* hsdm_solve_dm_real without any device allocation, for callers that cannot
 * allocate: code recorded into a HIP graph, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results and status codes as
 * hsdm_solve_dm_real, for n <= HSDM_NOALLOC_MAX_N (a larger n returns -2
 * with the reason in hsdm_last_error).  The workspace is a static device
 * array of the library (56 MiB, held by every GPU the library runs on until
 * the process ends), located at hsdm_init; the call makes no hipMalloc or
 * hipFree and no allocating library call.  Every call on one GPU shares that
 * array, from every handle: calls that overlap on one GPU race, so callers
 * must order them (one stream, or events).  The factor of S is never cached
 * (each call factors S), and per-launch timing is not recorded. */
#define HSDM_NOALLOC_MAX_N 512
int hsdm_solve_dm_real_noalloc(hsdm_handle h, int n, const double *H, int ldh, const double *S,
                               int lds, double n_electrons, double kT, double *D, int ldd,
                               double *E, int lde, double *eval, double *band_energy,
                               double *mu, void *stream);

/* Density matrices of a Hermitian pencil: the complex H_k, S_k of one unit
 * task of Eq. (13) (a k-point and spin channel), through the complex solver
 * interface of Sec. 2.1.  H, S, D and E are interleaved complex128 (real,
 * imaginary), column-major, leading dimensions counted in complex elements;
 * only the lower triangles of H and S are read, and the imaginary parts of
 * their diagonals are taken as zero.  Occupations as in hsdm_solve_dm_real
 * (f_max from HSDM_KEY_FMAX: 1 for one spin channel).
 *   D[ldd * n]      device, complex, Hermitian density matrix, both triangles (out)
 *   E[lde * n]      device, complex, energy-weighted density matrix (out), nullable
 *   eval[n]         device, ascending eigenvalues (out), nullable
 *   band_energy     HOST, sum_l f_l eps_l = Tr(D H) (out), nullable
 *   mu              HOST, chemical potential (out), nullable
 * Method: the real symmetric embedding [[Re A, -Im A], [Im A, Re A]] (size
 * 2n) of H and S has every eigenvalue of the pencil twice; it is solved by the
 * real path with one occupation per real eigenpair and 2 n_electrons, and D,
 * E are read from the left half of the real results (D = D_R[:n, :n] +
 * i D_R[n:, :n]).  Workspace: that of a real solve of size 2n plus
 * 4 (2n)^2 doubles, allocated on the first call of each size.  The factor of
 * S is cached by the content of S as in the real path.  Status codes as
 * hsdm_solve_dm_real. */
int hsdm_solve_dm_complex(hsdm_handle h, int n, const void *H, int ldh, const void *S, int lds,
                          double n_electrons, double kT, void *D, int ldd, void *E, int lde,
                          double *eval, double *band_energy, double *mu, void *stream);

/* Density matrices of nprob unit tasks that share one chemical potential:
 * the k-point x spin-channel problems of a periodic, spin-polarized system
 * (Eq. (13), Sec. 2.3), whose occupations are fixed together by the electron
 * count sum_p weight[p] sum_l f_pl = n_electrons (Eq. (16); a k-point's two
 * spin channels are two tasks with the same weight).  All tasks are real
 * (is_complex = 0: double) or all Hermitian (is_complex = 1: interleaved
 * complex128, as in hsdm_solve_dm_complex).  The arrays n, H, ldh, S, lds,
 * weight, D, ldd, E, lde are HOST arrays of nprob entries; H[p], S[p], D[p],
 * E[p] are device pointers.
 *   weight          nullable (all 1); entries > 0
 *   E               nullable, or entries nullable
 *   band_energy     HOST, sum_p weight[p] sum_l f_pl eps_pl (out), nullable
 *   mu              HOST, the shared chemical potential (out), nullable
 * kT > 0: Fermi-Dirac occupations, mu by bisection on the weighted count;
 * kT = 0: the Fermi level is the lowest eigenvalue of all tasks at which
 * f_max * sum weight reaches n_electrons, and the states of all tasks within
 * the degeneracy window of it share the remainder equally per unit weight.
 * Each task runs the path of the single solves (its factor of S cached by
 * the content of S[p], as in the single solves, in a task context owned by
 * the handle and kept until hsdm_finalize; hsdm_reinit forgets every task's
 * factor; tasks of one call with the same S[p], n[p], lds[p] share one
 * factorization); the tridiagonal
 * eigenvectors of all tasks are kept until the joint occupations are known,
 * then each task back-transforms its occupied vectors.  With several tasks
 * their independent phases run on the handle's worker streams, which start
 * after the work already queued on `stream` and which `stream` waits for
 * before it continues.  Status codes as the
 * single solves; argument k is reported as -k (n, H, ... arrays: -4 for a
 * missing array or a bad n[p], -5 ... -15 for the entry of problem p). */
int hsdm_solve_dm_batch(hsdm_handle h, int nprob, int is_complex, const int *n,
                        const void *const *H, const int *ldh, const void *const *S,
                        const int *lds, const double *weight, double n_electrons, double kT,
                        void *const *D, const int *ldd, void *const *E, const int *lde,
                        double *band_energy, double *mu, void *stream);

/* All eigenpairs of a Hermitian pencil H C = S C eps (Eq. (3) with the
 * complex H_k, S_k of Eq. (13); the complex eigensolver interface of
 * Sec. 2.1).  H, S, C interleaved complex128, column-major, leading
 * dimensions in complex elements; lower triangles of H and S read.
 *   eval[n]        device, ascending eigenvalues (out)
 *   C[ldc * ns]    device, complex eigenvectors (out), C^H S C = I, of the
 *                  lowest ns = n_states eigenvalues (HSDM_KEY_N_STATES; all n
 *                  by default; all 2n real vectors of the embedding are
 *                  still formed)
 * Method: the real embedding of size 2n (every eigenvalue twice); column l
 * of C is x + i y from the real eigenvector [x; y] of pair l.  For a complex
 * eigenvalue of multiplicity k (eigenvalues within 1e-10 max(1, |eps|)) the
 * 2k real eigenvectors are combined into k S-orthonormal complex ones by a
 * pivoted Cholesky of their complex Gram matrix (status +2 if that fails).
 * Workspace and factor cache as hsdm_solve_dm_complex. */
int hsdm_solve_ev_complex(hsdm_handle h, int n, const void *H, int ldh, const void *S, int lds,
                          double *eval, void *C, int ldc, void *stream);

/* Independent problems solved together (requests of a serving loop): real
 * and Hermitian tasks mixed (is_complex[p]), each with its own electron
 * count, kT and f_max (f_max nullable: the handle's), its own chemical
 * potential and band energy (HOST arrays mu[nprob], band_energy[nprob],
 * nullable).  Each task runs the path of the single solves; the bands of all
 * tasks are chased in shared cooperative launches.  Task contexts (workspace
 * and factor of S) are owned by the handle and picked by the content of S,
 * so a task whose S was factored in an earlier call (by any buffer holding
 * the same matrix) reuses the factor; otherwise the least recently used
 * context is taken.  Other
 * arguments, factor sharing within a call, the worker streams and status
 * codes as hsdm_solve_dm_batch (-3: a missing array or
 * a bad is_complex[p], -9: n_electrons[p], -10: kT[p], -11: f_max[p]). */
int hsdm_solve_dm_group(hsdm_handle h, int nprob, const int *is_complex, const int *n,
                        const void *const *H, const int *ldh, const void *const *S,
                        const int *lds, const double *n_electrons, const double *kT,
                        const double *f_max, void *const *D, const int *ldd, void *const *E,
                        const int *lde, double *band_energy, double *mu, void *stream);
/* Device bytes a task context of size n holds (its workspace; for Hermitian
 * tasks the real workspace of size 2n plus the embedding buffers). */
double hsdm_task_bytes(int n, int is_complex);
/* Device bytes held by the handle: its own workspace and its task contexts. */
double hsdm_workspace_bytes(hsdm_handle h);
/* Release least recently used task contexts (and with them their factors of
 * S) until the task contexts hold at most keep_bytes; synchronizes the
 * device first. */
int hsdm_release_tasks(hsdm_handle h, double keep_bytes);

/* ---- phase entry points (same conventions; used to test and compose) ---- */

/* S = L L^T and L^{-1}; L and Linv written in full (zeros above the diagonal). */
int hsdm_cholesky_inverse(hsdm_handle h, int n, const double *S, int lds, double *L, int ldl,
                          double *Linv, int ldli, void *stream);
/* Lower triangle of A = Linv H Linv^T (the standard form of Eq. (3)); the
 * strict upper triangle of A is left unspecified. */
int hsdm_standard_form(hsdm_handle h, int n, const double *H, int ldh, const double *Linv,
                       int ldli, double *A, int lda, void *stream);
/* Two-stage reduction of the symmetric A (lower triangle read) to the
 * tridiagonal (d[n], e[n-1]); if Q is non-null the orthogonal Q with
 * A = Q T Q^T is formed (Q[ldq * n]). */
int hsdm_tridiagonalize(hsdm_handle h, int n, const double *A, int lda, double *d, double *e,
                        double *Q, int ldq, void *stream);
/* Eigenpairs of the symmetric tridiagonal (d[n], e[n-1]) by divide and
 * conquer: w[n] ascending, Z[ldz * n]. */
int hsdm_tridiag_eigh(hsdm_handle h, int n, const double *d, const double *e, double *w,
                      double *Z, int ldz, void *stream);
/* Occupations f[n] (device) for ascending eval[n]; mu, band_energy and
 * n_occupied (#{f > fcut * fmax}) returned on the HOST (nullable). */
int hsdm_occupations(hsdm_handle h, int n, const double *eval, double n_electrons, double kT,
                     double deg_tol, double *f, double *mu, double *band_energy, int *n_occupied,
                     void *stream);
/* D = C diag(f) C^T and E = C diag(f eval) C^T from the first m columns of
 * C[ldc * m]; E nullable. */
int hsdm_density(hsdm_handle h, int n, int m, const double *C, int ldc, const double *f,
                 const double *eval, double *D, int ldd, double *E, int lde, void *stream);
/* FP64 GEMM on the matrix cores: C = alpha op(A) op(B) + beta C,
 * op(X) = X ('N') or X^T ('T'); op(A) is m x k, op(B) is k x n. */
int hsdm_dgemm(hsdm_handle h, char transa, char transb, int m, int n, int k, double alpha,
               const double *A, int lda, const double *B, int ldb, double beta, double *C,
               int ldc, void *stream);

/* ---- diagnostics ---- */
const char *hsdm_status_string(int status);
/* Text of the last error on this handle ("" if none). */
const char *hsdm_last_error(hsdm_handle h);
/* Detail of the last positive status (failing column for HSDM_NOT_SPD). */
int hsdm_status_detail(hsdm_handle h);
/* Per-phase times in ms of the last solve when HSDM_KEY_TIMING is on:
 * times[0..nphase-1] in the order of hsdm_phase_name(i); returns the number
 * of phases written (at most cap). */
int hsdm_phase_times(hsdm_handle h, double *times, int cap);
const char *hsdm_phase_name(int i);
/* How the last hsdm_solve_dm_real ran: 0 eagerly, 1 recorded as a graph
 * and run, 2 by replaying a recorded graph (HSDM_KEY_GRAPH); -1 null handle. */
int hsdm_last_graph(hsdm_handle h);
/* The GEMM tile table of the autotuner (HSDM_KEY_AUTOTUNE), process-wide:
 * hsdm_tune_entries returns its size; hsdm_tune_clear empties it;
 * hsdm_tune_save writes it to a text file (HSDM_OK, -1 path missing,
 * HSDM_DEVICE_ERROR if the file cannot be written); hsdm_tune_load merges
 * such a file into it and returns the number of entries read (-1 path
 * missing, -2 the file cannot be opened, -3 malformed: nothing merged).
 * Needs no GPU. */
int hsdm_tune_entries(void);
int hsdm_tune_clear(void);
int hsdm_tune_save(const char *path);
int hsdm_tune_load(const char *path);
/* Record of the refinement of the last real solve in the refined form
 * (HSDM_KEY_PRECISION = 1): returns the number of steps k (0 after an FP64
 * solve; -1 null handle, -3 cap < 0 or out missing) and writes, for the
 * first min(k, cap / 2) steps, out[2i] = delta (the separation below which
 * two eigenvalues are treated as one cluster) and out[2i + 1] = the largest
 * correction of step i (|e_ij|, or for a pair closer than delta the
 * correction it would need at separation delta). */
int hsdm_refine_history(hsdm_handle h, double *out, int cap);
/* Algorithmic FP64 flops of the phases of the last single solve when
 * HSDM_KEY_TIMING is on, in the order of hsdm_phase_name(i): the counts of
 * the method, not of this library's extra work -- Cholesky n^3/3 (0 when the
 * factor of S was cached), standard form n^3, full -> band 4n^3/3, band ->
 * tridiagonal 6 b n^2, divide and conquer the merge products at their sizes
 * after deflation, back-transforms 2n^2 m, 2n^2 m and n^2 m, D and E n^2 m
 * each (m: eigenvectors formed; the refined form transforms all n back and
 * its refinement phase counts 8 n^2 m_r per step on the m_r refined vectors
 * plus 2 n^2 (n - m_r) once; the other phases 0 in the FP64 form).
 * Multi-task solves write zeros.  Returns the number of phases written (at
 * most cap). */
int hsdm_phase_flops(hsdm_handle h, double *flops, int cap);

/* Per-kernel totals of the last solve when HSDM_KEY_TIMING is 2 or 3 (HIP events
 * recorded around each launch on the solve's stream; the solve synchronizes
 * before they are read).  hsdm_kernel_count returns the number of kernels
 * seen so far by this handle; hsdm_kernel_stat returns the name of kernel i
 * (NULL if i is out of range) and writes out[0] = total time in ms, out[1] =
 * algorithmic FP64 flops, out[2] = algorithmic bytes (0 where not defined),
 * out[3] = number of launches, all for the last solve. */
int hsdm_kernel_count(hsdm_handle h);
const char *hsdm_kernel_stat(hsdm_handle h, int i, double *out);
/* Restrict the per-launch timing of HSDM_KEY_TIMING 2 and 3 to the launches
 * of the kernel named `name` (as hsdm_kernel_stat names it; NULL or "" times
 * every kernel again), so that one kernel can be timed in every launch with
 * no events around the others.  Returns HSDM_OK or -1 (null handle). */
int hsdm_timing_kernel(hsdm_handle h, const char *name);
/* Measurement utility for the roofline's peaks, not a step of the method:
 * which = 0 runs `size` rounds (1 .. 1e7) of eight independent FP64 16x16x4
 * matrix-core products on every wavefront of two four-wavefront workgroups
 * per compute unit; which = 1 copies a buffer of `size` bytes (16 .. 64e9)
 * to another with one 16-byte load and store per thread and step.  Each is
 * launched twice on `stream` and the second launch is timed with HIP events:
 * out[0] = TFLOP/s (which = 0) or GB/s of bytes read plus written (1),
 * out[1] = ms, out[2] = flops or bytes.  The copy allocates and frees its two
 * buffers.  Returns HSDM_OK, -1 null handle, -2 which not 0 or 1, -3 size
 * out of range, -4 out missing, HSDM_DEVICE_ERROR (see hsdm_last_error). */
int hsdm_probe(hsdm_handle h, int which, double size, double *out, void *stream);
int hsdm_version(void);

#ifdef __cplusplus
}
#endif
#endif
