/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the dense H,S -> D path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  It may be used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark, and by nothing else.  It shares no code,
 * header, table or helper with the GPU path.
 *
 * What it computes (all references are to the ELSI 2.x paper, arXiv:1912.13403):
 *   - the generalized eigenproblem H C = S C eps of Eq. (3), all eigenpairs,
 *     eigenvectors S-orthonormal (C^T S C = I), eigenvalues ascending;
 *   - occupations f_l and the chemical potential mu from the eigenvalues and
 *     the electron count (Sec. 2.6, Fermi-Dirac; normalization as in Eq. (16)
 *     with a single unit task);
 *   - the density matrix p_ij = sum_l f_l c_il c_jl of Eq. (4);
 *   - the energy-weighted density matrix q_ij = sum_l eps_l f_l c_il c_jl of
 *     Eq. (17);
 *   - the band energy sum_l f_l eps_l.
 *
 * How: textbook dense steps, no blocking, no reordering of arithmetic beyond
 * running independent rows/columns on different OpenMP threads:
 *   1. Cholesky S = L L^T (the factorization the paper's benchmark section
 *      names as done once per geometry);
 *   2. standard form A = L^{-1} H L^{-T} by two forward substitutions
 *      (the "transformation to the standard form" of the benchmark section);
 *   3. Householder tridiagonalization A = Q T Q^T with Q accumulated;
 *   4. implicit QL iteration with a Wilkinson-type shift on T, rotations
 *      accumulated into Q;
 *   5. stable ascending sort of the eigenpairs;
 *   6. back-transformation C = L^{-T} Y by back substitution;
 *   7. occupations / mu, D, E, band energy.
 *
 * Storage: every matrix is column-major n x n with leading dimension n,
 * element (i,j) at a[i + j*n].  Only the lower triangle of H and S is read.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include <stdio.h>

#define AT(a, i, j, n) ((a)[(size_t)(j) * (size_t)(n) + (size_t)(i)])

/* With ORC_PROGRESS set in the environment, the whole solves report each
 * finished step on stderr (a long single-threaded run is then not silent).
 * No arithmetic depends on it. */
static void progress(const char *step, int n, int k) {
    static int on = -1;
    if (on < 0) on = getenv("ORC_PROGRESS") != NULL;
    if (!on) return;
    if (k >= 0)
        fprintf(stderr, "[oracle] n=%d %s %d\n", n, step, k);
    else
        fprintf(stderr, "[oracle] n=%d %s\n", n, step);
    fflush(stderr);
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* 1. Cholesky, column by column.  S is SPD as Eq. (3) requires of an overlap
 *    matrix; a non-positive pivot is reported as its 1-based column.
 *    L is written in full, with exact zeros above the diagonal.            */
int orc_cholesky(int n, const double *S, double *L) {
    /* row-major scratch so that every inner product runs over contiguous data */
    double *R = (double *)calloc((size_t)n * n, sizeof(double));
    if (!R) return -1;
    int info = 0;
    for (int j = 0; j < n && !info; j++) {
        const double *rj = R + (size_t)j * n;
        double s = AT(S, j, j, n);
        for (int k = 0; k < j; k++) s -= rj[k] * rj[k];
        if (!(s > 0.0)) { info = j + 1; break; }
        double ljj = sqrt(s);
        R[(size_t)j * n + j] = ljj;
#pragma omp parallel for schedule(static)
        for (int i = j + 1; i < n; i++) {
            const double *ri = R + (size_t)i * n;
            double t = AT(S, i, j, n);
            for (int k = 0; k < j; k++) t -= ri[k] * rj[k];
            R[(size_t)i * n + j] = t / ljj;
        }
    }
    for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) AT(L, i, j, n) = (i >= j) ? R[(size_t)i * n + j] : 0.0;
    free(R);
    return info;
}

/* Forward substitution L x = b for one column, L given row-major in R. */
static void forward_subst(int n, const double *R, const double *b, double *x) {
    for (int i = 0; i < n; i++) {
        const double *ri = R + (size_t)i * n;
        double t = b[i];
        for (int k = 0; k < i; k++) t -= ri[k] * x[k];
        x[i] = t / ri[i];
    }
}

/* ------------------------------------------------------------------------ */
/* 2. Standard form A = L^{-1} H L^{-T}.  X = L^{-1} H column by column, then
 *    A = L^{-1} X^T column by column (H symmetric, so X^T = H L^{-T}).
 *    A is symmetrized as (A + A^T)/2 at the end.                          */
void orc_standard_form(int n, const double *H, const double *L, double *A) {
    size_t nn = (size_t)n * n;
    double *R = (double *)malloc(nn * sizeof(double));   /* L row-major */
    double *Hf = (double *)malloc(nn * sizeof(double));  /* full symmetric H */
    double *X = (double *)malloc(nn * sizeof(double));
    double *Xt = (double *)malloc(nn * sizeof(double));
    for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
            R[(size_t)i * n + j] = AT(L, i, j, n);
            AT(Hf, i, j, n) = (i >= j) ? AT(H, i, j, n) : AT(H, j, i, n);
        }
#pragma omp parallel for schedule(dynamic, 8)
    for (int c = 0; c < n; c++) forward_subst(n, R, Hf + (size_t)c * n, X + (size_t)c * n);
    for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) AT(Xt, j, i, n) = AT(X, i, j, n);
#pragma omp parallel for schedule(dynamic, 8)
    for (int c = 0; c < n; c++) forward_subst(n, R, Xt + (size_t)c * n, A + (size_t)c * n);
    for (int j = 0; j < n; j++)
        for (int i = j + 1; i < n; i++) {
            double s = 0.5 * (AT(A, i, j, n) + AT(A, j, i, n));
            AT(A, i, j, n) = s;
            AT(A, j, i, n) = s;
        }
    free(R); free(Hf); free(X); free(Xt);
}

/* ------------------------------------------------------------------------ */
/* 3. Householder tridiagonalization of a full symmetric A (both triangles
 *    read).  Step k builds the reflector P_k = I - c v v^T that maps
 *    x = A[k+1:n, k] onto alpha e_1, alpha = -sign(x_0)|x|, and applies it on
 *    both sides of the trailing block:  p = c A v,  w = p - (c v^T p / 2) v,
 *    A <- A - v w^T - w v^T.  Q = P_0 P_1 ... P_{n-3} is accumulated from
 *    the last reflector backwards, so A = Q T Q^T.
 *    Output: d[0..n-1] diagonal, e[0..n-2] off-diagonal, Q n x n.          */
void orc_tridiagonalize(int n, const double *Ain, double *d, double *e, double *Q) {
    size_t nn = (size_t)n * n;
    double *W = (double *)malloc(nn * sizeof(double));
    double *V = (double *)calloc(nn, sizeof(double)); /* reflector k in column k */
    double *cf = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *p = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    memcpy(W, Ain, nn * sizeof(double));
    for (int k = 0; k + 2 < n; k++) {
        int r0 = k + 1;
        double x0 = AT(W, r0, k, n);
        double sig = 0.0;
        for (int i = r0 + 1; i < n; i++) sig += AT(W, i, k, n) * AT(W, i, k, n);
        if (sig == 0.0) { e[k] = x0; cf[k] = 0.0; continue; }
        double nrm = sqrt(x0 * x0 + sig);
        double alpha = (x0 > 0.0) ? -nrm : nrm;
        double *v = V + (size_t)k * n;
        v[r0] = x0 - alpha;
        for (int i = r0 + 1; i < n; i++) v[i] = AT(W, i, k, n);
        double c = 2.0 / (v[r0] * v[r0] + sig);
        cf[k] = c;
        e[k] = alpha;
        /* p_i = c * (A v)_i, using the symmetry of A: (A v)_i = A[:,i] . v */
#pragma omp parallel for schedule(static)
        for (int i = r0; i < n; i++) {
            const double *ai = W + (size_t)i * n;
            double t = 0.0;
            for (int j = r0; j < n; j++) t += ai[j] * v[j];
            p[i] = c * t;
        }
        double vp = 0.0;
        for (int i = r0; i < n; i++) vp += v[i] * p[i];
        double K = 0.5 * c * vp;
        for (int i = r0; i < n; i++) p[i] -= K * v[i]; /* p now holds w */
#pragma omp parallel for schedule(static)
        for (int j = r0; j < n; j++) {
            double *aj = W + (size_t)j * n;
            double vj = v[j], wj = p[j];
            for (int i = r0; i < n; i++) aj[i] -= v[i] * wj + p[i] * vj;
        }
    }
    for (int i = 0; i < n; i++) d[i] = AT(W, i, i, n);
    if (n >= 2) e[n - 2] = AT(W, n - 1, n - 2, n);
    /* Q = P_0 ... P_{n-3}: start from I and apply P_k from the left for
     * k = n-3 down to 0; P_k only touches rows/columns k+1.. of the product. */
    memset(Q, 0, nn * sizeof(double));
    for (int i = 0; i < n; i++) AT(Q, i, i, n) = 1.0;
    for (int k = n - 3; k >= 0; k--) {
        double c = cf[k];
        if (c == 0.0) continue;
        const double *v = V + (size_t)k * n;
        int r0 = k + 1;
#pragma omp parallel for schedule(static)
        for (int j = r0; j < n; j++) {
            double *qj = Q + (size_t)j * n;
            double t = 0.0;
            for (int i = r0; i < n; i++) t += v[i] * qj[i];
            t *= c;
            for (int i = r0; i < n; i++) qj[i] -= t * v[i];
        }
    }
    free(W); free(V); free(cf); free(p);
}

/* ------------------------------------------------------------------------ */
/* 4. Implicit QL on the symmetric tridiagonal (d, e), e[i] couples i and
 *    i+1.  For the unreduced block [l, m] the shift is the eigenvalue of the
 *    leading 2x2 closer to d[l]; one implicit step chases the rotation from
 *    the bottom (m) to the top (l).  The rotations of each step are applied
 *    to the columns of Z after the step (every row of Z sees them in the
 *    same order as a serial update would).  At most 30 steps per
 *    eigenvalue; returns 2 if that is exceeded.                            */
static void apply_rotations(int n, double *Z, const double *cs, const double *sn, int hi, int lo) {
    /* rotation i acts on columns (i, i+1); applied for i = hi down to lo.
     * Rows are independent: each thread takes blocks of 64 rows and applies
     * the rotations to them in the order above, so every element of Z sees
     * exactly the sequence of operations a serial update would apply. */
    const int RB = 64;
    const int nblk = (n + RB - 1) / RB;
#pragma omp parallel for schedule(static)
    for (int blk = 0; blk < nblk; blk++) {
        const int r0 = blk * RB, r1 = (r0 + RB < n) ? r0 + RB : n;
        for (int i = hi; i >= lo; i--) {
            double *zi = Z + (size_t)i * n, *zj = Z + (size_t)(i + 1) * n;
            const double c = cs[i], s = sn[i];
            for (int r = r0; r < r1; r++) {
                double a = zi[r], b = zj[r];
                zj[r] = s * a + c * b;
                zi[r] = c * a - s * b;
            }
        }
    }
}

int orc_tql(int n, double *d, const double *ein, double *Z) {
    double *e = (double *)calloc((size_t)n + 1, sizeof(double));
    double *cs = (double *)malloc(((size_t)n + 1) * sizeof(double));
    double *sn = (double *)malloc(((size_t)n + 1) * sizeof(double));
    for (int i = 0; i + 1 < n; i++) e[i] = ein[i];
    int status = 0;
    for (int l = 0; l < n && !status; l++) {
        if (l > 0 && l % 512 == 0) progress("QL: eigenvalues done", n, l);
        int steps = 0;
        for (;;) {
            int m = l;
            for (; m + 1 < n; m++) {
                double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= DBL_EPSILON * dd || fabs(e[m]) <= DBL_MIN) break;
            }
            if (m == l) break;
            if (++steps > 30) { status = 2; break; }
            /* shift: eigenvalue of [[d_l, e_l],[e_l, d_{l+1}]] nearest d_l;
             * g holds d_m - shift. */
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            int early = 0;
            for (; i >= l; i--) {
                double f = s * e[i];
                double b = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) { /* the block splits: recover and restart */
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = 1;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                cs[i] = c;
                sn[i] = s;
            }
            if (early) {
                if (m - 1 >= i + 1) apply_rotations(n, Z, cs, sn, m - 1, i + 1);
                continue;
            }
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
            apply_rotations(n, Z, cs, sn, m - 1, l);
        }
    }
    free(e); free(cs); free(sn);
    return status;
}

/* 5. Stable ascending sort of eigenpairs (ties keep the original order). */
static int cmp_pair(const void *a, const void *b) {
    const double *x = (const double *)a, *y = (const double *)b;
    if (x[0] < y[0]) return -1;
    if (x[0] > y[0]) return 1;
    return (x[1] < y[1]) ? -1 : (x[1] > y[1]);
}

void orc_sort_pairs(int n, double *d, double *Z) {
    double *key = (double *)malloc((size_t)2 * n * sizeof(double));
    double *T = (double *)malloc((size_t)n * n * sizeof(double));
    for (int i = 0; i < n; i++) { key[2 * i] = d[i]; key[2 * i + 1] = (double)i; }
    qsort(key, (size_t)n, 2 * sizeof(double), cmp_pair);
    memcpy(T, Z, (size_t)n * n * sizeof(double));
    for (int j = 0; j < n; j++) {
        int src = (int)key[2 * j + 1];
        d[j] = key[2 * j];
        memcpy(Z + (size_t)j * n, T + (size_t)src * n, (size_t)n * sizeof(double));
    }
    free(key); free(T);
}

/* 6. C = L^{-T} Y by back substitution, m columns. */
void orc_back_transform(int n, int m, const double *L, const double *Y, double *C) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int c = 0; c < m; c++) {
        const double *y = Y + (size_t)c * n;
        double *x = C + (size_t)c * n;
        for (int i = n - 1; i >= 0; i--) {
            const double *li = L + (size_t)i * n; /* column i of L */
            double t = y[i];
            for (int k = i + 1; k < n; k++) t -= li[k] * x[k];
            x[i] = t / li[i];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* 7a. Occupations and chemical potential (Sec. 2.6: given the electron
 *     count and the eigenvalues, the occupation numbers and mu follow).
 *
 *   kT > 0: Fermi-Dirac f(eps) = f_max / (1 + exp((eps - mu)/kT)), evaluated
 *           without overflow; mu by bisection on g(mu) = sum_l f_l - N_e
 *           (monotone increasing) inside [eps_min - 50kT - 1,
 *           eps_max + 50kT + 1], until lo and hi are adjacent doubles or 200
 *           halvings; mu is the midpoint.
 *   kT = 0: step occupations, the kT -> 0+ limit: states below the Fermi
 *           level get f_max; the states within deg_tol of the Fermi level
 *           share the remaining electrons equally; mu is the Fermi level
 *           when it is shared, else the midpoint of the highest occupied
 *           and lowest empty level.
 * eps must be ascending.  Returns 0, or 3 if the input is not finite.       */
static double fermi(double x, double fmax) {
    if (x >= 0.0) { double t = exp(-x); return fmax * t / (1.0 + t); }
    return fmax / (1.0 + exp(x));
}

static double occ_sum(int n, const double *eps, double fmax, double mu, double kT) {
    double s = 0.0;
    for (int l = 0; l < n; l++) s += fermi((eps[l] - mu) / kT, fmax);
    return s;
}

int orc_occupations(int n, const double *eps, double fmax, double ne, double kT,
                    double deg_tol, double *f, double *mu_out) {
    for (int l = 0; l < n; l++)
        if (!isfinite(eps[l])) return 3;
    if (kT > 0.0) {
        double lo = eps[0] - 50.0 * kT - 1.0, hi = eps[n - 1] + 50.0 * kT + 1.0;
        for (int it = 0; it < 200; it++) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (occ_sum(n, eps, fmax, mid, kT) < ne) lo = mid; else hi = mid;
        }
        double mu = 0.5 * (lo + hi);
        for (int l = 0; l < n; l++) f[l] = fermi((eps[l] - mu) / kT, fmax);
        *mu_out = mu;
        return 0;
    }
    for (int l = 0; l < n; l++) f[l] = 0.0;
    if (ne <= 0.0) { *mu_out = (n > 0) ? eps[0] : 0.0; return 0; }
    int nstates = (int)ceil(ne / fmax - 1e-12); /* states touched by N_e */
    if (nstates < 1) nstates = 1;
    if (nstates > n) nstates = n;
    double ef = eps[nstates - 1];
    int nb = 0, ng = 0;
    for (int l = 0; l < n; l++) {
        if (eps[l] < ef - deg_tol) nb++;
        else if (eps[l] <= ef + deg_tol) ng++;
    }
    double share = (ne - fmax * nb) / ng;
    int partial = share < fmax * (1.0 - 1e-15);
    for (int l = 0; l < n; l++) {
        if (eps[l] < ef - deg_tol) f[l] = fmax;
        else if (eps[l] <= ef + deg_tol) f[l] = share;
    }
    if (partial || nb + ng >= n) *mu_out = ef;
    else *mu_out = 0.5 * (eps[nb + ng - 1] + eps[nb + ng]);
    return 0;
}

/* 7b. D (Eq. 4) and E (Eq. 17) over the first m columns of C, all terms. */
void orc_density(int n, int m, const double *C, const double *f, const double *eps,
                 double *D, double *E) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; j++) {
        double *dj = D + (size_t)j * n;
        double *ej = E ? E + (size_t)j * n : NULL;
        for (int i = 0; i < n; i++) { dj[i] = 0.0; if (ej) ej[i] = 0.0; }
        for (int l = 0; l < m; l++) {
            const double *cl = C + (size_t)l * n;
            double a = f[l] * cl[j];
            double b = a * eps[l];
            for (int i = 0; i < n; i++) dj[i] += cl[i] * a;
            if (ej)
                for (int i = 0; i < n; i++) ej[i] += cl[i] * b;
        }
    }
}

/* Pairwise sum, for the band energy sum_l f_l eps_l. */
static double pairwise(const double *a, const double *b, int lo, int hi) {
    if (hi - lo <= 8) {
        double s = 0.0;
        for (int i = lo; i < hi; i++) s += a[i] * b[i];
        return s;
    }
    int mid = lo + (hi - lo) / 2;
    return pairwise(a, b, lo, mid) + pairwise(a, b, mid, hi);
}

double orc_band_energy(int n, const double *f, const double *eps) { return pairwise(f, eps, 0, n); }

/* ------------------------------------------------------------------------ */
/* Whole solves.  Return 0, 1 (S not positive definite, *info_col = column),
 * 2 (QL did not converge) or 3 (mu failed).                                */
static int eigen_pairs(int n, const double *H, const double *S, double *eval, double *C,
                       double *Lkeep, int *info_col) {
    size_t nn = (size_t)n * n;
    double *L = Lkeep ? Lkeep : (double *)malloc(nn * sizeof(double));
    double *A = (double *)malloc(nn * sizeof(double));
    double *Q = (double *)malloc(nn * sizeof(double));
    double *e = (double *)calloc((size_t)n + 1, sizeof(double));
    int st = orc_cholesky(n, S, L);
    if (st) { if (info_col) *info_col = st; st = 1; goto done; }
    progress("Cholesky done", n, -1);
    orc_standard_form(n, H, L, A);
    progress("standard form done", n, -1);
    orc_tridiagonalize(n, A, eval, e, Q);
    progress("tridiagonalization done", n, -1);
    st = orc_tql(n, eval, e, Q);
    if (st) goto done;
    progress("QL done", n, -1);
    orc_sort_pairs(n, eval, Q);
    orc_back_transform(n, n, L, Q, C);
    progress("back-transform done", n, -1);
done:
    if (!Lkeep) free(L);
    free(A); free(Q); free(e);
    return st;
}

int orc_solve_ev(int n, const double *H, const double *S, double *eval, double *C, int *info_col) {
    return eigen_pairs(n, H, S, eval, C, NULL, info_col);
}

int orc_solve_dm(int n, const double *H, const double *S, double fmax, double ne, double kT,
                 double deg_tol, double *eval, double *C, double *f, double *D, double *E,
                 double *mu, double *band_energy, int *info_col) {
    int st = eigen_pairs(n, H, S, eval, C, NULL, info_col);
    if (st) return st;
    st = orc_occupations(n, eval, fmax, ne, kT, deg_tol, f, mu);
    if (st) return st;
    orc_density(n, n, C, f, eval, D, E);
    *band_energy = orc_band_energy(n, f, eval);
    return 0;
}
