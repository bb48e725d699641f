/*
 * oracle.c -- plain FP64 CPU oracle for the interpolative decomposition (ID).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * GPU library.
 *
 * What it computes (Advani & O'Hagan, "Efficient Algorithms for Constructing
 * an Interpolative Decomposition"):
 *   - Section 2 (problem statement): A is m x n with m <= n; rank k.
 *   - Section 2.1: column-pivoted QR  A P = Q R  selects the k columns
 *     C = A P_k; Z minimises ||A - C Z||_F.  For the ID this least-squares
 *     solution is Z = [I  R11^{-1} R12] P^T, i.e. the triangular solves that
 *     Section 2.1 reduces the normal equations to (eq. final_eq), done here
 *     directly on R12 instead of through C^T A.
 *   - Section 4.1 (future work): the QR is stopped after k columns.
 *   - Definition 1: k columns of Z form the identity.
 *
 * The pivot rule is Businger-Golub: at every step take the remaining column
 * whose residual (the part of it orthogonal to the columns already chosen)
 * has the largest 2-norm.  Here that residual norm is recomputed exactly,
 * from scratch, at every step (no downdating), and a tie goes to the column
 * with the smallest original index.  Everything is unblocked Householder QR
 * with physical column swaps, in double precision, in the textbook order.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so
 * (OpenMP only splits independent columns; it changes no arithmetic.)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define COL(W, ld, j) ((W) + (size_t)(j) * (size_t)(ld))

/* Exact 2-norm of x[0:len] by plain summation of squares. */
static double norm2(const double *x, int64_t len) {
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += x[i] * x[i];
    return sqrt(s);
}

/*
 * oracle_cpqr: truncated Householder QR with Businger-Golub column pivoting.
 *
 *   W      in/out  m x n, column-major, leading dimension m.  On return its
 *                  first k_out rows hold R (upper trapezoidal, in pivoted
 *                  column order) and rows k_out.. of columns k_out.. hold the
 *                  trailing residual block R22.
 *   kmax           largest number of steps.
 *   stop_abs       tolerance mode: stop before step j when the residual
 *                  Frobenius norm sqrt(sum_{l>=j} nu_l^2) <= stop_abs
 *                  (pass a negative value to disable).
 *   forced/nforced the first nforced pivots are taken from forced[] (original
 *                  column indices) instead of the argmax (used to follow a
 *                  different but equally valid pivot choice).
 *   perm   out     n entries: perm[c] = original index of the column now at
 *                  position c.
 *   nu1, nu2, nuo  out (kmax each, may be NULL): per step, the largest and
 *                  second largest residual norm, and the original norm of the
 *                  chosen column.
 *   resid  out     kmax+1 entries (may be NULL): residual Frobenius norm
 *                  before each step (resid[k_out] is ||R22||_F at the end).
 * Returns k_out, the number of steps taken (k_out < kmax when the tolerance
 * was met or the largest residual norm became exactly zero).
 */
int oracle_cpqr(double *W, int64_t m, int64_t n, int kmax, double stop_abs,
                const int32_t *forced, int nforced, int32_t *perm,
                double *nu1, double *nu2, double *nuo, double *resid) {
    double *nu = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *orig = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    for (int64_t c = 0; c < n; ++c) perm[c] = (int32_t)c;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) orig[c] = norm2(COL(W, m, c), m);

    int64_t kcap = kmax;
    if (kcap > m) kcap = m;
    if (kcap > n) kcap = n;
    int j = 0;
    for (; j <= kcap; ++j) {
        /* residual norms of the remaining columns, rows j..m-1 */
#pragma omp parallel for schedule(static)
        for (int64_t c = j; c < n; ++c) nu[c] = norm2(COL(W, m, c) + j, m - j);
        double fro = 0.0;
        for (int64_t c = j; c < n; ++c) fro += nu[c] * nu[c];
        fro = sqrt(fro);
        if (resid) resid[j] = fro;
        if (j == kcap) break;
        if (stop_abs >= 0.0 && fro <= stop_abs) break;

        /* pivot: largest residual norm, smallest original index on ties */
        int64_t p = -1;
        if (j < nforced) {
            for (int64_t c = j; c < n; ++c)
                if (perm[c] == forced[j]) p = c;
        } else {
            for (int64_t c = j; c < n; ++c)
                if (p < 0 || nu[c] > nu[p] || (nu[c] == nu[p] && perm[c] < perm[p])) p = c;
        }
        if (p < 0) break;
        double second = 0.0;
        for (int64_t c = j; c < n; ++c)
            if (c != p && nu[c] > second) second = nu[c];
        if (nu1) nu1[j] = nu[p];
        if (nu2) nu2[j] = second;
        if (nuo) nuo[j] = orig[perm[p]];
        if (nu[p] == 0.0) break; /* rank(A) == j: nothing left to select */

        /* swap columns j and p */
        if (p != j) {
            double *a = COL(W, m, j), *b = COL(W, m, p);
            for (int64_t r = 0; r < m; ++r) { double t = a[r]; a[r] = b[r]; b[r] = t; }
            int32_t t = perm[j]; perm[j] = perm[p]; perm[p] = t;
        }

        /* Householder reflector H = I - tau v v^T with H x = beta e_1 */
        double *x = COL(W, m, j) + j;
        int64_t len = m - j;
        double alpha = norm2(x, len);
        double beta = x[0] >= 0.0 ? -alpha : alpha;
        double denom = x[0] - beta;
        double tau = (beta - x[0]) / beta;
        v[0] = 1.0;
        for (int64_t r = 1; r < len; ++r) v[r] = x[r] / denom;
        x[0] = beta;
        for (int64_t r = 1; r < len; ++r) x[r] = 0.0;

        /* apply H to every remaining column */
#pragma omp parallel for schedule(static)
        for (int64_t c = j + 1; c < n; ++c) {
            double *y = COL(W, m, c) + j;
            double s = 0.0;
            for (int64_t r = 0; r < len; ++r) s += v[r] * y[r];
            s *= tau;
            for (int64_t r = 0; r < len; ++r) y[r] -= s * v[r];
        }
    }
    free(nu);
    free(orig);
    free(v);
    return j;
}

/*
 * oracle_trsm: back substitution T = R11^{-1} R12 (Section 2.1, triangular
 * solves).  R is the k x n upper-trapezoidal block of the factorisation,
 * column-major with leading dimension ldr; T is k x (n-k), column-major,
 * leading dimension k.  Column c of T solves R11 t = R[:, k + c].
 */
void oracle_trsm(const double *R, int64_t ldr, int k, int64_t n, double *T) {
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n - k; ++c) {
        const double *b = R + (size_t)(k + c) * (size_t)ldr;
        double *t = T + (size_t)c * (size_t)k;
        for (int i = k - 1; i >= 0; --i) {
            double s = b[i];
            for (int q = i + 1; q < k; ++q) s -= R[i + (size_t)q * ldr] * t[q];
            t[i] = s / R[i + (size_t)i * ldr];
        }
    }
}

/*
 * oracle_id: the whole deterministic ID of an m x n matrix (m <= n assumed;
 * the caller transposes otherwise, following the dual-ID footnote of
 * Section 2).
 *
 *   A      in   m x n column-major, leading dimension lda (not modified).
 *   k      in   fixed rank (k > 0), or 0 for tolerance mode with eps.
 *   eps    in   tolerance mode: smallest k with ||R22||_F <= eps ||A||_F,
 *               capped at kmax.
 *   J      out  kmax entries: selected original column indices, in order.
 *   Z      out  kmax x n column-major (leading dimension kmax): Z[:, J[c]] is
 *               the c-th unit vector, the other columns hold T.
 *   R      out  kmax x n column-major, leading dimension kmax, may be NULL:
 *               the first k_out rows of R in ORIGINAL column order.
 *   nu1, nu2, nuo, resid: as in oracle_cpqr (may be NULL).
 * Returns k_out.
 */
int oracle_id(const double *A, int64_t m, int64_t n, int64_t lda, int k, double eps, int kmax,
              const int32_t *forced, int nforced, int32_t *J, double *Z, double *R,
              double *nu1, double *nu2, double *nuo, double *resid) {
    double *W = (double *)malloc(sizeof(double) * (size_t)m * (size_t)(n > 0 ? n : 1));
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t c = 0; c < n; ++c) memcpy(COL(W, m, c), A + (size_t)c * (size_t)lda, sizeof(double) * (size_t)m);

    double stop_abs = -1.0;
    int steps = k > 0 ? k : kmax;
    if (k <= 0) {
        double fro = 0.0;
        for (int64_t c = 0; c < n; ++c) {
            double t = norm2(COL(W, m, c), m);
            fro += t * t;
        }
        stop_abs = eps * sqrt(fro);
    }
    int kout = oracle_cpqr(W, m, n, steps, stop_abs, forced, nforced, perm, nu1, nu2, nuo, resid);

    /* R rows 0..kout-1 as a kout x n block with leading dimension m */
    double *T = (double *)malloc(sizeof(double) * (size_t)(kout > 0 ? kout : 1) * (size_t)(n - kout > 0 ? n - kout : 1));
    if (kout > 0) oracle_trsm(W, m, kout, n, T);

    int ldz = kmax;
    for (int64_t c = 0; c < n; ++c)
        for (int i = 0; i < ldz; ++i) Z[i + (size_t)c * ldz] = 0.0;
    for (int c = 0; c < kout; ++c) {
        J[c] = perm[c];
        Z[c + (size_t)perm[c] * ldz] = 1.0;
    }
    for (int c = kout; c < kmax; ++c) J[c] = -1;
    for (int64_t c = kout; c < n; ++c)
        for (int i = 0; i < kout; ++i) Z[i + (size_t)perm[c] * ldz] = T[i + (size_t)(c - kout) * kout];
    if (R) {
        for (int64_t c = 0; c < n; ++c)
            for (int i = 0; i < ldz; ++i)
                R[i + (size_t)perm[c] * ldz] = i < kout ? W[i + (size_t)c * m] : 0.0;
    }
    free(T);
    free(W);
    free(perm);
    return kout;
}

/*
 * oracle_matmul: C = A B in plain FP64 (A: m x p, B: p x n, all column-major,
 * leading dimensions lda, ldb, ldc).  Used for the sketch Y = Omega A of the
 * randomized ID and for residual checks.
 */
void oracle_matmul(const double *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc,
                   int64_t m, int64_t p, int64_t n) {
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        double *cc = C + (size_t)c * ldc;
        for (int64_t i = 0; i < m; ++i) cc[i] = 0.0;
        const double *bc = B + (size_t)c * ldb;
        for (int64_t q = 0; q < p; ++q) {
            double b = bc[q];
            const double *ac = A + (size_t)q * lda;
            for (int64_t i = 0; i < m; ++i) cc[i] += ac[i] * b;
        }
    }
}

/*
 * Thread count of the OpenMP loops above (timing only: the results do not
 * depend on it, every parallel loop writes disjoint columns).
 */
#include <omp.h>
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_threads(void) { return omp_get_max_threads(); }
