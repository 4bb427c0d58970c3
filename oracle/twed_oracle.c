/*
 * twed_oracle.c -- plain FP64 CPU Time Warp Edit Distance.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP library.
 *
 * What it computes (the plain definition, written out):
 *
 *   Section "Time Warp Edit Distance" (sequential steps 1-6) together with the
 *   cost terms of Marteau (2009) to which that section defers for the
 *   stiffness nu and the deletion penalty lambda:
 *
 *     A' and B' are the series padded with a zero point at index 0 (the
 *     footnotes of steps 1, 2 and 5a take out-of-range samples as zero
 *     vectors); timestamps are padded with 0 in the same way.
 *
 *     delta(x, y)  = ( sum_k |x_k - y_k|^p )^(1/p)      (Lp point distance,
 *                    with the root, section "cuTWED Implementation Remarks")
 *     del_A(i)     = delta(A'_i, A'_{i-1}) + nu*|TA'_i - TA'_{i-1}| + lambda
 *     del_B(j)     = delta(B'_j, B'_{j-1}) + nu*|TB'_j - TB'_{j-1}| + lambda
 *     mat(i, j)    = (delta(A'_i, B'_j) + delta(A'_{i-1}, B'_{j-1}))
 *                    + nu*(|TA'_i - TB'_j| + |TA'_{i-1} - TB'_{j-1}|)
 *
 *     DP[0][0] = 0, DP[i][0] = DP[0][j] = +inf                    (step 3)
 *     DP[i][j] = min(DP[i-1][j] + del_A(i),                         (step 5)
 *                    DP[i][j-1] + del_B(j),
 *                    DP[i-1][j-1] + mat(i, j))
 *     TWED     = DP[nA][nB]                                         (step 6)
 *
 * Readings taken where the printed formulas are garbled:
 *   - the match term compares sample values (not consecutive differences),
 *     and includes the point cost of the cell;
 *   - the time term of the match pairs TA with TB at the column index;
 *   - nu multiplies every time term, lambda is added to deletions only;
 *   - the 1/p root is taken; in one dimension every p gives |x - y|
 *     mathematically, and the code below still evaluates the general form.
 *
 * Compiled with -O2 -ffp-contract=off: every operation rounds exactly as
 * written, in the association shown above.
 *
 * Optional planted mistakes (ORACLE_MUTANT=k) exist only so that the test
 * suite can show that its pins detect each of them; the normal build defines
 * none.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

/* Lp distance between two points of `dim` components. */
static double point_dist(const double *x, const double *y, int dim, double p)
{
#if ORACLE_MUTANT == 3
    /* planted: no 1/p root */
    double s = 0.0;
    for (int k = 0; k < dim; k++) s += pow(fabs(x[k] - y[k]), p);
    return s;
#else
    double s = 0.0;
    if (p == 1.0) {
        for (int k = 0; k < dim; k++) s += fabs(x[k] - y[k]);
        return s;
    }
    if (p == 2.0) {
        for (int k = 0; k < dim; k++) {
            double d = x[k] - y[k];
            s += d * d;
        }
        return sqrt(s);
    }
    for (int k = 0; k < dim; k++) s += pow(fabs(x[k] - y[k]), p);
    return pow(s, 1.0 / p);
#endif
}

/* Zero-padded copy: out[0] = 0-vector, out[i] = in[i-1] for i = 1..n. */
static double *pad_points(const double *in, int64_t n, int dim)
{
    double *out = (double *)calloc((size_t)(n + 1) * (size_t)dim, sizeof(double));
    if (!out) return NULL;
#if ORACLE_MUTANT == 6
    /* planted: the pad repeats the first sample instead of the zero vector */
    memcpy(out, in, (size_t)dim * sizeof(double));
#endif
    memcpy(out + dim, in, (size_t)n * (size_t)dim * sizeof(double));
    return out;
}

static double *pad_times(const double *in, int64_t n)
{
    double *out = (double *)calloc((size_t)(n + 1), sizeof(double));
    if (!out) return NULL;
    memcpy(out + 1, in, (size_t)n * sizeof(double));
    return out;
}

typedef struct {
    const double *Ap, *TAp, *Bp, *TBp; /* padded, index 0 is the pad */
    int64_t nA, nB;
    int dim;
    double nu, lambda, p;
} problem;

static double del_cost(const double *Xp, const double *TXp, int64_t i, const problem *pr)
{
    double d = point_dist(Xp + i * pr->dim, Xp + (i - 1) * pr->dim, pr->dim, pr->p);
#if ORACLE_MUTANT == 5
    /* planted: nu left out of the deletion cost */
    return d + fabs(TXp[i] - TXp[i - 1]) + pr->lambda;
#else
    return d + pr->nu * fabs(TXp[i] - TXp[i - 1]) + pr->lambda;
#endif
}

static double mat_cost(int64_t i, int64_t j, const problem *pr)
{
    const int dim = pr->dim;
    double d1 = point_dist(pr->Ap + i * dim, pr->Bp + j * dim, dim, pr->p);
#if ORACLE_MUTANT == 1
    /* planted: the lagged point term of the match is dropped */
    double d2 = 0.0;
#else
    double d2 = point_dist(pr->Ap + (i - 1) * dim, pr->Bp + (j - 1) * dim, dim, pr->p);
#endif
#if ORACLE_MUTANT == 2
    /* planted: TB indexed by the row (the printed typo) */
    int64_t jt = i < pr->nB ? i : pr->nB;
    double t1 = fabs(pr->TAp[i] - pr->TBp[jt]);
    double t2 = fabs(pr->TAp[i - 1] - pr->TBp[jt - 1]);
#else
    double t1 = fabs(pr->TAp[i] - pr->TBp[j]);
    double t2 = fabs(pr->TAp[i - 1] - pr->TBp[j - 1]);
#endif
    double m = (d1 + d2) + pr->nu * (t1 + t2);
#if ORACLE_MUTANT == 4
    /* planted: the deletion penalty also charged on a match */
    m = m + pr->lambda;
#endif
    return m;
}

static double min3(double a, double b, double c)
{
    double m = a < b ? a : b;
    return m < c ? m : c;
}

/* One DP cell from its three neighbours (step 5 of the sequential algorithm). */
static double cell(double up, double left, double diag, int64_t i, int64_t j,
                   const double *delA, const double *delB, const problem *pr)
{
#if ORACLE_MUTANT == 7
    /* planted: the two deletion costs swapped */
    return min3(up + delB[j], left + delA[i], diag + mat_cost(i, j, pr));
#else
    return min3(up + delA[i], left + delB[j], diag + mat_cost(i, j, pr));
#endif
}

static double boundary_value(void)
{
#if ORACLE_MUTANT == 8
    /* planted: boundary row and column set to 0 instead of +inf */
    return 0.0;
#else
    return INFINITY;
#endif
}

/* Fills padded copies and the deletion-cost arrays; returns 0 on success. */
static int setup(const double *A, const double *TA, int64_t nA, const double *B,
                 const double *TB, int64_t nB, int dim, double nu, double lambda,
                 double p, problem *pr, double **bufs, double **delA, double **delB)
{
    double *Ap = pad_points(A, nA, dim), *TAp = pad_times(TA, nA);
    double *Bp = pad_points(B, nB, dim), *TBp = pad_times(TB, nB);
    double *dA = (double *)calloc((size_t)(nA + 1), sizeof(double));
    double *dB = (double *)calloc((size_t)(nB + 1), sizeof(double));
    bufs[0] = Ap; bufs[1] = TAp; bufs[2] = Bp; bufs[3] = TBp;
    *delA = dA; *delB = dB;
    if (!Ap || !TAp || !Bp || !TBp || !dA || !dB) return -1;
    pr->Ap = Ap; pr->TAp = TAp; pr->Bp = Bp; pr->TBp = TBp;
    pr->nA = nA; pr->nB = nB; pr->dim = dim;
    pr->nu = nu; pr->lambda = lambda; pr->p = p;
    for (int64_t i = 1; i <= nA; i++) dA[i] = del_cost(Ap, TAp, i, pr);
    for (int64_t j = 1; j <= nB; j++) dB[j] = del_cost(Bp, TBp, j, pr);
    return 0;
}

static void release(double **bufs, double *delA, double *delB)
{
    for (int k = 0; k < 4; k++) free(bufs[k]);
    free(delA);
    free(delB);
}

/*
 * Full (nA+1) x (nB+1) matrix, row-major double loop (steps 3-6).
 * If DP is non-NULL it receives every cell, row-major, row stride nB+1.
 * Returns DP[nA][nB], or NAN on bad arguments / allocation failure.
 */
double twed_oracle_matrix(const double *A, const double *TA, int64_t nA,
                          const double *B, const double *TB, int64_t nB,
                          int32_t dim, double nu, double lambda, double p,
                          double *DP)
{
    if (nA < 1 || nB < 1 || dim < 1) return NAN;
    problem pr;
    double *bufs[4] = {0}, *delA = NULL, *delB = NULL;
    if (setup(A, TA, nA, B, TB, nB, dim, nu, lambda, p, &pr, bufs, &delA, &delB)) {
        release(bufs, delA, delB);
        return NAN;
    }
    const int64_t W = nB + 1;
    double *M = DP;
    if (!M) M = (double *)malloc((size_t)(nA + 1) * (size_t)W * sizeof(double));
    if (!M) {
        release(bufs, delA, delB);
        return NAN;
    }
    M[0] = 0.0;
    for (int64_t j = 1; j <= nB; j++) M[j] = boundary_value();
    for (int64_t i = 1; i <= nA; i++) M[i * W] = boundary_value();
    for (int64_t i = 1; i <= nA; i++)
        for (int64_t j = 1; j <= nB; j++)
            M[i * W + j] = cell(M[(i - 1) * W + j], M[i * W + j - 1],
                                M[(i - 1) * W + j - 1], i, j, delA, delB, &pr);
    double r = M[nA * W + nB];
    if (M != DP) free(M);
    release(bufs, delA, delB);
    return r;
}

/*
 * The same cells, in the same order, keeping two rows only (for problems
 * whose full matrix does not fit in memory).  Bitwise equal to
 * twed_oracle_matrix: each cell is evaluated by the same code from the same
 * operands.
 */
double twed_oracle_rows(const double *A, const double *TA, int64_t nA,
                        const double *B, const double *TB, int64_t nB,
                        int32_t dim, double nu, double lambda, double p)
{
    if (nA < 1 || nB < 1 || dim < 1) return NAN;
    problem pr;
    double *bufs[4] = {0}, *delA = NULL, *delB = NULL;
    if (setup(A, TA, nA, B, TB, nB, dim, nu, lambda, p, &pr, bufs, &delA, &delB)) {
        release(bufs, delA, delB);
        return NAN;
    }
    double *prev = (double *)malloc((size_t)(nB + 1) * sizeof(double));
    double *cur = (double *)malloc((size_t)(nB + 1) * sizeof(double));
    if (!prev || !cur) {
        free(prev); free(cur);
        release(bufs, delA, delB);
        return NAN;
    }
    prev[0] = 0.0;
    for (int64_t j = 1; j <= nB; j++) prev[j] = boundary_value();
    for (int64_t i = 1; i <= nA; i++) {
        cur[0] = boundary_value();
        for (int64_t j = 1; j <= nB; j++)
            cur[j] = cell(prev[j], cur[j - 1], prev[j - 1], i, j, delA, delB, &pr);
        double *t = prev; prev = cur; cur = t;
    }
    double r = prev[nB];
    free(prev); free(cur);
    release(bufs, delA, delB);
    return r;
}

/* ---- band state and alignment path ----------------------------------------- */

/*
 * Point cost of cell (i, j): delta(A'_i, B'_j) + nu*|TA'_i - TB'_j|.  A match
 * cost is the sum of two of them, mat(i, j) = e(i, j) + e(i-1, j-1) (up to
 * the order of the additions).
 */
static double point_cost(int64_t i, int64_t j, const problem *pr)
{
    const int dim = pr->dim;
    return point_dist(pr->Ap + i * dim, pr->Bp + j * dim, dim, pr->p) +
           pr->nu * fabs(pr->TAp[i] - pr->TBp[j]);
}

/*
 * The full DP matrix and, beside it, X[i][j] = DP[i][j] + e(i, j): the
 * quantity a row of the band must carry so that the match into (i+1, j+1)
 * can be formed from DP[i][j] without the samples of row i (the state that a
 * sweep resumed below row i, or right of column j, starts from; section
 * "Improved Time Warp Edit Distance", the band holds the whole state).
 * DP and X are row-major with row stride nB+1.  Returns DP[nA][nB].
 */
double twed_oracle_matrix_x(const double *A, const double *TA, int64_t nA,
                            const double *B, const double *TB, int64_t nB,
                            int32_t dim, double nu, double lambda, double p,
                            double *DP, double *X)
{
    if (nA < 1 || nB < 1 || dim < 1 || !DP || !X) return NAN;
    double r = twed_oracle_matrix(A, TA, nA, B, TB, nB, dim, nu, lambda, p, DP);
    problem pr;
    double *bufs[4] = {0}, *delA = NULL, *delB = NULL;
    if (setup(A, TA, nA, B, TB, nB, dim, nu, lambda, p, &pr, bufs, &delA, &delB)) {
        release(bufs, delA, delB);
        return NAN;
    }
    const int64_t W = nB + 1;
    for (int64_t i = 0; i <= nA; i++)
        for (int64_t j = 0; j <= nB; j++)
            X[i * W + j] = DP[i * W + j] + point_cost(i, j, &pr);
    release(bufs, delA, delB);
    return r;
}

/*
 * One optimal alignment path, read back from (nA, nB) to (0, 0) over the
 * full matrix: at each cell the move whose candidate (the three terms of
 * step 5) is the minimum, preferring the match, then the deletion in A (from
 * the cell above), then the deletion in B (from the cell on the left).
 * Writes the cells from (0, 0) to (nA, nB) as (i, j) pairs into path
 * (capacity nA + nB + 1 pairs) and returns their number, or -1 if the path
 * cannot be followed (non-finite distance, allocation failure).
 */
int64_t twed_oracle_path(const double *A, const double *TA, int64_t nA,
                         const double *B, const double *TB, int64_t nB,
                         int32_t dim, double nu, double lambda, double p,
                         int64_t *path)
{
    if (nA < 1 || nB < 1 || dim < 1 || !path) return -1;
    const int64_t W = nB + 1;
    double *M = (double *)malloc((size_t)(nA + 1) * (size_t)W * sizeof(double));
    if (!M) return -1;
    double r = twed_oracle_matrix(A, TA, nA, B, TB, nB, dim, nu, lambda, p, M);
    problem pr;
    double *bufs[4] = {0}, *delA = NULL, *delB = NULL;
    if (!isfinite(r) || setup(A, TA, nA, B, TB, nB, dim, nu, lambda, p, &pr, bufs, &delA, &delB)) {
        release(bufs, delA, delB);
        free(M);
        return -1;
    }
    int64_t i = nA, j = nB, n = 0;
    const int64_t cap = nA + nB + 1;
    for (;;) {
        path[2 * n] = i;
        path[2 * n + 1] = j;
        n++;
        if (i == 0 && j == 0) break;
        if (i == 0 || j == 0 || n >= cap) {
            n = -1;
            break;
        }
        const double cm = M[(i - 1) * W + j - 1] + mat_cost(i, j, &pr);
        const double cu = M[(i - 1) * W + j] + delA[i];
        const double cl = M[i * W + j - 1] + delB[j];
        if (cm <= cu && cm <= cl) {
            i--;
            j--;
        } else if (cu <= cl) {
            i--;
        } else {
            j--;
        }
    }
    if (n > 0) {
        /* reverse into (0, 0) .. (nA, nB) order */
        for (int64_t a = 0, b = n - 1; a < b; a++, b--) {
            int64_t ti = path[2 * a], tj = path[2 * a + 1];
            path[2 * a] = path[2 * b];
            path[2 * a + 1] = path[2 * b + 1];
            path[2 * b] = ti;
            path[2 * b + 1] = tj;
        }
    }
    release(bufs, delA, delB);
    free(M);
    return n;
}

/*
 * Cost of a given path: the sum, from (0, 0) forwards, of the cost of each
 * step (mat(i, j) into (i, j) for a diagonal step, del_A(i) for a step down,
 * del_B(j) for a step right).  Returns NAN if the cells do not form an
 * admissible path from (0, 0) to (nA, nB) (steps other than those three, or
 * a cell on row 0 / column 0 other than (0, 0)).
 */
double twed_oracle_path_cost(const double *A, const double *TA, int64_t nA,
                             const double *B, const double *TB, int64_t nB,
                             int32_t dim, double nu, double lambda, double p,
                             const int64_t *path, int64_t len)
{
    if (nA < 1 || nB < 1 || dim < 1 || !path || len < 2) return NAN;
    problem pr;
    double *bufs[4] = {0}, *delA = NULL, *delB = NULL;
    if (setup(A, TA, nA, B, TB, nB, dim, nu, lambda, p, &pr, bufs, &delA, &delB)) {
        release(bufs, delA, delB);
        return NAN;
    }
    double cost = 0.0;
    int ok = path[0] == 0 && path[1] == 0 && path[2 * (len - 1)] == nA && path[2 * (len - 1) + 1] == nB;
    for (int64_t k = 1; ok && k < len; k++) {
        const int64_t i0 = path[2 * (k - 1)], j0 = path[2 * (k - 1) + 1];
        const int64_t i = path[2 * k], j = path[2 * k + 1];
        if (i < 1 || j < 1 || i > nA || j > nB) ok = 0;
        else if (i == i0 + 1 && j == j0 + 1) cost = cost + mat_cost(i, j, &pr);
        else if (i == i0 + 1 && j == j0) cost = cost + delA[i];
        else if (i == i0 && j == j0 + 1) cost = cost + delB[j];
        else ok = 0;
    }
    release(bufs, delA, delB);
    return ok ? cost : NAN;
}

/* ---- sibling dynamic programs -----------------------------------------------
 *
 * Section "Generalized Dynamic Programming Extensions" (its "Direct
 * Extension: LCS") notes that other programs whose cells need only the cells
 * above, to the left and diagonally above-left can be swept the same way.
 * Their plain definitions, two rows of memory each:
 *
 *   DTW   D[0][0] = 0, D[i][0] = D[0][j] = +inf,
 *         D[i][j] = delta(A_i, B_j) + min(D[i-1][j], D[i][j-1], D[i-1][j-1])
 *   edit  E[i][0] = i, E[0][j] = j,
 *         E[i][j] = min(E[i-1][j] + 1, E[i][j-1] + 1, E[i-1][j-1] + [A_i != B_j])
 *   LCS   L[i][0] = L[0][j] = 0,
 *         L[i][j] = A_i == B_j ? L[i-1][j-1] + 1 : max(L[i-1][j], L[i][j-1])
 *
 * (samples 1-based as in the TWED definition; edit and LCS compare 1-D
 * samples for equality).
 */
double twed_oracle_dtw(const double *A, int64_t nA, const double *B, int64_t nB, int32_t dim, double p)
{
    if (nA < 1 || nB < 1 || dim < 1) return NAN;
    double *prev = (double *)malloc((size_t)(nB + 1) * sizeof(double));
    double *cur = (double *)malloc((size_t)(nB + 1) * sizeof(double));
    if (!prev || !cur) {
        free(prev); free(cur);
        return NAN;
    }
    prev[0] = 0.0;
    for (int64_t j = 1; j <= nB; j++) prev[j] = INFINITY;
    for (int64_t i = 1; i <= nA; i++) {
        cur[0] = INFINITY;
        for (int64_t j = 1; j <= nB; j++) {
            const double d = point_dist(A + (i - 1) * dim, B + (j - 1) * dim, dim, p);
            cur[j] = d + min3(prev[j], cur[j - 1], prev[j - 1]);
        }
        double *t = prev; prev = cur; cur = t;
    }
    double r = prev[nB];
    free(prev); free(cur);
    return r;
}

int64_t twed_oracle_edit(const double *A, int64_t nA, const double *B, int64_t nB)
{
    if (nA < 1 || nB < 1) return -1;
    int64_t *prev = (int64_t *)malloc((size_t)(nB + 1) * sizeof(int64_t));
    int64_t *cur = (int64_t *)malloc((size_t)(nB + 1) * sizeof(int64_t));
    if (!prev || !cur) {
        free(prev); free(cur);
        return -1;
    }
    for (int64_t j = 0; j <= nB; j++) prev[j] = j;
    for (int64_t i = 1; i <= nA; i++) {
        cur[0] = i;
        for (int64_t j = 1; j <= nB; j++) {
            int64_t v = prev[j] + 1;
            if (cur[j - 1] + 1 < v) v = cur[j - 1] + 1;
            const int64_t m = prev[j - 1] + (A[i - 1] != B[j - 1]);
            if (m < v) v = m;
            cur[j] = v;
        }
        int64_t *t = prev; prev = cur; cur = t;
    }
    int64_t r = prev[nB];
    free(prev); free(cur);
    return r;
}

int64_t twed_oracle_lcs(const double *A, int64_t nA, const double *B, int64_t nB)
{
    if (nA < 1 || nB < 1) return -1;
    int64_t *prev = (int64_t *)calloc((size_t)(nB + 1), sizeof(int64_t));
    int64_t *cur = (int64_t *)calloc((size_t)(nB + 1), sizeof(int64_t));
    if (!prev || !cur) {
        free(prev); free(cur);
        return -1;
    }
    for (int64_t i = 1; i <= nA; i++) {
        cur[0] = 0;
        for (int64_t j = 1; j <= nB; j++) {
            if (A[i - 1] == B[j - 1]) cur[j] = prev[j - 1] + 1;
            else cur[j] = prev[j] > cur[j - 1] ? prev[j] : cur[j - 1];
        }
        int64_t *t = prev; prev = cur; cur = t;
    }
    int64_t r = prev[nB];
    free(prev); free(cur);
    return r;
}

/* ---- batches: independent pairs spread over threads ---------------------- */

typedef struct {
    const double *X, *TX, *Y, *TY;
    const int64_t *offX, *offY, *pairs;
    int64_t nPairs;
    int dim;
    double nu, lambda, p;
    double *D;
    int64_t next; /* shared work counter */
    pthread_mutex_t lock;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *job = (batch_job *)arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int64_t k = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (k >= job->nPairs) break;
        int64_t i = job->pairs[2 * k], j = job->pairs[2 * k + 1];
        int64_t a0 = job->offX[i], a1 = job->offX[i + 1];
        int64_t b0 = job->offY[j], b1 = job->offY[j + 1];
        job->D[k] = twed_oracle_rows(job->X + a0 * job->dim, job->TX + a0, a1 - a0,
                                     job->Y + b0 * job->dim, job->TY + b0, b1 - b0,
                                     job->dim, job->nu, job->lambda, job->p);
    }
    return NULL;
}

/*
 * TWED for an explicit list of (i, j) pairs between two packed collections
 * (values X: sum(n) x dim, times TX, offsets offX of length nX+1; same for Y).
 * D[k] receives the distance of pairs[2k], pairs[2k+1].  nthreads >= 1.
 */
void twed_oracle_pairs(const double *X, const double *TX, const int64_t *offX,
                       const double *Y, const double *TY, const int64_t *offY,
                       const int64_t *pairs, int64_t nPairs, int32_t dim,
                       double nu, double lambda, double p, double *D,
                       int32_t nthreads)
{
    batch_job job;
    job.X = X; job.TX = TX; job.Y = Y; job.TY = TY;
    job.offX = offX; job.offY = offY; job.pairs = pairs; job.nPairs = nPairs;
    job.dim = dim; job.nu = nu; job.lambda = lambda; job.p = p; job.D = D;
    job.next = 0;
    pthread_mutex_init(&job.lock, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 1; t < nthreads; t++)
        if (pthread_create(&th[started], NULL, batch_worker, &job) == 0) started++;
    batch_worker(&job);
    for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&job.lock);
}

int32_t twed_oracle_mutant(void) { return ORACLE_MUTANT; }
