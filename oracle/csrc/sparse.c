/*
 * Oracle (test infrastructure only): sparse products and conjugate gradients
 * for the block Lanczos reference eigensolver.  Written to be read, with
 * OpenMP over rows so that the reference runs at full size on the host cores;
 * it shares no code with the GPU library.
 *
 * oracle_spmm:  Y = A X for a CSR matrix A (n x n, int32 indices) and a
 *               row-major block X (n x k), one output row at a time.
 * oracle_cg:    conjugate gradients (Hestenes & Stiefel 1952) on A x_j = b_j
 *               for every column j of a row-major block B (n x k), all from
 *               x = 0, each column with its own alpha_j, beta_j; a column
 *               stops when ||r_j|| <= tol ||b_j|| or after maxit iterations.
 *
 * Reductions over rows are summed per thread over a fixed row range and the
 * thread partials added in thread order, so a run is reproducible for a fixed
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static void spmm_rows(int64_t r0, int64_t r1, const int32_t *rp, const int32_t *ci, const double *va, int k,
                      const double *X, double *Y)
{
    for (int64_t i = r0; i < r1; ++i) {
        double *y = Y + (size_t)i * k;
        for (int j = 0; j < k; ++j) y[j] = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const double a = va[e];
            const double *x = X + (size_t)ci[e] * k;
            for (int j = 0; j < k; ++j) y[j] += a * x[j];
        }
    }
}

void oracle_spmm(int64_t n, const int32_t *rp, const int32_t *ci, const double *va, int k, const double *X,
                 double *Y)
{
#pragma omp parallel
    {
        int nt = 1, t = 0;
#ifdef _OPENMP
        nt = omp_get_num_threads();
        t = omp_get_thread_num();
#endif
        const int64_t per = (n + nt - 1) / nt;
        const int64_t r0 = (int64_t)t * per < n ? (int64_t)t * per : n;
        const int64_t r1 = r0 + per < n ? r0 + per : n;
        spmm_rows(r0, r1, rp, ci, va, k, X, Y);
    }
}

/* Column sums sum_i u[i][j] * v[i][j] over all rows, reproducible for a fixed
 * thread count (part: nthreads x k scratch). */
static void coldots(int64_t n, int k, const double *U, const double *V, double *out, double *part, int nt)
{
#pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        const int64_t per = (n + nt - 1) / nt;
        const int64_t r0 = (int64_t)t * per < n ? (int64_t)t * per : n;
        const int64_t r1 = r0 + per < n ? r0 + per : n;
        double *p = part + (size_t)t * k;
        for (int j = 0; j < k; ++j) p[j] = 0.0;
        for (int64_t i = r0; i < r1; ++i)
            for (int j = 0; j < k; ++j) p[j] += U[(size_t)i * k + j] * V[(size_t)i * k + j];
    }
    for (int j = 0; j < k; ++j) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += part[(size_t)t * k + j];
        out[j] = s;
    }
}

/* B, X: n x k row-major; its: int[k] (iterations per column, may be NULL).
 * Returns 0, or -1 when a column meets p^T A p <= 0 (A not positive definite),
 * -2 on allocation failure. */
int oracle_cg(int64_t n, const int32_t *rp, const int32_t *ci, const double *va, int k, const double *B,
              double *X, double tol, int maxit, int *its)
{
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    const size_t nk = (size_t)n * k;
    double *r = (double *)malloc(sizeof(double) * nk);
    double *p = (double *)malloc(sizeof(double) * nk);
    double *q = (double *)malloc(sizeof(double) * nk);
    double *part = (double *)malloc(sizeof(double) * (size_t)nt * k);
    double *rr = (double *)malloc(sizeof(double) * k);
    double *rr0 = (double *)malloc(sizeof(double) * k);
    double *pq = (double *)malloc(sizeof(double) * k);
    double *al = (double *)malloc(sizeof(double) * k);
    double *be = (double *)malloc(sizeof(double) * k);
    int *act = (int *)malloc(sizeof(int) * k);
    int rc = 0;
    if (!r || !p || !q || !part || !rr || !rr0 || !pq || !al || !be || !act) {
        rc = -2;
        goto done;
    }
    memcpy(r, B, sizeof(double) * nk);
    memcpy(p, B, sizeof(double) * nk);
    memset(X, 0, sizeof(double) * nk);
    coldots(n, k, r, r, rr, part, nt);
    int nact = 0;
    for (int j = 0; j < k; ++j) {
        rr0[j] = rr[j];
        act[j] = rr[j] > 0.0;
        nact += act[j];
        if (its) its[j] = 0;
    }
    for (int it = 0; it < maxit && nact > 0; ++it) {
        oracle_spmm(n, rp, ci, va, k, p, q);
        coldots(n, k, p, q, pq, part, nt);
        for (int j = 0; j < k; ++j) {
            al[j] = 0.0;
            if (!act[j]) continue;
            if (!(pq[j] > 0.0)) {
                rc = -1;
                act[j] = 0;
                continue;
            }
            al[j] = rr[j] / pq[j];
        }
#pragma omp parallel for num_threads(nt) schedule(static)
        for (int64_t i = 0; i < n; ++i)
            for (int j = 0; j < k; ++j) {
                const size_t o = (size_t)i * k + j;
                X[o] += al[j] * p[o];
                r[o] -= al[j] * q[o];
            }
        double *rn = pq;   /* reuse */
        coldots(n, k, r, r, rn, part, nt);
        nact = 0;
        for (int j = 0; j < k; ++j) {
            be[j] = 0.0;
            if (!act[j]) continue;
            if (its) its[j] = it + 1;
            be[j] = rn[j] / rr[j];
            rr[j] = rn[j];
            if (rn[j] <= tol * tol * rr0[j]) act[j] = 0;
            else nact++;
        }
#pragma omp parallel for num_threads(nt) schedule(static)
        for (int64_t i = 0; i < n; ++i)
            for (int j = 0; j < k; ++j) {
                if (!act[j]) continue;
                const size_t o = (size_t)i * k + j;
                p[o] = r[o] + be[j] * p[o];
            }
    }
done:
    free(r);
    free(p);
    free(q);
    free(part);
    free(rr);
    free(rr0);
    free(pq);
    free(al);
    free(be);
    free(act);
    return rc;
}
