/*
 * Oracle (test infrastructure only): dense symmetric eigendecomposition by the
 * cyclic two-sided Jacobi method.  Written for checking, not for speed; it
 * shares no code with the GPU library.
 *
 * Method (textbook, e.g. Golub & Van Loan, "Matrix Computations", the
 * symmetric Schur decomposition by Jacobi rotations): each rotation J(p,q)
 * annihilates the off-diagonal entry a_pq of A <- J^T A J and the product of
 * all rotations accumulates the eigenvectors V <- V J.  Pairs (p,q) are visited
 * in the round-robin ("circle") tournament order, so one round is a perfect
 * matching of disjoint pairs whose rotations commute and are applied together
 * (rows first, then columns), in parallel with OpenMP.  A rotation is skipped
 * when |a_pq| <= eps * sqrt(|a_pp| |a_qq|); the iteration stops after a sweep
 * (n'-1 rounds) in which no rotation was applied.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* a: n x n row-major symmetric, overwritten (diagonal ends up holding the
 * eigenvalues).  v: n x n row-major, receives eigenvectors as columns.
 * Returns the number of sweeps used, or -1 if max_sweeps was exhausted. */
int oracle_jacobi_eigh(int n, double *a, double *v, int max_sweeps)
{
    if (n <= 0) return 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) v[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    if (n == 1) return 0;
    const double eps = 2.220446049250313e-16;
    const int np = (n % 2) ? n + 1 : n;     /* one dummy player when n is odd */
    const int npairs = np / 2;
    int *pp = (int *)malloc(sizeof(int) * npairs);
    int *qq = (int *)malloc(sizeof(int) * npairs);
    double *cs = (double *)malloc(sizeof(double) * npairs);
    double *sn = (double *)malloc(sizeof(double) * npairs);
    double *dp = (double *)malloc(sizeof(double) * npairs);
    double *dq = (double *)malloc(sizeof(double) * npairs);
    int *act = (int *)malloc(sizeof(int) * npairs);
    int sweeps = 0, done = 0;
    while (!done && sweeps < max_sweeps) {
        long nrot = 0;
        for (int r = 0; r < np - 1; ++r) {
            /* circle method: player np-1 fixed, the others rotate */
            for (int i = 0; i < npairs; ++i) {
                int x, y;
                if (i == 0) { x = r; y = np - 1; }
                else { x = (r + i) % (np - 1); y = (r - i + (np - 1)) % (np - 1); }
                pp[i] = x < y ? x : y;
                qq[i] = x < y ? y : x;
            }
            int nact = 0;
            for (int i = 0; i < npairs; ++i) {
                int p = pp[i], q = qq[i];
                act[i] = 0;
                if (q >= n) continue;                 /* dummy player */
                double apq = a[(size_t)p * n + q];
                double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                if (apq == 0.0 || fabs(apq) <= eps * sqrt(fabs(app) * fabs(aqq))) continue;
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                cs[i] = c; sn[i] = t * c;
                dp[i] = app - t * apq; dq[i] = aqq + t * apq;
                act[i] = 1; ++nact;
            }
            if (nact == 0) continue;
            nrot += nact;
            /* rows: A <- J^T A */
#pragma omp parallel for schedule(static) if (n >= 96)
            for (int i = 0; i < npairs; ++i) {
                if (!act[i]) continue;
                double *rp = a + (size_t)pp[i] * n, *rq = a + (size_t)qq[i] * n;
                double c = cs[i], s = sn[i];
                for (int k = 0; k < n; ++k) {
                    double x = rp[k], y = rq[k];
                    rp[k] = c * x - s * y;
                    rq[k] = s * x + c * y;
                }
            }
            /* columns: A <- A J, V <- V J */
#pragma omp parallel for schedule(static) if (n >= 96)
            for (int k = 0; k < n; ++k) {
                double *ra = a + (size_t)k * n, *rv = v + (size_t)k * n;
                for (int i = 0; i < npairs; ++i) {
                    if (!act[i]) continue;
                    int p = pp[i], q = qq[i];
                    double c = cs[i], s = sn[i];
                    double x = ra[p], y = ra[q];
                    ra[p] = c * x - s * y;
                    ra[q] = s * x + c * y;
                    x = rv[p]; y = rv[q];
                    rv[p] = c * x - s * y;
                    rv[q] = s * x + c * y;
                }
            }
            /* the annihilated 2x2 blocks, set exactly */
            for (int i = 0; i < npairs; ++i) {
                if (!act[i]) continue;
                int p = pp[i], q = qq[i];
                a[(size_t)p * n + q] = 0.0;
                a[(size_t)q * n + p] = 0.0;
                a[(size_t)p * n + p] = dp[i];
                a[(size_t)q * n + q] = dq[i];
            }
        }
        ++sweeps;
        if (nrot == 0) done = 1;
    }
    free(pp); free(qq); free(cs); free(sn); free(dp); free(dq); free(act);
    return done ? sweeps : -1;
}
