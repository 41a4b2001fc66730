// Host dense linear algebra of the small Rayleigh-Ritz problem (Section 3.2,
// STEP 3; the paper calls LAPACK dsyevx) and of STEP 5.  No LAPACK: the
// symmetric eigensolver is Householder reduction to tridiagonal form followed
// by the implicit QL iteration with Wilkinson-type shifts.  The QL iteration
// follows the published procedure tql2 (Bowdler, Martin, Reinsch and
// Wilkinson, "The QR and QL algorithms for symmetric matrices", Numer. Math.
// 11, 1968; Wilkinson and Reinsch, Handbook for Automatic Computation II,
// contribution II/3), step for step: the shift from the leading 2 x 2 block,
// the plane rotations chasing the bulge, and the early exit when a rotation
// radius vanishes.  Rotations of one QL sweep are recorded and then applied
// to the eigenvector matrix in parallel over its rows (OpenMP).
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

namespace gcge {

// Threads for a parallel loop of `work` multiply-adds: one below ~16K (the
// fork/join costs more than the loop), then one per ~8K up to the pool size.
static inline int nthreads_for(long work) {
    if (work < 16384) return 1;
    return (int)std::max<long>(1, std::min<long>(omp_get_max_threads(), work / 8192));
}

// Householder tridiagonalization of the symmetric n x n matrix held in a
// (column j at a + j * n; symmetric, so row-major input is the same).
// On exit d, e hold the tridiagonal T = Q^T A Q; the Householder vectors are
// stored below the subdiagonal of the columns of a (v_k[0] = 1 implied) with
// scalars tau[k]; Q = H_0 H_1 ... H_{n-3}, H_k = I - tau_k v_k v_k^T.
static void tridiagonalize(int n, double *a, double *d, double *e, double *tau) {
    std::vector<double> p(n), w(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        double *x = a + (size_t)k * n + (k + 1);   // column k, rows k+1 .. n-1
        const double alpha = x[0];
        double xn2 = 0.0;
        for (int i = 1; i < m; ++i) xn2 += x[i] * x[i];
        if (xn2 == 0.0) {
            tau[k] = 0.0;
            e[k] = alpha;
            continue;
        }
        const double beta = -std::copysign(std::sqrt(alpha * alpha + xn2), alpha);
        tau[k] = (beta - alpha) / beta;
        const double sc = 1.0 / (alpha - beta);
        for (int i = 1; i < m; ++i) x[i] *= sc;
        x[0] = 1.0;
        e[k] = beta;
        const double t = tau[k];
        double *A22 = a + (size_t)(k + 1) * n + (k + 1);   // column j of A22 at A22 + j * n
        const int nt = nthreads_for((long)m * m);
        // p = tau A22 v (A22 symmetric: p_i = tau * A22(:, i) . v)
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int i = 0; i < m; ++i) {
            const double *col = A22 + (size_t)i * n;
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += col[j] * x[j];
            p[i] = t * s;
        }
        double pv = 0.0;
        for (int i = 0; i < m; ++i) pv += p[i] * x[i];
        const double K = -0.5 * t * pv;
        for (int i = 0; i < m; ++i) w[i] = p[i] + K * x[i];
        // A22 -= v w^T + w v^T
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int j = 0; j < m; ++j) {
            double *col = A22 + (size_t)j * n;
            const double wj = w[j], vj = x[j];
            for (int i = 0; i < m; ++i) col[i] -= x[i] * wj + w[i] * vj;
        }
    }
    for (int k = 0; k < n; ++k) d[k] = a[(size_t)k * n + k];
    if (n >= 2) e[n - 2] = a[(size_t)(n - 2) * n + (n - 1)];
    e[n - 1] = 0.0;
    if (n >= 2) tau[n - 2] = 0.0;
    tau[n - 1] = 0.0;
}

// Implicit QL on (d, e) accumulating the rotations into Z (n x n row-major,
// starts as the identity); eigenvectors of T end up as the columns of Z.
static int tridiag_ql(int n, double *d, double *e, double *Z) {
    const double eps = 2.220446049250313e-16;
    std::vector<int> ri(n);
    std::vector<double> rc(n), rs(n);
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        while (true) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) return -1;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            int nrot = 0;
            bool early = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i];
                const double b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                ri[nrot] = i;
                rc[nrot] = c;
                rs[nrot] = s;
                ++nrot;
            }
            if (nrot > 0 && Z != nullptr) {
                const int nt = nthreads_for((long)nrot * n * 6);
#pragma omp parallel for schedule(static) num_threads(nt)
                for (int rb = 0; rb < n; rb += 4) {
                    const int re = std::min(n, rb + 4);
                    for (int t = 0; t < nrot; ++t) {
                        const int i = ri[t];
                        const double cc = rc[t], ss = rs[t];
                        for (int row = rb; row < re; ++row) {
                            double *z = Z + (size_t)row * n;
                            const double f = z[i + 1];
                            z[i + 1] = ss * z[i] + cc * f;
                            z[i] = cc * z[i] - ss * f;
                        }
                    }
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return 0;
}

int sym_eig(int n, double *a, double *w, double *z, int nwant) {
    if (n <= 0) return 0;
    if (nwant < 0 || nwant > n) return -2;
    std::vector<double> d(n), e(n), tau(n);
    tridiagonalize(n, a, d.data(), e.data(), tau.data());
    std::vector<double> Z;
    const bool vec = (z != nullptr && nwant > 0);
    if (vec) {
        Z.assign((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    }
    if (tridiag_ql(n, d.data(), e.data(), vec ? Z.data() : nullptr) != 0) return -1;
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
    for (int i = 0; i < n; ++i) w[i] = d[ord[i]];
    if (!vec) return 0;
    // selected eigenvectors of T, one contiguous column each: Y[j][i]
    std::vector<double> Y((size_t)nwant * n);
    for (int j = 0; j < nwant; ++j) {
        const int c = ord[j];
        double *y = Y.data() + (size_t)j * n;
        for (int i = 0; i < n; ++i) y[i] = Z[(size_t)i * n + c];
    }
    // back-transform: x = H_0 H_1 ... H_{n-3} y
    const int nt = nthreads_for((long)n * n * nwant);
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int j = 0; j < nwant; ++j) {
        double *y = Y.data() + (size_t)j * n;
        for (int k = n - 3; k >= 0; --k) {
            const double t = tau[k];
            if (t == 0.0) continue;
            const double *v = a + (size_t)k * n + (k + 1);   // v[0] = 1
            double s = 0.0;
            const int m = n - k - 1;
            for (int i = 0; i < m; ++i) s += v[i] * y[k + 1 + i];
            s *= t;
            for (int i = 0; i < m; ++i) y[k + 1 + i] -= s * v[i];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < nwant; ++j) z[(size_t)i * nwant + j] = Y[(size_t)j * n + i];
    return 0;
}

int jacobi_small(int n, double *a, double *w, double *v) {
    const double eps = 2.220446049250313e-16;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) v[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        int nrot = 0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[p * n + q];
                const double app = a[p * n + p], aqq = a[q * n + q];
                if (apq == 0.0 || std::fabs(apq) <= eps * std::sqrt(std::fabs(app) * std::fabs(aqq))) continue;
                ++nrot;
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {   // rows p, q
                    const double x = a[p * n + k], y = a[q * n + k];
                    a[p * n + k] = c * x - s * y;
                    a[q * n + k] = s * x + c * y;
                }
                for (int k = 0; k < n; ++k) {   // columns p, q
                    const double x = a[k * n + p], y = a[k * n + q];
                    a[k * n + p] = c * x - s * y;
                    a[k * n + q] = s * x + c * y;
                    const double vx = v[k * n + p], vy = v[k * n + q];
                    v[k * n + p] = c * vx - s * vy;
                    v[k * n + q] = s * vx + c * vy;
                }
                a[p * n + q] = a[q * n + p] = 0.0;
            }
        if (nrot == 0) {
            std::vector<int> ord(n);
            std::iota(ord.begin(), ord.end(), 0);
            std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return a[x * n + x] < a[y * n + y]; });
            std::vector<double> vt((size_t)n * n);
            for (int j = 0; j < n; ++j) {
                w[j] = a[ord[j] * n + ord[j]];
                for (int i = 0; i < n; ++i) vt[i * n + j] = v[i * n + ord[j]];
            }
            std::memcpy(v, vt.data(), sizeof(double) * n * n);
            return 0;
        }
    }
    return -1;
}

void matmul_tn(int k, int m, int n, const double *A, const double *B, double *C) {
    // C[i][j] = sum_r A[r][i] B[r][j]
    const int nt = nthreads_for((long)k * m * n);
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int i = 0; i < m; ++i) {
        double *c = C + (size_t)i * n;
        for (int j = 0; j < n; ++j) c[j] = 0.0;
        for (int r = 0; r < k; ++r) {
            const double a = A[(size_t)r * m + i];
            if (a == 0.0) continue;
            const double *b = B + (size_t)r * n;
            for (int j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
}

void matmul_nn(int m, int k, int n, const double *A, const double *B, double *C) {
    const int nt = nthreads_for((long)k * m * n);
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int i = 0; i < m; ++i) {
        double *c = C + (size_t)i * n;
        for (int j = 0; j < n; ++j) c[j] = 0.0;
        const double *a = A + (size_t)i * k;
        for (int r = 0; r < k; ++r) {
            const double av = a[r];
            if (av == 0.0) continue;
            const double *b = B + (size_t)r * n;
            for (int j = 0; j < n; ++j) c[j] += av * b[j];
        }
    }
}

int p_hat(int dim, int nx, const double *xhat, int shift, int n_old, int n_new, double drop_tol, double *phat) {
    // ptilde: columns shift .. shift+n_new-1 of xhat with rows 0 .. n_old-1 zeroed (eq. CP_tilde)
    const int nn = std::max(0, std::min(n_new, nx - shift));
    if (nn <= 0) return 0;
    std::vector<double> pt((size_t)dim * nn);
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < nn; ++j) pt[(size_t)i * nn + j] = (i < n_old) ? 0.0 : xhat[(size_t)i * nx + shift + j];
    std::vector<double> nrm0(nn, 0.0);
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < nn; ++j) nrm0[j] += pt[(size_t)i * nn + j] * pt[(size_t)i * nn + j];
    for (int j = 0; j < nn; ++j) nrm0[j] = std::sqrt(nrm0[j]);
    // L2 orthogonalization against xhat, twice: pt -= xhat (xhat^T pt)
    std::vector<double> cf((size_t)nx * nn), up((size_t)dim * nn);
    for (int pass = 0; pass < 2; ++pass) {
        matmul_tn(dim, nx, nn, xhat, pt.data(), cf.data());
        matmul_nn(dim, nx, nn, xhat, cf.data(), up.data());
        for (size_t t = 0; t < pt.size(); ++t) pt[t] -= up[t];
    }
    // modified Gram-Schmidt among the columns, twice, dropping small ones
    int np = 0;
    std::vector<double> v(dim);
    for (int j = 0; j < nn; ++j) {
        for (int i = 0; i < dim; ++i) v[i] = pt[(size_t)i * nn + j];
        for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < np; ++q) {
                double s = 0.0;
                for (int i = 0; i < dim; ++i) s += phat[(size_t)i * n_new + q] * v[i];
                for (int i = 0; i < dim; ++i) v[i] -= s * phat[(size_t)i * n_new + q];
            }
        double s = 0.0;
        for (int i = 0; i < dim; ++i) s += v[i] * v[i];
        s = std::sqrt(s);
        if (nrm0[j] > 0.0 && s > drop_tol * nrm0[j]) {
            for (int i = 0; i < dim; ++i) phat[(size_t)i * n_new + np] = v[i] / s;
            ++np;
        }
    }
    for (int i = 0; i < dim; ++i)
        for (int q = np; q < n_new; ++q) phat[(size_t)i * n_new + q] = 0.0;
    return np;
}

}  // namespace gcge
