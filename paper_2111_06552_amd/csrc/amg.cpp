// Smoothed-aggregation algebraic multigrid, the preconditioner of the STEP 6
// linear systems (Section 2 suggests an algebraic multigrid preconditioner for
// STEP 6 with the shift theta = 0 when A comes from a PDE discretization).
// The paper does not fix the AMG; this one is smoothed aggregation (Vanek,
// Mandel and Brezina, Computing 56, 1996) with these choices:
//   strength      j != i is strong for row i when |a_ij| >= eps_l sqrt(|a_ii a_jj|),
//                 eps_l = eps_0 * 2^-l at level l (eps_0 = 0.02 by default: the
//                 27-point Q1 stiffness couples a row to each neighbour by
//                 about 1/30 of its diagonal);
//   aggregation   rows in order; phase 1: a row whose strong neighbours are all
//                 free seeds an aggregate with them (no strong neighbour: a
//                 singleton); phase 2: a row left joins the phase-1 aggregate
//                 of its strongest phase-1-aggregated neighbour (neighbours in
//                 column order, a later one wins only when |a_ij| is larger
//                 by a relative 1e-8, so rounding cannot change the choice);
//   prolongator   P = (I - omega D^-1 A) P_t, P_t[i, agg(i)] = |agg(i)|^-1/2,
//                 omega = 4 / (3 rho), rho = max_i sum_j |a_ij| / a_ii;
//   coarse level  R = P^T, A_next = R A P; a level is the last one when it has
//                 at most coarse_max rows, at the level limit, when it stores
//                 more than 400 entries per row (Galerkin products of denser
//                 levels cost more than they save), or when aggregation would
//                 keep more than half of its rows; the last level is inverted
//                 densely (Cholesky, at most 4096 rows, else the setup fails)
//                 and applied as a GEMM;
//   V-cycle       x = w b (one damped Jacobi sweep from zero, w = omega D^-1),
//                 t = b - A x, x += P V(R t), y = x + w (b - A x): symmetric
//                 and positive definite, so it preconditions CG.
// The setup runs on the host (OpenMP over rows; fixed summation orders, so
// the hierarchy does not depend on the thread count); every step of the
// V-cycle is a device kernel.
#include "gcge.h"
#include "internal.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

namespace gcge {

namespace {

constexpr double TIE_REL = 1e-8;

int status_of(hipError_t e) { return e == hipErrorOutOfMemory ? GCGE_ERR_OOM : GCGE_ERR_HIP; }

// host CSR, n rows x m columns, sorted unique column indices per row
struct HCsr {
    int64_t n = 0, m = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> va;
    int64_t nnz() const { return rp.empty() ? 0 : rp[n]; }
};

bool diag_of(const HCsr &A, std::vector<double> &d) {
    d.assign(A.n, 0.0);
    for (int64_t i = 0; i < A.n; ++i)
        for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e)
            if (A.ci[e] == i) d[i] = A.va[e];
    for (int64_t i = 0; i < A.n; ++i)
        if (!(d[i] > 0.0)) return false;
    return true;
}

void aggregate(const HCsr &A, const std::vector<double> &d, double eps, std::vector<int32_t> &agg, int64_t &nagg) {
    const int64_t n = A.n;
    std::vector<uint8_t> strong(A.nnz());
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
            const int64_t j = A.ci[e];
            strong[e] = (j != i && std::fabs(A.va[e]) >= eps * std::sqrt(std::fabs(d[i] * d[j]))) ? 1 : 0;
        }
    agg.assign(n, -1);
    nagg = 0;
    for (int64_t i = 0; i < n; ++i) {   // phase 1
        if (agg[i] >= 0) continue;
        bool free_nb = true;
        for (int32_t e = A.rp[i]; e < A.rp[i + 1] && free_nb; ++e)
            if (strong[e] && agg[A.ci[e]] >= 0) free_nb = false;
        if (!free_nb) continue;
        agg[i] = (int32_t)nagg;
        for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e)
            if (strong[e]) agg[A.ci[e]] = (int32_t)nagg;
        ++nagg;
    }
    const std::vector<int32_t> p1 = agg;
    for (int64_t i = 0; i < n; ++i) {   // phase 2
        if (agg[i] >= 0) continue;
        int64_t best = -1;
        double ba = -1.0;
        for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
            if (!strong[e] || p1[A.ci[e]] < 0) continue;
            const double a = std::fabs(A.va[e]);
            if (best < 0 || a > ba * (1.0 + TIE_REL)) {
                best = A.ci[e];
                ba = a;
            }
        }
        // a row left after phase 1 was blocked by a phase-1-aggregated strong
        // neighbour, so best >= 0
        agg[i] = best >= 0 ? p1[best] : (int32_t)nagg++;
    }
}

double gershgorin(const HCsr &A, const std::vector<double> &d) {
    double rho = 0.0;
    for (int64_t i = 0; i < A.n; ++i) {
        double s = 0.0;
        for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) s += std::fabs(A.va[e]);
        rho = std::max(rho, s / d[i]);
    }
    return rho;
}

// Rows of a sparse matrix built row by row in parallel, chunk by chunk.
// Returns false when the result has more entries than int32 row pointers hold.
template <typename RowFn>
bool build_rows(int64_t n, int64_t m, HCsr &out, RowFn &&row) {
    out.n = n;
    out.m = m;
    out.rp.assign(n + 1, 0);
    const int64_t CH = 4096;
    const int64_t nch = (n + CH - 1) / CH;
    std::vector<std::vector<int32_t>> cci(nch);
    std::vector<std::vector<double>> cva(nch);
    std::vector<std::vector<int32_t>> ccnt(nch);
#pragma omp parallel
    {
        std::vector<std::pair<int32_t, double>> buf;
        std::vector<double> acc(m, 0.0);
        std::vector<int64_t> mark(m, -1);
#pragma omp for schedule(dynamic, 1)
        for (int64_t c = 0; c < nch; ++c) {
            const int64_t r0 = c * CH, r1 = std::min(n, r0 + CH);
            ccnt[c].resize(r1 - r0);
            for (int64_t i = r0; i < r1; ++i) {
                buf.clear();
                row(i, buf, acc, mark);
                std::sort(buf.begin(), buf.end(),
                          [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
                              return a.first < b.first;
                          });
                ccnt[c][i - r0] = (int32_t)buf.size();
                for (const auto &pv : buf) {
                    cci[c].push_back(pv.first);
                    cva[c].push_back(pv.second);
                }
            }
        }
    }
    int64_t total = 0;
    for (int64_t c = 0; c < nch; ++c) total += (int64_t)cci[c].size();
    if (total > INT32_MAX) return false;
    for (int64_t c = 0; c < nch; ++c)
        for (size_t t = 0; t < ccnt[c].size(); ++t) out.rp[c * CH + t + 1] = ccnt[c][t];
    for (int64_t i = 0; i < n; ++i) out.rp[i + 1] += out.rp[i];
    out.ci.resize(out.rp[n]);
    out.va.resize(out.rp[n]);
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t off = out.rp[c * CH];
        std::copy(cci[c].begin(), cci[c].end(), out.ci.begin() + off);
        std::copy(cva[c].begin(), cva[c].end(), out.va.begin() + off);
    }
    return true;
}

// P = (I - omega D^-1 A) P_t: row i holds the aggregates of the columns of
// row i of A; entry a gets -omega/a_ii sum_{j in row i, agg(j) = a} a_ij t_a,
// plus t_a at a = agg(i).
bool smoothed_p(const HCsr &A, const std::vector<double> &d, const std::vector<int32_t> &agg, int64_t nagg,
                double omega, HCsr &P) {
    std::vector<int64_t> cnt(nagg, 0);
    for (int32_t a : agg) ++cnt[a];
    std::vector<double> t(nagg);
    for (int64_t a = 0; a < nagg; ++a) t[a] = 1.0 / std::sqrt((double)cnt[a]);
    return build_rows(A.n, nagg, P,
               [&](int64_t i, std::vector<std::pair<int32_t, double>> &buf, std::vector<double> &acc,
                   std::vector<int64_t> &mark) {
                   for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
                       const int32_t a = agg[A.ci[e]];
                       if (mark[a] != i) {
                           mark[a] = i;
                           acc[a] = 0.0;
                           buf.push_back({a, 0.0});
                       }
                       acc[a] += A.va[e] * t[a];
                   }
                   const double s = -omega / d[i];
                   for (auto &pv : buf) {
                       pv.second = s * acc[pv.first];
                       if (pv.first == agg[i]) pv.second += t[pv.first];
                   }
               });
}

void transpose(const HCsr &P, HCsr &R) {
    R.n = P.m;
    R.m = P.n;
    R.rp.assign(R.n + 1, 0);
    for (int64_t e = 0; e < P.nnz(); ++e) ++R.rp[P.ci[e] + 1];
    for (int64_t i = 0; i < R.n; ++i) R.rp[i + 1] += R.rp[i];
    R.ci.resize(P.nnz());
    R.va.resize(P.nnz());
    std::vector<int64_t> pos(R.rp.begin(), R.rp.end() - 1);
    for (int64_t i = 0; i < P.n; ++i)   // rows in order: columns of R come out sorted
        for (int32_t e = P.rp[i]; e < P.rp[i + 1]; ++e) {
            const int64_t q = pos[P.ci[e]]++;
            R.ci[q] = (int32_t)i;
            R.va[q] = P.va[e];
        }
}

// C = A B (Gustavson, row by row; sums in the order of A's row and B's rows)
bool spgemm(const HCsr &A, const HCsr &B, HCsr &C) {
    return build_rows(A.n, B.m, C,
               [&](int64_t i, std::vector<std::pair<int32_t, double>> &buf, std::vector<double> &acc,
                   std::vector<int64_t> &mark) {
                   for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
                       const double a = A.va[e];
                       const int64_t k = A.ci[e];
                       for (int32_t f = B.rp[k]; f < B.rp[k + 1]; ++f) {
                           const int32_t c = B.ci[f];
                           if (mark[c] != i) {
                               mark[c] = i;
                               acc[c] = 0.0;
                               buf.push_back({c, 0.0});
                           }
                           acc[c] += a * B.va[f];
                       }
                   }
                   for (auto &pv : buf) pv.second = acc[pv.first];
               });
}

// Dense inverse of an SPD matrix through its Cholesky factor (row-major).
bool spd_inverse(const HCsr &A, std::vector<double> &inv) {
    const int64_t n = A.n;
    std::vector<double> L((size_t)n * n, 0.0), M((size_t)n * n, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int32_t e = A.rp[i]; e < A.rp[i + 1]; ++e) M[(size_t)i * n + A.ci[e]] = A.va[e];
    for (int64_t j = 0; j < n; ++j) {
        double s = M[(size_t)j * n + j];
        for (int64_t p = 0; p < j; ++p) s -= L[(size_t)j * n + p] * L[(size_t)j * n + p];
        if (!(s > 0.0)) return false;
        const double ljj = std::sqrt(s);
        L[(size_t)j * n + j] = ljj;
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            double v = M[(size_t)i * n + j];
            for (int64_t p = 0; p < j; ++p) v -= L[(size_t)i * n + p] * L[(size_t)j * n + p];
            L[(size_t)i * n + j] = v / ljj;
        }
    }
    // Linv (lower) by forward substitution, column by column; inv = Linv^T Linv
    std::vector<double> Li((size_t)n * n, 0.0);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t c = 0; c < n; ++c)
        for (int64_t i = c; i < n; ++i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int64_t p = c; p < i; ++p) v -= L[(size_t)i * n + p] * Li[(size_t)p * n + c];
            Li[(size_t)i * n + c] = v / L[(size_t)i * n + i];
        }
    inv.assign((size_t)n * n, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int64_t p = std::max(i, j); p < n; ++p) s += Li[(size_t)p * n + i] * Li[(size_t)p * n + j];
            inv[(size_t)i * n + j] = s;
        }
    return true;
}

hipError_t upload(std::vector<void *> &owned, void **dst, const void *src, size_t bytes) {
    *dst = nullptr;
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) return e;
    owned.push_back(*dst);
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
}

hipError_t upload_csr(std::vector<void *> &owned, const HCsr &H, DevCsr<double> &D) {
    D.n = H.n;
    D.nnz = H.nnz();
    D.uorder = nullptr;
    void *rp = nullptr, *ci = nullptr, *va = nullptr;
    hipError_t e = upload(owned, &rp, H.rp.data(), sizeof(int32_t) * H.rp.size());
    if (e == hipSuccess) e = upload(owned, &ci, H.ci.data(), sizeof(int32_t) * H.ci.size());
    if (e == hipSuccess) e = upload(owned, &va, H.va.data(), sizeof(double) * H.va.size());
    D.rowptr = (const int32_t *)rp;
    D.colind = (const int32_t *)ci;
    D.val = (const double *)va;
    return e;
}

// FP32 copy of the values of an uploaded level matrix (same index arrays).
hipError_t upload_f32(std::vector<void *> &owned, const HCsr &H, const DevCsr<double> &D, DevCsr<float> &F) {
    std::vector<float> v(H.va.begin(), H.va.end());
    void *p = nullptr;
    hipError_t e = upload(owned, &p, v.data(), sizeof(float) * v.size());
    F.n = D.n;
    F.nnz = D.nnz;
    F.rowptr = D.rowptr;
    F.colind = D.colind;
    F.val = (const float *)p;
    F.uorder = nullptr;
    return e;
}

inline size_t pad256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

void Amg::release() {
    for (void *p : owned) (void)hipFree(p);
    owned.clear();
    if (work) (void)hipFree(work);
    work = nullptr;
    work_bytes = 0;
    kcap = 0;
    ldw = 0;
    lv.clear();
    cinv = nullptr;
    agg.clear();
    rows.clear();
    nnz.clear();
    omega.clear();
    rho.clear();
}

int Amg::build(const DevCsr<double> &A0, int max_levels, int coarse_max, double strength, hipStream_t st,
               std::string &err) {
    release();
    if (max_levels < 1 || max_levels > AMG_MAX_LEVELS || coarse_max < 1 || A0.n < 1 || !(strength >= 0.0) ||
        strength >= 1.0) {
        err = "amg: invalid setup parameters";
        return GCGE_ERR_INVALID_ARG;
    }
    HCsr cur;
    cur.n = cur.m = A0.n;
    cur.rp.resize(A0.n + 1);
    cur.ci.resize(A0.nnz);
    cur.va.resize(A0.nnz);
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess)
        e = hipMemcpy(cur.rp.data(), A0.rowptr, sizeof(int32_t) * (A0.n + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess && A0.nnz)
        e = hipMemcpy(cur.ci.data(), A0.colind, sizeof(int32_t) * A0.nnz, hipMemcpyDeviceToHost);
    if (e == hipSuccess && A0.nnz)
        e = hipMemcpy(cur.va.data(), A0.val, sizeof(double) * A0.nnz, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        err = std::string("amg: download: ") + hipGetErrorString(e);
        return status_of(e);
    }
    for (int lev = 0;; ++lev) {
        std::vector<double> d;
        if (!diag_of(cur, d)) {
            err = "amg: the operator needs a positive diagonal at level " + std::to_string(lev);
            release();
            return GCGE_ERR_NOT_SPD;
        }
        AmgLevel L;
        L.n = cur.n;
        rows.push_back(cur.n);
        nnz.push_back(cur.nnz());
        if (lev == 0) {
            L.A = A0;
        } else {
            e = upload_csr(owned, cur, L.A);
            if (e == hipSuccess) e = upload_f32(owned, cur, L.A, L.A32);
        }
        bool last = cur.n <= coarse_max || lev == max_levels - 1 || cur.nnz() > AMG_MAX_ROW_FILL * cur.n;
        std::vector<int32_t> ag;
        int64_t nagg = 0;
        if (!last) {
            aggregate(cur, d, strength * std::ldexp(1.0, -lev), ag, nagg);
            if (2 * nagg > cur.n) last = true;
        }
        if (last) {
            if (cur.n > AMG_COARSE_LIMIT) {
                err = "amg: coarsening stops at level " + std::to_string(lev) + " with " + std::to_string(cur.n) +
                      " rows and " + std::to_string(cur.nnz() / cur.n) + " entries per row, above the " +
                      std::to_string(AMG_COARSE_LIMIT) + " rows of a dense coarsest level: this operator is not "
                      "suited to the aggregation multigrid";
                release();
                return GCGE_ERR_INVALID_ARG;
            }
            std::vector<double> inv;
            if (!spd_inverse(cur, inv)) {
                err = "amg: coarsest operator is not positive definite";
                release();
                return GCGE_ERR_NOT_SPD;
            }
            void *p = nullptr;
            if (e == hipSuccess) e = upload(owned, &p, inv.data(), sizeof(double) * inv.size());
            cinv = (double *)p;
            lv.push_back(L);
            break;
        }
        const double r = gershgorin(cur, d);
        const double om = 4.0 / (3.0 * r);
        std::vector<double> w(cur.n);
        for (int64_t i = 0; i < cur.n; ++i) w[i] = om / d[i];
        std::vector<float> w32(w.begin(), w.end());
        void *pw = nullptr, *pw32 = nullptr;
        if (e == hipSuccess) e = upload(owned, &pw, w.data(), sizeof(double) * w.size());
        if (e == hipSuccess) e = upload(owned, &pw32, w32.data(), sizeof(float) * w32.size());
        L.w = (double *)pw;
        L.w32 = (float *)pw32;
        HCsr P, R, AP, Ac;
        bool fits = smoothed_p(cur, d, ag, nagg, om, P);
        if (fits) transpose(P, R);
        fits = fits && spgemm(cur, P, AP) && spgemm(R, AP, Ac);
        if (!fits) {
            err = "amg: a product of level " + std::to_string(lev) + " exceeds 2^31 stored entries";
            release();
            return GCGE_ERR_INVALID_ARG;
        }
        if (e == hipSuccess) e = upload_csr(owned, P, L.P);
        if (e == hipSuccess) e = upload_csr(owned, R, L.R);
        if (e == hipSuccess) e = upload_f32(owned, P, L.P, L.P32);
        if (e == hipSuccess) e = upload_f32(owned, R, L.R, L.R32);
        if (e != hipSuccess) break;
        agg.push_back(std::move(ag));
        omega.push_back(om);
        rho.push_back(r);
        lv.push_back(L);
        cur = std::move(Ac);
    }
    if (e != hipSuccess) {
        err = std::string("amg: upload: ") + hipGetErrorString(e);
        release();
        return status_of(e);
    }
    return GCGE_OK;
}

template <typename T>
int Amg::apply(const T *b, int64_t ldb, int k, T *y, int64_t ldy, T *part, int *nparts, hipStream_t st,
               std::string &err, const int *skip, bool exact_out) {
    constexpr bool F32 = std::is_same<T, float>::value;
    if (lv.empty()) {
        err = "amg: no hierarchy";
        return GCGE_ERR_INVALID_ARG;
    }
    if (k < 0 || k > 128 || ldb < k || ldy < k) {
        err = "amg: invalid apply arguments";
        return GCGE_ERR_INVALID_ARG;
    }
    if (F32 && lv.size() > 1 && lv[0].A32.val == nullptr) {
        err = "amg: no FP32 level-0 operator";
        return GCGE_ERR_INVALID_ARG;
    }
    if (nparts) *nparts = 0;
    if (k == 0) return GCGE_OK;
    hipError_t e = hipSuccess;
    const int L = (int)lv.size() - 1;
    const int64_t ldk = (k + 3) / 4 * 4;   // 16-byte rows for FP64 and FP32
    if (k > kcap) {
        // x, t on every smoothed level, b, y on every level but the finest
        // (sized for FP64), and two FP64 blocks for the coarsest solve
        size_t bytes = 0;
        for (int l = 0; l <= L; ++l) {
            const size_t v = pad256(sizeof(double) * lv[l].n * ldk);
            bytes += (l < L ? 2 * v : 0) + (l > 0 ? 2 * v : 0);
        }
        bytes += 2 * pad256(sizeof(double) * lv[L].n * ldk);
        if (work) (void)hipFree(work);
        work = nullptr;
        work_bytes = 0;
        kcap = 0;
        e = hipMalloc((void **)&work, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) {
            work = nullptr;
            err = std::string("amg: work vectors: ") + hipGetErrorString(e);
            return status_of(e);
        }
        work_bytes = bytes;
        kcap = k;
        ldw = ldk;
    }
    std::vector<T *> X(L + 1, nullptr), Tv(L + 1, nullptr), Bv(L + 1, nullptr), Y(L + 1, nullptr);
    double *c64a = nullptr, *c64b = nullptr;
    {
        char *p = (char *)work;
        for (int l = 0; l <= L; ++l) {
            const size_t v = pad256(sizeof(double) * lv[l].n * ldw);
            if (l < L) {
                X[l] = (T *)p;
                Tv[l] = (T *)(p + v);
                p += 2 * v;
            }
            if (l > 0) {
                Bv[l] = (T *)p;
                Y[l] = (T *)(p + v);
                p += 2 * v;
            }
        }
        c64a = (double *)p;
        c64b = (double *)(p + pad256(sizeof(double) * lv[L].n * ldw));
    }
    auto A_of = [&](int l) -> DevCsr<T> {
        if constexpr (F32) return lv[l].A32; else return lv[l].A;
    };
    auto P_of = [&](int l) -> DevCsr<T> {
        if constexpr (F32) return lv[l].P32; else return lv[l].P;
    };
    auto R_of = [&](int l) -> DevCsr<T> {
        if constexpr (F32) return lv[l].R32; else return lv[l].R;
    };
    auto w_of = [&](int l) -> const T * {
        if constexpr (F32) return lv[l].w32; else return lv[l].w;
    };
    // descend: pre-smoothing, residual, restriction
    const T *bl = b;
    int64_t ldbl = ldb;
    for (int l = 0; l < L && e == hipSuccess; ++l) {
        e = scale_rows<T>(lv[l].n, k, w_of(l), bl, ldbl, X[l], ldw, st);
        Affine<T> res;
        res.b = bl;
        res.ldb = ldbl;
        if (e == hipSuccess)
            e = spmm_affine<T>(A_of(l), X[l], ldw, k, Tv[l], ldw, res, st, nullptr, 0, nullptr, nullptr, skip);
        Affine<T> restrict_;   // b_next = R t  (0 - (-1) R t)
        restrict_.ws = T(-1);
        if (e == hipSuccess)
            e = spmm_affine<T>(R_of(l), Tv[l], ldw, k, Bv[l + 1], ldw, restrict_, st, nullptr, 0, nullptr, nullptr,
                               skip);
        bl = Bv[l + 1];
        ldbl = ldw;
    }
    // coarsest level: y_L = A_L^-1 b_L (dense inverse, FP64 GEMM)
    if (e == hipSuccess) {
        const int64_t nc = lv[L].n;
        T *yL = L == 0 ? y : Y[L];
        const int64_t ldyL = L == 0 ? ldy : ldw;
        Segs S;
        S.add(cinv, nc, (int)nc);
        if constexpr (F32) {
            e = copy_cols<float, double>(nc, k, bl, ldbl, c64a, ldw, nullptr, st);
            if (e == hipSuccess) e = gemm(nc, S, c64a, ldw, k, 1.0, 0.0, c64b, ldw, st);
            if (e == hipSuccess) e = copy_cols<double, float>(nc, k, c64b, ldw, yL, ldyL, nullptr, st);
        } else {
            e = gemm(nc, S, bl, ldbl, k, 1.0, 0.0, yL, ldyL, st);
        }
        if (L == 0 && part != nullptr && e == hipSuccess) e = coldot_part<T>(nc, k, y, ldy, b, ldb, part, nparts, st);
    }
    // ascend: coarse correction, post-smoothing
    for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
        const T *bb = l == 0 ? b : Bv[l];
        const int64_t ldbb = l == 0 ? ldb : ldw;
        Affine<T> cor;
        cor.z = X[l];
        cor.ldz = ldw;
        cor.ws = T(-1);
        e = spmm_affine<T>(P_of(l), Y[l + 1], ldw, k, X[l], ldw, cor, st, nullptr, 0, nullptr, nullptr, skip);
        Affine<T> sm;
        sm.b = bb;
        sm.ldb = ldbb;
        sm.z = X[l];
        sm.ldz = ldw;
        sm.w = w_of(l);
        sm.ws = T(1);
        sm.exact = l == 0 && exact_out;
        T *out = l == 0 ? y : Y[l];
        const int64_t ldo = l == 0 ? ldy : ldw;
        if (e == hipSuccess) {
            if (l == 0 && part != nullptr)
                e = spmm_affine<T>(A_of(l), X[l], ldw, k, out, ldo, sm, st, b, ldb, part, nparts, skip);
            else
                e = spmm_affine<T>(A_of(l), X[l], ldw, k, out, ldo, sm, st, nullptr, 0, nullptr, nullptr, skip);
        }
    }
    if (e != hipSuccess) {
        err = std::string("amg: V-cycle: ") + hipGetErrorString(e);
        return status_of(e);
    }
    return GCGE_OK;
}
template int Amg::apply<double>(const double *, int64_t, int, double *, int64_t, double *, int *, hipStream_t,
                                std::string &, const int *, bool);
template int Amg::apply<float>(const float *, int64_t, int, float *, int64_t, float *, int *, hipStream_t,
                               std::string &, const int *, bool);

}  // namespace gcge
