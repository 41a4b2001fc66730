// Operator setup (union pattern, shifted values), host<->device staging, and
// the B-orthogonalization of STEP 2: block Gram-Schmidt against the already
// B-orthonormal [X, P] followed by RecursiveOrthSVD (Algorithm 3).
#include "operator.h"

#include <algorithm>
#include <map>
#include <cmath>
#include <cstring>
#include <vector>

namespace gcge {

hipError_t scatter_values(int64_t nnz, const int32_t *map, const double *src, double *dst, hipStream_t st);

#define GCGE_TRY(expr)                           \
    do {                                         \
        hipError_t _e = (expr);                  \
        if (_e != hipSuccess) return _e;         \
    } while (0)

// ------------------------------------------------------------------ Stager
// Waits for the stream by polling it: the host decisions of STEP 2 (leaf
// eigensolves, pass tests) wait on a small download about twenty times per
// iteration, and a blocking wait wakes up tens of microseconds after the copy
// has finished.
static hipError_t spin_wait(hipStream_t st) {
    for (;;) {
        const hipError_t e = hipStreamQuery(st);
        if (e != hipErrorNotReady) return e;
    }
}

hipError_t Stager::upload(void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return hipSuccess;
    const size_t need = (bytes + 255) / 256 * 256;
    if (off + need > cap) {
        GCGE_TRY(sync());
        if (need > cap) {
            if (ring) GCGE_TRY(hipHostFree(ring));
            ring = nullptr;
            cap = 0;
            size_t nc = std::max<size_t>(need, 16u << 20);
            GCGE_TRY(hipHostMalloc((void **)&ring, nc, hipHostMallocDefault));
            cap = nc;
        }
    }
    std::memcpy(ring + off, src, bytes);
    GCGE_TRY(hipMemcpyAsync(dst, ring + off, bytes, hipMemcpyHostToDevice, st));
    off += need;
    return hipSuccess;
}

hipError_t Stager::download(void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return sync();
    const size_t need = (bytes + 255) / 256 * 256;
    if (off + need > cap) {
        GCGE_TRY(sync());
        if (need > cap) {
            if (ring) GCGE_TRY(hipHostFree(ring));
            ring = nullptr;
            cap = 0;
            size_t nc = std::max<size_t>(need, 16u << 20);
            GCGE_TRY(hipHostMalloc((void **)&ring, nc, hipHostMallocDefault));
            cap = nc;
        }
    }
    GCGE_TRY(hipMemcpyAsync(ring + off, src, bytes, hipMemcpyDeviceToHost, st));
    GCGE_TRY(spin_wait(st));
    std::memcpy(dst, ring + off, bytes);
    off = 0;
    return hipSuccess;
}

hipError_t Stager::sync() {
    GCGE_TRY(spin_wait(st));
    off = 0;
    return hipSuccess;
}

void Stager::release() {
    if (ring) (void)hipHostFree(ring);
    ring = nullptr;
    cap = off = 0;
}

// ---------------------------------------------------------- SpMM unit order
// Operators of grids in natural order couple most rows to a row a fixed
// distance S ahead (the next plane).  Swept in natural order, the vector rows
// one plane back have left the 4 MB L2 of an XCD before they are gathered
// again, so every vector row is fetched about three times.  When such an S
// exists, each XCD's contiguous range of 64-row units is visited by blocks of
// positions within a plane, plane after plane: units whose (row mod S) falls
// in the same block of SPMM_BX rows come together, so a row's neighbours in
// the adjacent planes were gathered a few thousand rows earlier.  Only the
// visiting order changes; products are identical to natural order.
constexpr int64_t SPMM_BX = 1024;   // rows of a block within a plane
constexpr int SPMM_XCD = 8;

std::vector<int32_t> spmm_unit_order(int64_t n, const int32_t *rp, const int32_t *ci, int64_t *plane) {
    *plane = 0;
    const int64_t nu = (n + 63) / 64;
    if (n < 4 * 256) return {};
    // the largest forward offset beyond 64 rows that half of the sampled rows have
    const int64_t step = std::max<int64_t>(1, n / 20000);
    std::map<int64_t, int64_t> cnt;
    int64_t samples = 0;
    for (int64_t r = 0; r < n; r += step) {
        ++samples;
        for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int64_t off = (int64_t)ci[e] - r;
            if (off > 64) ++cnt[off];
        }
    }
    int64_t S = 0;
    for (const auto &kv : cnt)
        if (2 * kv.second >= samples) S = std::max(S, kv.first);
    if (S < 256 || n < 4 * S) return {};
    *plane = S;
    std::vector<int32_t> order(nu);
    const int64_t per = (nu + SPMM_XCD - 1) / SPMM_XCD;
    std::vector<std::pair<std::pair<int64_t, int64_t>, int32_t>> keys;
    for (int64_t u0 = 0; u0 < nu; u0 += per) {
        const int64_t u1 = std::min(nu, u0 + per);
        keys.clear();
        for (int64_t u = u0; u < u1; ++u) {
            const int64_t row = u * 64;
            keys.push_back({{(row % S) / SPMM_BX, row / S}, (int32_t)u});
        }
        std::stable_sort(keys.begin(), keys.end(),
                         [](const auto &x, const auto &y) { return x.first < y.first; });
        for (int64_t j = 0; j < u1 - u0; ++j) order[u0 + j] = keys[j].second;
    }
    return order;
}

// ---------------------------------------------------------------- Operator
static bool check_pattern(int64_t n, int64_t nnz, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                          std::string &err, const char *name) {
    if (rp[0] != 0 || (int64_t)rp[n] != nnz) {
        err = std::string(name) + ": rowptr[0] must be 0 and rowptr[n] must equal nnz";
        return false;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) {
            err = std::string(name) + ": rowptr is not monotone";
            return false;
        }
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= n) {
                err = std::string(name) + ": column index out of range";
                return false;
            }
            if (e > rp[i] && ci[e] <= ci[e - 1]) {
                err = std::string(name) + ": column indices of a row must be sorted and unique";
                return false;
            }
        }
    }
    return true;
}

int Operator::build(const gcge_csr *A, int b_kind, const void *B, hipStream_t st, std::string &err) {
    destroy();
    n = A->n;
    bkind = b_kind;
    nnzA = A->nnz;
    const gcge_csr *Bc = (b_kind == GCGE_B_CSR) ? (const gcge_csr *)B : nullptr;
    nnzB = Bc ? Bc->nnz : 0;
    std::vector<int32_t> arp(n + 1), aci(nnzA), brp, bci;
    hipError_t e;
#define GCGE_HIP(expr)                                                       \
    do {                                                                     \
        e = (expr);                                                          \
        if (e != hipSuccess) {                                               \
            err = std::string(#expr) + ": " + hipGetErrorString(e);         \
            return e == hipErrorOutOfMemory ? GCGE_ERR_OOM : GCGE_ERR_HIP;   \
        }                                                                    \
    } while (0)
    GCGE_HIP(hipMemcpy(arp.data(), A->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
    if (nnzA) GCGE_HIP(hipMemcpy(aci.data(), A->colind, sizeof(int32_t) * nnzA, hipMemcpyDeviceToHost));
    if (!check_pattern(n, nnzA, arp, aci, err, "A")) return GCGE_ERR_INVALID_ARG;
    if (Bc) {
        if (Bc->n != n) {
            err = "B must have the dimension of A";
            return GCGE_ERR_INVALID_ARG;
        }
        brp.resize(n + 1);
        bci.resize(nnzB);
        GCGE_HIP(hipMemcpy(brp.data(), Bc->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
        if (nnzB) GCGE_HIP(hipMemcpy(bci.data(), Bc->colind, sizeof(int32_t) * nnzB, hipMemcpyDeviceToHost));
        if (!check_pattern(n, nnzB, brp, bci, err, "B")) return GCGE_ERR_INVALID_ARG;
    }
    // union pattern: A's entries, B's entries (CSR) or the diagonal (identity / diagonal B)
    std::vector<int32_t> urp(n + 1), uci, ma(nnzA), mb(nnzB), dp(n);
    uci.reserve(nnzA + (Bc ? nnzB : n) / 8 + 16);
    urp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t pa = arp[i], ea = arp[i + 1];
        int32_t pb = 0, eb = 0;
        if (Bc) {
            pb = brp[i];
            eb = brp[i + 1];
        }
        bool diag_done = false;
        while (true) {
            int64_t ca = pa < ea ? aci[pa] : INT64_MAX;
            int64_t cb;
            if (Bc) cb = pb < eb ? bci[pb] : INT64_MAX;
            else cb = diag_done ? INT64_MAX : i;
            if (ca == INT64_MAX && cb == INT64_MAX) break;
            const int64_t c = std::min(ca, cb);
            const int32_t pos = (int32_t)uci.size();
            uci.push_back((int32_t)c);
            if (ca == c) ma[pa++] = pos;
            if (cb == c) {
                if (Bc) mb[pb++] = pos;
                else diag_done = true;
            }
            if (c == i) dp[i] = pos;
        }
        if ((int64_t)uci.size() > INT32_MAX) {
            err = "union pattern has more than 2^31 entries";
            return GCGE_ERR_INVALID_ARG;
        }
        urp[i + 1] = (int32_t)uci.size();
    }
    nnz = (int64_t)uci.size();
    same_pattern = (nnz == nnzA) && (!Bc || nnz == nnzB);
    GCGE_HIP(hipMalloc((void **)&rowptr, sizeof(int32_t) * (n + 1)));
    GCGE_HIP(hipMalloc((void **)&colind, sizeof(int32_t) * std::max<int64_t>(nnz, 1)));
    GCGE_HIP(hipMemcpy(rowptr, urp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
    if (nnz) GCGE_HIP(hipMemcpy(colind, uci.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
    GCGE_HIP(hipMalloc((void **)&mapA, sizeof(int32_t) * std::max<int64_t>(nnzA, 1)));
    if (nnzA) GCGE_HIP(hipMemcpy(mapA, ma.data(), sizeof(int32_t) * nnzA, hipMemcpyHostToDevice));
    if (Bc) {
        GCGE_HIP(hipMalloc((void **)&mapB, sizeof(int32_t) * std::max<int64_t>(nnzB, 1)));
        if (nnzB) GCGE_HIP(hipMemcpy(mapB, mb.data(), sizeof(int32_t) * nnzB, hipMemcpyHostToDevice));
    } else {
        GCGE_HIP(hipMalloc((void **)&dpos, sizeof(int32_t) * n));
        GCGE_HIP(hipMemcpy(dpos, dp.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    }
    {
        const std::vector<int32_t> uo = spmm_unit_order(n, urp.data(), uci.data(), &plane);
        if (!uo.empty()) {
            GCGE_HIP(hipMalloc((void **)&uorder, sizeof(int32_t) * uo.size()));
            GCGE_HIP(hipMemcpy(uorder, uo.data(), sizeof(int32_t) * uo.size(), hipMemcpyHostToDevice));
        }
    }
    GCGE_HIP(hipMalloc((void **)&a, sizeof(double) * std::max<int64_t>(nnz, 1)));
    if (Bc) GCGE_HIP(hipMalloc((void **)&b, sizeof(double) * std::max<int64_t>(nnz, 1)));
    if (b_kind == GCGE_B_DIAG) GCGE_HIP(hipMalloc((void **)&dg, sizeof(double) * n));
    const void *bv = nullptr;
    if (b_kind == GCGE_B_DIAG) bv = B;
    if (Bc) bv = Bc->val;
    int rc = set_values(A->val, bv, st, err);
#undef GCGE_HIP
    return rc;
}

int Operator::set_values(const double *a_val, const void *b_val, hipStream_t st, std::string &err) {
    hipError_t e = hipSuccess;
    if (a_val) {
        if (nnz) e = hipMemsetAsync(a, 0, sizeof(double) * nnz, st);
        if (e == hipSuccess) e = scatter_values(nnzA, mapA, a_val, a, st);
    }
    if (e == hipSuccess && b_val) {
        if (bkind == GCGE_B_CSR) {
            if (nnz) e = hipMemsetAsync(b, 0, sizeof(double) * nnz, st);
            if (e == hipSuccess) e = scatter_values(nnzB, mapB, (const double *)b_val, b, st);
        } else if (bkind == GCGE_B_DIAG) {
            e = hipMemcpyAsync(dg, b_val, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        err = std::string("operator values: ") + hipGetErrorString(e);
        return GCGE_ERR_HIP;
    }
    return GCGE_OK;
}

void Operator::destroy() {
    int32_t *ip[] = {rowptr, colind, dpos, mapA, mapB, uorder};
    for (auto p : ip)
        if (p) (void)hipFree(p);
    uorder = nullptr;
    plane = 0;
    double *dp[] = {a, b, dg};
    for (auto p : dp)
        if (p) (void)hipFree(p);
    rowptr = colind = dpos = mapA = mapB = nullptr;
    a = b = dg = nullptr;
    n = nnz = nnzA = nnzB = 0;
}

hipError_t Operator::shifted(double theta, double *m, float *m32, hipStream_t st) const {
    if (bkind == GCGE_B_CSR) return shift_values(nnz, a, b, n, nullptr, nullptr, theta, m, m32, st);
    return shift_values(nnz, a, nullptr, n, dpos, (bkind == GCGE_B_DIAG) ? dg : nullptr, theta, m, m32, st);
}

hipError_t bop_apply(const BOp &B, int64_t n, const double *X, int64_t ldx, int k, double *Y, int64_t ldy,
                     hipStream_t st) {
    if (B.kind == GCGE_B_IDENTITY) return copy_cols<double, double>(n, k, X, ldx, Y, ldy, nullptr, st);
    if (B.kind == GCGE_B_DIAG) return scale_rows(n, k, B.dg, X, ldx, Y, ldy, st);
    for (int c0 = 0; c0 < k; c0 += 128) {
        const int kk = std::min(128, k - c0);
        GCGE_TRY(spmm<double>(B.csr, nullptr, nullptr, nullptr, 0, 0, X + c0, ldx, kk, Y + c0, ldy, nullptr, 0,
                              nullptr, nullptr, st));
    }
    return hipSuccess;
}

hipError_t Operator::apply_b(const double *X, int64_t ldx, int k, double *Y, int64_t ldy, hipStream_t st) const {
    return bop_apply(bop(), n, X, ldx, k, Y, ldy, st);
}

hipError_t Operator::residual(const double *X, int64_t ldx, int k, const double *sigma, double *R, int64_t ldr,
                              double *part, int *nparts, hipStream_t st) const {
    DevCsr<double> Ac = A_csr();
    if (bkind == GCGE_B_CSR)
        return spmm<double>(Ac, b, nullptr, sigma, 2, 1, X, ldx, k, R, ldr, nullptr, 0, part, nparts, st);
    return spmm<double>(Ac, nullptr, (bkind == GCGE_B_DIAG) ? dg : nullptr, sigma, 1, 1, X, ldx, k, R, ldr, nullptr,
                        0, part, nparts, st);
}

// ------------------------------------------------------ orthogonalization
namespace {

struct OrthCtx {
    int64_t n;
    const BOp &B;
    double *W;
    int64_t ldw;
    double *BW;   // CSR only
    int64_t ldbw;
    const OrthOptions &opt;
    Workspace &ws;
    Stager &stg;
    hipStream_t st;
    OrthStats *os;
    std::string &err;
    int c;   // leaf size

    bool csr() const { return B.kind == GCGE_B_CSR; }
    const double *dweight() const { return B.kind == GCGE_B_DIAG ? B.dg : nullptr; }

    int fail(hipError_t e, const char *what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? GCGE_ERR_OOM : GCGE_ERR_HIP;
    }

    // C (host, m x k) = X^T Y with Y already B-applied (CSR) or weighted by d
    int gram_host(const Segs &X, const double *Y, int64_t ldy, int k, bool yB, std::vector<double> &C) {
        const int m = X.total();
        C.assign((size_t)m * k, 0.0);
        if (m == 0 || k == 0) return GCGE_OK;
        hipError_t e = ws.ensure_small(sizeof(double) * ((size_t)m * k + 64));
        if (e != hipSuccess) return fail(e, "workspace");
        e = gram(n, X, Y, ldy, k, yB ? nullptr : dweight(), ws.small, k, ws, st);
        if (e != hipSuccess) return fail(e, "gram");
        e = stg.download(C.data(), ws.small, sizeof(double) * m * k);
        if (e != hipSuccess) return fail(e, "download");
        if (os) os->grams++;
        return GCGE_OK;
    }

    // Y = alpha X S + beta Y with S host (m x k)
    int gemm_host(const Segs &X, const std::vector<double> &S, int k, double alpha, double beta, double *Y,
                  int64_t ldy) {
        const int m = X.total();
        if (m == 0 || k == 0) return GCGE_OK;
        // S goes to the second half of the small workspace (the first half holds Gram results)
        hipError_t e = ws.ensure_small(sizeof(double) * (2 * (size_t)m * k + 64));
        if (e != hipSuccess) return fail(e, "workspace");
        double *Sd = ws.small + (size_t)m * k + 32;
        e = stg.upload(Sd, S.data(), sizeof(double) * m * k);
        if (e != hipSuccess) return fail(e, "upload");
        e = gemm(n, X, Sd, k, k, alpha, beta, Y, ldy, st);
        if (e != hipSuccess) return fail(e, "gemm");
        return GCGE_OK;
    }

    // B-norms of columns [s, s+k) (host)
    int bnorms(int s, int k, std::vector<double> &nu) {
        Segs X;
        X.add(W + s, ldw, k);
        std::vector<double> C;
        int rc = csr() ? gram_host(X, BW + s, ldbw, k, true, C) : gram_host(X, W + s, ldw, k, false, C);
        if (rc) return rc;
        nu.resize(k);
        for (int j = 0; j < k; ++j) nu[j] = std::sqrt(std::max(C[(size_t)j * k + j], 0.0));
        return GCGE_OK;
    }

    int refresh_bw(int s, int k) {
        if (!csr() || k == 0) return GCGE_OK;
        hipError_t e = bop_apply(B, n, W + s, ldw, k, BW + s, ldbw, st);
        return e == hipSuccess ? GCGE_OK : fail(e, "B W");
    }

    // keep the columns [s, s+k) with flag set, compacting them to the front
    int compact(int s, int k, const std::vector<char> &keep, int *kept) {
        int dst = 0;
        int j = 0;
        while (j < k) {
            if (!keep[j]) {
                ++j;
                continue;
            }
            int j2 = j;
            while (j2 < k && keep[j2]) ++j2;
            if (dst != j) {
                hipError_t e = shift_cols_left(n, W + s, ldw, dst, j, j2 - j, st);
                if (e == hipSuccess && csr()) e = shift_cols_left(n, BW + s, ldbw, dst, j, j2 - j, st);
                if (e != hipSuccess) return fail(e, "compact");
            }
            dst += j2 - j;
            j = j2;
        }
        *kept = dst;
        if (os) os->dropped += k - dst;
        return GCGE_OK;
    }

    // scale columns [s, s+k) to unit B-norm, dropping those with nu^2 <= thr
    int normalize(int s, int k, double thr, int *kept) {
        std::vector<double> nu;
        int rc = bnorms(s, k, nu);
        if (rc) return rc;
        std::vector<char> keep(k);
        std::vector<double> sc(k);
        for (int j = 0; j < k; ++j) {
            keep[j] = nu[j] * nu[j] > thr && std::isfinite(nu[j]);
            sc[j] = keep[j] ? 1.0 / nu[j] : 0.0;
        }
        hipError_t e = ws.ensure_colvec(sizeof(double) * (k + 8));
        if (e != hipSuccess) return fail(e, "workspace");
        e = stg.upload(ws.colvec, sc.data(), sizeof(double) * k);
        if (e == hipSuccess) e = copy_cols<double, double>(n, k, W + s, ldw, W + s, ldw, ws.colvec, st);
        if (e == hipSuccess && csr()) e = copy_cols<double, double>(n, k, BW + s, ldbw, BW + s, ldbw, ws.colvec, st);
        if (e != hipSuccess) return fail(e, "scale");
        return compact(s, k, keep, kept);
    }

    // Algorithm 2 on columns [0, k): blocks of b consecutive columns; inside a
    // block each column is B-orthogonalized against the block's kept columns
    // by Gram-Schmidt (two passes, one reduction each: the coefficients and
    // the column's own squared B-norm, the norm after the projection following
    // by Pythagoras), normalized or dropped (squared B-norm ratio at most
    // drop_tol), then the block's kept columns are deflated from all later
    // columns (repeated until the coefficients are small).  Kept columns are
    // moved to the front as they are accepted.
    int mbo(int k, int b, int *kept) {
        int out = 0, cur = 0;
        hipError_t e = ws.ensure_colvec(sizeof(double) * 16);
        if (e != hipSuccess) return fail(e, "workspace");
        while (cur < k) {
            const int blk_end = std::min(cur + b, k);
            const int bs0 = out;
            for (int j = cur; j < blk_end; ++j) {
                // one reduction per pass: [U, w]^T B w gives the coefficients
                // against the block's kept columns U and the squared B-norm of w
                double nrm0 = 0.0, nrm = 0.0;
                for (int pass = 0; pass < 2; ++pass) {
                    const int nu = out - bs0;
                    Segs X;
                    std::vector<double> c;
                    int rc;
                    if (csr()) {
                        X.add(BW + bs0, ldbw, nu);
                        X.add(BW + j, ldbw, 1);
                    } else {
                        X.add(W + bs0, ldw, nu);
                        X.add(W + j, ldw, 1);
                    }
                    rc = gram_host(X, W + j, ldw, 1, csr(), c);
                    if (rc) return rc;
                    double cc = 0.0;
                    for (int i = 0; i < nu; ++i) cc += c[i] * c[i];
                    if (pass == 0) nrm0 = c[nu];
                    nrm = c[nu] - cc;   // squared B-norm after this pass's projection
                    if (nu == 0) break;
                    c.resize(nu);
                    Segs Uw;
                    Uw.add(W + bs0, ldw, nu);
                    rc = gemm_host(Uw, c, 1, -1.0, 1.0, W + j, ldw);
                    if (rc) return rc;
                    if (csr()) {
                        Segs Ub;
                        Ub.add(BW + bs0, ldbw, nu);
                        rc = gemm_host(Ub, c, 1, -1.0, 1.0, BW + j, ldbw);
                        if (rc) return rc;
                    }
                }
                // columns enter with unit B-norm (normalized after the deflation
                // against Q), so the squared norm left is compared with drop_tol
                // itself: a column that the deflations of earlier blocks reduced
                // to rounding is dependent too
                const bool keep = nrm0 > 0.0 && std::isfinite(nrm) && nrm > opt.drop_tol;
                if (!keep) {
                    if (os) os->dropped++;
                    continue;
                }
                const double sc = 1.0 / std::sqrt(nrm);
                e = stg.upload(ws.colvec, &sc, sizeof(double));
                if (e == hipSuccess) e = copy_cols<double, double>(n, 1, W + j, ldw, W + out, ldw, ws.colvec, st);
                if (e == hipSuccess && csr()) e = copy_cols<double, double>(n, 1, BW + j, ldbw, BW + out, ldbw, ws.colvec, st);
                if (e != hipSuccess) return fail(e, "normalize");
                ++out;
            }
            const int nb = out - bs0, nr = k - blk_end;
            if (nb > 0 && nr > 0) {
                for (int pass = 0; pass < opt.max_pass; ++pass) {
                    Segs X1;
                    std::vector<double> R;
                    int rc;
                    if (csr()) {
                        X1.add(BW + bs0, ldbw, nb);
                        rc = gram_host(X1, W + blk_end, ldw, nr, true, R);
                    } else {
                        X1.add(W + bs0, ldw, nb);
                        rc = gram_host(X1, W + blk_end, ldw, nr, false, R);
                    }
                    if (rc) return rc;
                    double rmax = 0.0;
                    for (double v : R) rmax = std::max(rmax, std::fabs(v));
                    Segs W1;
                    W1.add(W + bs0, ldw, nb);
                    rc = gemm_host(W1, R, nr, -1.0, 1.0, W + blk_end, ldw);
                    if (rc) return rc;
                    if (csr()) {
                        Segs B1;
                        B1.add(BW + bs0, ldbw, nb);
                        rc = gemm_host(B1, R, nr, -1.0, 1.0, BW + blk_end, ldbw);
                        if (rc) return rc;
                    }
                    if (rmax <= opt.orth_tol) break;
                }
            }
            cur = blk_end;
        }
        *kept = out;
        return GCGE_OK;
    }

    // Algorithm 3 on columns [s, e); returns kept count via *kept
    int rec(int s, int e, int *kept) {
        const int len = e - s;
        if (len <= 0) {
            *kept = 0;
            return GCGE_OK;
        }
        if (len <= c) {
            int k = len;
            for (int pass = 0; pass < opt.max_pass && k > 0; ++pass) {
                Segs X;
                X.add(W + s, ldw, k);
                std::vector<double> M;
                int rc = csr() ? gram_host(X, BW + s, ldbw, k, true, M) : gram_host(X, W + s, ldw, k, false, M);
                if (rc) return rc;
                for (int i = 0; i < k; ++i)
                    for (int j = i + 1; j < k; ++j) M[i * k + j] = M[j * k + i] = 0.5 * (M[i * k + j] + M[j * k + i]);
                std::vector<double> lam(k), Q((size_t)k * k);
                if (jacobi_small(k, M.data(), lam.data(), Q.data()) != 0) {
                    err = "leaf eigensolve did not converge";
                    return GCGE_ERR_INTERNAL;
                }
                int kk = 0;
                double dev = 0.0;
                std::vector<int> keepc;
                for (int j = 0; j < k; ++j)
                    if (lam[j] > opt.drop_tol && std::isfinite(lam[j])) keepc.push_back(j);
                kk = (int)keepc.size();
                std::vector<double> S((size_t)k * std::max(kk, 1));
                for (int q = 0; q < kk; ++q) {
                    const int j = keepc[q];
                    dev = std::max(dev, std::fabs(lam[j] - 1.0));
                    const double isq = 1.0 / std::sqrt(lam[j]);
                    for (int i = 0; i < k; ++i) S[(size_t)i * kk + q] = Q[(size_t)i * k + j] * isq;
                }
                if (opt.skip_final && kk == k && dev <= opt.orth_tol) break;   // already orthonormal
                if (os) os->dropped += k - kk;
                if (kk > 0) {
                    rc = gemm_host(X, S, kk, 1.0, 0.0, W + s, ldw);
                    if (rc) return rc;
                    if (csr()) {
                        Segs XB;
                        XB.add(BW + s, ldbw, k);
                        rc = gemm_host(XB, S, kk, 1.0, 0.0, BW + s, ldbw);
                        if (rc) return rc;
                    }
                }
                k = kk;
                if (dev <= opt.orth_tol) break;
            }
            *kept = k;
            return GCGE_OK;
        }
        const int h = len / 2;
        int k1 = 0, k2 = 0;
        int rc = rec(s, s + h, &k1);
        if (rc) return rc;
        const int s2 = s + h, l2 = e - s2;
        if (k1 > 0) {
            for (int pass = 0; pass < opt.max_pass; ++pass) {
                Segs X1;
                std::vector<double> R;
                if (csr()) {
                    X1.add(BW + s, ldbw, k1);
                    rc = gram_host(X1, W + s2, ldw, l2, true, R);
                } else {
                    X1.add(W + s, ldw, k1);
                    rc = gram_host(X1, W + s2, ldw, l2, false, R);
                }
                if (rc) return rc;
                double rmax = 0.0;
                for (double v : R) rmax = std::max(rmax, std::fabs(v));
                if (opt.skip_final && rmax <= opt.orth_tol) break;
                Segs W1;
                W1.add(W + s, ldw, k1);
                rc = gemm_host(W1, R, l2, -1.0, 1.0, W + s2, ldw);
                if (rc) return rc;
                if (csr()) {
                    Segs B1;
                    B1.add(BW + s, ldbw, k1);
                    rc = gemm_host(B1, R, l2, -1.0, 1.0, BW + s2, ldbw);
                    if (rc) return rc;
                }
                if (rmax <= opt.orth_tol) break;
            }
        }
        rc = rec(s2, e, &k2);
        if (rc) return rc;
        if (k1 < h && k2 > 0) {
            hipError_t ee = shift_cols_left(n, W, ldw, s + k1, s2, k2, st);
            if (ee == hipSuccess && csr()) ee = shift_cols_left(n, BW, ldbw, s + k1, s2, k2, st);
            if (ee != hipSuccess) return fail(ee, "compact");
        }
        *kept = k1 + k2;
        return GCGE_OK;
    }
};

}  // namespace

int orth_block(int64_t n, const BOp &B, const Segs &Q, double *W, int64_t ldw, int k, double *BW, int64_t ldbw,
               const OrthOptions &opt, Workspace &ws, Stager &stg, hipStream_t st, int *kept, OrthStats *os,
               std::string &err) {
    *kept = 0;
    if (k <= 0) return GCGE_OK;
    OrthCtx C{n, B, W, ldw, BW, ldbw, opt, ws, stg, st, os, err, 16};
    int rc = C.refresh_bw(0, k);
    if (rc) return rc;
    int kk = 0;
    rc = C.normalize(0, k, 0.0, &kk);   // exact zero columns only
    if (rc) return rc;
    if (Q.total() > 0 && kk > 0) {
        for (int pass = 0; pass < opt.max_pass && kk > 0; ++pass) {
            std::vector<double> R;
            rc = C.csr() ? C.gram_host(Q, BW, ldbw, kk, true, R) : C.gram_host(Q, W, ldw, kk, false, R);
            if (rc) return rc;
            double rmax = 0.0;
            for (double v : R) rmax = std::max(rmax, std::fabs(v));
            if (opt.skip_final && pass > 0 && rmax <= opt.orth_tol) break;
            rc = C.gemm_host(Q, R, kk, -1.0, 1.0, W, ldw);
            if (rc) return rc;
            rc = C.refresh_bw(0, kk);
            if (rc) return rc;
            if (pass == 0) {
                // columns that were (almost) inside span(Q) are dependent: drop them
                int k2 = 0;
                rc = C.normalize(0, kk, opt.drop_tol, &k2);
                if (rc) return rc;
                kk = k2;
            } else if (rmax <= opt.orth_tol) {
                break;
            }
        }
    }
    if (kk == 0) return GCGE_OK;
    int out = 0;
    if (opt.algorithm == 2) {
        const int b = opt.mbo_block > 0 ? opt.mbo_block : std::max(1, std::min(kk / 4, 200));
        rc = C.mbo(kk, b, &out);
    } else {
        C.c = std::min(kk, 16);
        rc = C.rec(0, kk, &out);
    }
    if (rc) return rc;
    *kept = out;
    return GCGE_OK;
}

}  // namespace gcge
