// Operator setup (union pattern, shifted values), host<->device staging, and
// the B-orthogonalization of STEP 2: block Gram-Schmidt against the already
// B-orthonormal [X, P] followed by RecursiveOrthSVD (Algorithm 3).
#include "operator.h"

#include <algorithm>
#include <chrono>
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
// Waits for the stream: polls it for up to 100 us (a short download is back
// well before a blocking wait would wake up, tens of microseconds after the
// copy), then blocks, so that a long phase (an inner CG solve) does not keep
// a host core spinning.
static hipError_t spin_wait(hipStream_t st) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipStreamQuery(st);
        if (e != hipErrorNotReady) return e;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(100)) return hipStreamSynchronize(st);
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
    std::vector<int32_t> urp(n + 1), uci, ma(nnzA), mb(nnzB), dp(n, -1);   // dp: -1 = no stored diagonal
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
    }
    GCGE_HIP(hipMalloc((void **)&dpos, sizeof(int32_t) * n));
    GCGE_HIP(hipMemcpy(dpos, dp.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
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
        return e == hipErrorOutOfMemory ? GCGE_ERR_OOM : GCGE_ERR_HIP;
    }
    return GCGE_OK;
}

int Operator::check_b_positive(hipStream_t st, std::string &err) const {
    if (bkind == GCGE_B_IDENTITY) return GCGE_OK;
    int bad = (int)n;
    int *dbad = nullptr;
    hipError_t e = hipMalloc((void **)&dbad, sizeof(int));
    if (e == hipSuccess) e = first_nonpositive_diag(n, dpos, bkind == GCGE_B_CSR ? b : nullptr,
                                                    bkind == GCGE_B_DIAG ? dg : nullptr, dbad, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, dbad, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (dbad) (void)hipFree(dbad);
    if (e != hipSuccess) {
        err = std::string("B check: ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? GCGE_ERR_OOM : GCGE_ERR_HIP;
    }
    if (bad < n) {
        err = "B is not positive definite: its diagonal entry in row " + std::to_string(bad) +
              (bkind == GCGE_B_CSR ? " is missing, not positive or not finite" : " is not positive or not finite");
        return GCGE_ERR_NOT_SPD;
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

// STEP 2 as one enqueued sequence: every pass of every loop of the
// deflation against [X, P] and of Algorithm 3 (or 2) is launched by the host
// up front (at most max_pass per loop); the stopping tests and the drop
// decisions run on the device and gate the later launches (orth_pass_test,
// orth_leaf, orth_norm_scale write the flags; gram, gemm, copy_cols and the B
// product read them).  A dropped direction becomes a zero column in place, so
// every launch has a size known on the host; orth_finish moves the kept
// columns to the front at the end, and the kept count is the one value the
// host waits for.
struct DevOrth {
    int64_t n;
    const BOp &B;
    double *W;
    int64_t ldw;
    double *BW;   // CSR only: B W, kept in step with W
    int64_t ldbw;
    int k;        // columns of W (fixed; dropped ones are zero)
    const OrthOptions &opt;
    Workspace &ws;
    hipStream_t st;
    std::string &err;
    int *ints = nullptr;        // device flags (layout in internal.h)
    double *G = nullptr;        // k x k, and the mq x k coefficients against Q
    double *Ml = nullptr;       // leaf Gram (<= 16 x 16)
    double *Sl = nullptr;       // leaf transform (<= 16 x 16)
    double *Rn = nullptr;       // node / block coefficients (<= k x k), Algorithm 2 column coefficients
    double *scale = nullptr;    // per-column scales (k)
    double *state = nullptr;    // Algorithm 2 norms (2)
    int nloops = 0, next_loop = 0;
    int grams = 0;
    hipError_t e = hipSuccess;  // first launch error

    bool csr() const { return B.kind == GCGE_B_CSR; }
    const double *dweight() const { return B.kind == GCGE_B_DIAG ? B.dg : nullptr; }
    int *loop(int i) { return orth_loop(ints, k, i); }
    int new_loop() { return next_loop++; }
    void chk(hipError_t r) {
        if (e == hipSuccess) e = r;
    }

    // C = X^T B Y for X = W (or BW for CSR when bx) columns [xs, xs + m) and
    // Y = W columns [ys, ys + kk); ldc = kk
    void gram_w(int xs, int m, int ys, int kk, double *C, const int *go) {
        if (m <= 0 || kk <= 0) return;
        Segs X;
        if (csr()) X.add(BW + xs, ldbw, m);
        else X.add(W + xs, ldw, m);
        chk(gram(n, X, W + ys, ldw, kk, csr() ? nullptr : dweight(), C, kk, ws, st, go));
        ++grams;
    }
    // the leaf / norm Gram X^T B X with Y = B X for CSR (X = W columns [s, s + m))
    void gram_self(int s, int m, double *C, const int *go) {
        Segs X;
        X.add(W + s, ldw, m);
        if (csr()) chk(gram(n, X, BW + s, ldbw, m, nullptr, C, m, ws, st, go));
        else chk(gram(n, X, W + s, ldw, m, dweight(), C, m, ws, st, go));
        ++grams;
    }
    // W[:, ys..ys+kk) (and BW) = alpha W[:, xs..xs+m) S + beta (same)
    void update(int xs, int m, const double *S, int64_t lds, int ys, int kk, double alpha, double beta,
                const int *go) {
        if (m <= 0 || kk <= 0) return;
        Segs X;
        X.add(W + xs, ldw, m);
        chk(gemm(n, X, S, lds, kk, alpha, beta, W + ys, ldw, st, go));
        if (csr()) {
            Segs XB;
            XB.add(BW + xs, ldbw, m);
            chk(gemm(n, XB, S, lds, kk, alpha, beta, BW + ys, ldbw, st, go));
        }
    }
    // BW = B W for columns [0, k) (CSR only)
    void refresh_bw(const int *go) {
        if (!csr()) return;
        for (int c0 = 0; c0 < k; c0 += 128) {
            Affine<double> af;   // y = 0 - (-1) (B x)
            af.ws = -1.0;
            chk(spmm_affine<double>(B.csr, W + c0, ldw, std::min(128, k - c0), BW + c0, ldbw, af, st, nullptr, 0,
                                    nullptr, nullptr, go));
        }
    }
    // unit B-norm columns; those with squared norm <= thr are dropped
    void normalize(double thr, const int *go) {
        gram_self(0, k, G, go);
        chk(orth_norm_scale(G, k, k, thr, ints, scale, go, st));
        chk(copy_cols<double, double>(n, k, W, ldw, W, ldw, scale, st, go));
        if (csr()) chk(copy_cols<double, double>(n, k, BW, ldbw, BW, ldbw, scale, st, go));
    }

    // repeat R = Q^T B W, W -= Q R until small; after the first pass the
    // columns that lay in span(Q) are dropped and the rest renormalized
    void deflate(const Segs &Q) {
        const int mq = Q.total();
        const int L = new_loop();
        for (int pass = 0; pass < opt.max_pass; ++pass) {
            int *lp = loop(L);
            chk(gram(n, Q, csr() ? BW : W, csr() ? ldbw : ldw, k, csr() ? nullptr : dweight(), G, k, ws, st, lp));
            ++grams;
            chk(orth_pass_test(G, mq, k, k, opt.orth_tol, opt.skip_final && pass > 0, pass > 0, lp, st));
            chk(gemm(n, Q, G, k, k, -1.0, 1.0, W, ldw, st, lp + 1));
            refresh_bw(lp + 1);
            if (pass == 0) normalize(opt.drop_tol, lp + 1);
        }
    }

    // Algorithm 3 on columns [s, e)
    void rec(int s, int e, int c) {
        const int len = e - s;
        if (len <= 0) return;
        if (len <= c) {
            const int L = new_loop();
            for (int pass = 0; pass < opt.max_pass; ++pass) {
                int *lp = loop(L);
                gram_self(s, len, Ml, lp);
                chk(orth_leaf(Ml, len, opt.drop_tol, opt.orth_tol, opt.skip_final ? 1 : 0, ints, s, Sl, lp, st));
                update(s, len, Sl, len, s, len, 1.0, 0.0, lp + 1);
            }
            return;
        }
        const int s2 = s + len / 2, l2 = e - s2;
        rec(s, s2, c);
        const int L = new_loop();
        for (int pass = 0; pass < opt.max_pass; ++pass) {
            int *lp = loop(L);
            gram_w(s, s2 - s, s2, l2, Rn, lp);
            chk(orth_pass_test(Rn, s2 - s, l2, l2, opt.orth_tol, opt.skip_final ? 1 : 0, 1, lp, st));
            update(s, s2 - s, Rn, l2, s2, l2, -1.0, 1.0, lp + 1);
        }
        rec(s2, e, c);
    }

    // Algorithm 2 on columns [0, k): blocks of b columns; inside a block each
    // column is B-orthogonalized against the block's earlier columns by
    // Gram-Schmidt (two passes, one reduction each: the coefficients and the
    // column's own squared B-norm, the norm after the projection following by
    // Pythagoras), normalized or dropped (squared B-norm after the projection
    // at most drop_tol; the columns enter with unit B-norm), then the block is
    // deflated from all later columns (repeated until the coefficients are small)
    void mbo(int b) {
        double *cvec = Rn + (size_t)k * k;   // (nu + 1) coefficients of one column
        for (int cur = 0; cur < k; cur += b) {
            const int blk_end = std::min(cur + b, k);
            for (int j = cur; j < blk_end; ++j) {
                const int nu = j - cur;
                for (int pass = 0; pass < 2; ++pass) {
                    Segs X;
                    if (csr()) {
                        X.add(BW + cur, ldbw, nu);
                        X.add(BW + j, ldbw, 1);
                    } else {
                        X.add(W + cur, ldw, nu);
                        X.add(W + j, ldw, 1);
                    }
                    chk(gram(n, X, W + j, ldw, 1, csr() ? nullptr : dweight(), cvec, 1, ws, st));
                    ++grams;
                    chk(orth_mbo_coef(cvec, nu, pass, state, st));
                    update(cur, nu, cvec, 1, j, 1, -1.0, 1.0, nullptr);
                }
                chk(orth_mbo_keep(state, opt.drop_tol, ints, j, scale + j, st));
                chk(copy_cols<double, double>(n, 1, W + j, ldw, W + j, ldw, scale + j, st));
                if (csr()) chk(copy_cols<double, double>(n, 1, BW + j, ldbw, BW + j, ldbw, scale + j, st));
            }
            const int nb = blk_end - cur, nr = k - blk_end;
            if (nr <= 0) continue;
            const int L = new_loop();
            for (int pass = 0; pass < opt.max_pass; ++pass) {
                int *lp = loop(L);
                gram_w(cur, nb, blk_end, nr, Rn, lp);
                chk(orth_pass_test(Rn, nb, nr, nr, opt.orth_tol, 0, 1, lp, st));
                update(cur, nb, Rn, nr, blk_end, nr, -1.0, 1.0, lp + 1);
            }
        }
    }
};

}  // namespace

int orth_block(int64_t n, const BOp &B, const Segs &Q, double *W, int64_t ldw, int k, double *BW, int64_t ldbw,
               const OrthOptions &opt, Workspace &ws, Stager &stg, hipStream_t st, int *kept, OrthStats *os,
               std::string &err) {
    *kept = 0;
    if (k <= 0) return GCGE_OK;
    DevOrth D{n, B, W, ldw, BW, ldbw, k, opt, ws, st, err};
    const int mq = Q.total();
    const int b2 = opt.mbo_block > 0 ? std::min(opt.mbo_block, k) : std::max(1, std::min(k / 4, 200));
    D.nloops = 1 + (opt.algorithm == 2 ? (k + b2 - 1) / b2 : 2 * k);
    // device state: coefficient blocks, then the flags
    const size_t big = (size_t)std::max(mq, k) * k;
    const size_t kr = ((size_t)k + 31) / 32 * 32;
    const size_t ndbl = big + 256 + 256 + (size_t)k * k + kr + kr + 8;
    const size_t nint = ORTH_ALIVE + k + 2 * (size_t)D.nloops;
    // the Gram partials are sized for the largest product once, so that no
    // buffer is reallocated while the sequence below is in flight
    hipError_t e = ws.ensure_orth(ndbl * sizeof(double) + nint * sizeof(int) + 256);
    if (e == hipSuccess) e = ws.ensure_part(gram_part_bytes_max());
    if (e != hipSuccess) {
        err = std::string("workspace: ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? GCGE_ERR_OOM : GCGE_ERR_HIP;
    }
    double *base = reinterpret_cast<double *>(ws.orth);
    D.G = base;
    D.Ml = D.G + big;
    D.Sl = D.Ml + 256;
    D.Rn = D.Sl + 256;                       // k x k, then k Algorithm 2 column coefficients
    D.scale = D.Rn + (size_t)k * k + kr;
    D.state = D.scale + kr;
    D.ints = reinterpret_cast<int *>(D.state + 8);

    D.chk(orth_init(D.ints, k, D.nloops, st));
    D.refresh_bw(nullptr);
    D.normalize(0.0, nullptr);   // exact zero columns only
    if (mq > 0) D.deflate(Q);
    if (opt.algorithm == 2) D.mbo(b2);
    else D.rec(0, k, std::min(k, 16));
    D.chk(orth_finish(n, W, ldw, k, D.ints, st));
    if (D.e != hipSuccess) {
        err = std::string("orthogonalization: ") + hipGetErrorString(D.e);
        return D.e == hipErrorOutOfMemory ? GCGE_ERR_OOM : GCGE_ERR_HIP;
    }
    int kk = 0;
    e = stg.download(&kk, D.ints, sizeof(int));
    if (e != hipSuccess) {
        err = std::string("orthogonalization: ") + hipGetErrorString(e);
        return GCGE_ERR_HIP;
    }
    if (kk < 0 || kk > k) {
        err = "orthogonalization: inconsistent kept count";
        return GCGE_ERR_INTERNAL;
    }
    *kept = kk;
    if (os) {
        os->grams += D.grams;
        os->dropped += k - kk;
    }
    return GCGE_OK;
}

}  // namespace gcge
