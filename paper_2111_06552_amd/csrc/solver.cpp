// GCG eigensolver driver (paper Section 2, Algorithm 1, with the computation
// reductions of Section 3.2 and the moving mechanism of Section 3.3) and the
// C ABI of libgcge.so.
//
// One GCG iteration, in the order the host enqueues it on the solver stream:
//   STEP 4  residuals of the active block X_n, locking of the leading run of
//           converged pairs (they move to the locked block X_c);
//   STEP 5  coefficients phat of the next P (eq. CP_tilde, L2 orthogonalized
//           against xhat) and P = V_u phat;
//   STEP 6  column-wise CG on (A - theta B) delta = R from delta = 0, theta the
//           largest converged eigenvalue (the correction form of the paper's
//           (A - theta B) W = B X (Lambda - theta) from the initial guess X);
//   STEP 2  W = delta B-orthogonalized against [X_c, X_u, P], then
//           RecursiveOrthSVD (Algorithm 3);
//   STEP 3  AW, G = [X_u, P, W]^T A W, the structured Abar
//           [[Lambda_u, 0, a1], [0, a0, a2], [a1^T, a2^T, a3]] with
//           a0 = phat^T Abar_old phat, its smallest eigenpairs, and the Ritz
//           rotation X_u <- V_u xhat (all eigenpairs at a move).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "gcge.h"
#include "internal.h"
#include "operator.h"

using namespace gcge;

namespace {

thread_local std::string g_thread_err;

int hip_status(hipError_t e) { return e == hipErrorOutOfMemory ? GCGE_ERR_OOM : GCGE_ERR_HIP; }

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

struct Buffers {
    std::vector<void *> allocs;
    hipError_t alloc(void **p, size_t bytes) {
        hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
        if (e == hipSuccess) allocs.push_back(*p);
        return e;
    }
    void release() {
        for (void *p : allocs) (void)hipFree(p);
        allocs.clear();
    }
};

// Device time of selected launches, bracketed by HIP events on the launch
// stream (option "profile").  Events come from a reusable pool; the elapsed
// times are read once at the end of a solve.
struct KProf {
    bool on = false;
    int64_t full_cols = -1;   // CG launches over this many columns are also summed separately
    std::vector<hipEvent_t> pool;
    size_t next = 0;
    struct Mark {
        int cls, b, e;
        int64_t cols;
    };
    std::vector<Mark> marks;
    int record(hipStream_t st) {
        if (next == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            pool.push_back(e);
        }
        const int i = (int)next++;
        if (hipEventRecord(pool[i], st) != hipSuccess) return -1;
        return i;
    }
    int begin(hipStream_t st) { return on ? record(st) : -1; }
    void end(int cls, int b, int64_t cols, hipStream_t st) {
        if (!on || b < 0) return;
        const int e = record(st);
        if (e >= 0) marks.push_back(Mark{cls, b, e, cols});
    }
    void finish(gcge_stats &S) {
        for (const Mark &m : marks) {
            float ms = 0.f;
            if (hipEventSynchronize(pool[m.e]) == hipSuccess && hipEventElapsedTime(&ms, pool[m.b], pool[m.e]) == hipSuccess) {
                S.prof_ms[m.cls] += ms;
                S.prof_launches[m.cls] += 1;
                S.prof_columns[m.cls] += m.cols;
                if (m.cls < 3 && m.cols == full_cols) {
                    S.prof_full_ms[m.cls] += ms;
                    S.prof_full_launches[m.cls] += 1;
                }
            }
        }
        marks.clear();
        next = 0;
    }
    void release() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
        marks.clear();
        next = 0;
    }
};

// Column-wise CG driver shared by the solver and gcge_cg.  With a
// search-direction history (hist_slots >= 2 slots of n x ld vectors at hist,
// alpha rows at hist_alpha) the directions go to the ring and x is formed by
// cg_fold (before a slot still needed would be overwritten, and at the end)
// instead of an update of x in every step; the results are the same to the
// bit.
template <typename T>
struct CgRunner {
    int64_t n;
    Workspace &ws;
    hipStream_t st;
    int *pinned_flag;
    hipEvent_t ev;
    std::string &err;
    KProf *prof = nullptr;
    T *hist = nullptr;
    int hist_slots = 0;
    T *hist_alpha = nullptr;

    static constexpr int ASTRIDE = 128;   // alpha row stride of the history
    bool lazy(int k, int64_t ld) const {
        return hist != nullptr && hist_alpha != nullptr && cg_hist_ok<T>(n, k, ld, hist_slots);
    }
    T *slot(int j, int64_t ld) const { return hist + (size_t)(j % hist_slots) * n * ld; }
    CgState<T> step_state(CgState<T> cs, int j) const {
        cs.alpha = hist_alpha + (size_t)(j % hist_slots) * ASTRIDE;
        return cs;
    }
    // x (+)= the terms of steps first .. end-1 (class 7 of the profile; its
    // column count is the n-vectors moved: the terms, x written, x read
    // unless init, times k)
    hipError_t fold(T *x, int64_t ld, int k, int first, int end, bool init) {
        const int pb = prof ? prof->begin(st) : -1;
        const hipError_t e = cg_fold<T>(n, k, x, ld, hist, n * ld, hist_slots, hist_alpha, ASTRIDE, first,
                                        end - first, init, st);
        if (prof) prof->end(7, pb, (int64_t)k * (end - first + (init ? 1 : 2)), st);
        return e;
    }

    int run(const DevCsr<T> &M, const double *R, int64_t ldr, const double *rscale, int k, int maxit,
            double rel_tol, T *x, T *r, T *p, T *q, int64_t ld, CgState<T> cs, int64_t *total_its) {
        hipError_t e = ws.ensure_part(sizeof(double) * (size_t)k * max_row_parts() + 256);
        if (e != hipSuccess) return fail(e, "workspace");
        T *part = (T *)ws.part;
        int nparts = 0;
        const bool lz = lazy(k, ld);
        int first = 0;        // first step not yet in x (history)
        bool have_x = false;  // x holds the steps before first
        e = cg_init<T>(R, ldr, rscale, k, n, r, lz ? slot(0, ld) : p, lz ? nullptr : x, ld, part, &nparts, cs, st);
        if (e == hipSuccess) e = cg_init_finish<T>(part, nparts, k, cs, st);
        if (e != hipSuccess) return fail(e, "cg init");
        bool pending = false;
        int it = 0;
        for (; it < maxit; ++it) {
            const CgState<T> ci = lz ? step_state(cs, it) : cs;
            T *pc = lz ? slot(it, ld) : p;
            int pb = prof ? prof->begin(st) : -1;
            e = cg_spmm<T>(M, pc, q, ld, k, part, &nparts, ci.flags, st);
            if (prof) prof->end(0, pb, k, st);
            if (e == hipSuccess) e = cg_alpha<T>(part, nparts, k, ci, st);
            pb = prof ? prof->begin(st) : -1;
            if (e == hipSuccess) e = cg_update_r<T>(n, k, q, r, ld, part, &nparts, ci, st);
            if (prof) prof->end(1, pb, k, st);
            if (e == hipSuccess) e = cg_beta<T>(part, nparts, k, rel_tol, ci, st);
            if (lz) {
                // the slot of p_(it+1) still holds p_(it+1-H): fold through this step first
                if (e == hipSuccess && it + 1 - first >= hist_slots) {
                    e = fold(x, ld, k, first, it + 1, !have_x);
                    first = it + 1;
                    have_x = true;
                }
                pb = prof ? prof->begin(st) : -1;
                if (e == hipSuccess) e = cg_update_p<T>(n, k, pc, slot(it + 1, ld), r, ld, ci, st);
                if (prof) prof->end(2, pb, k, st);
            } else {
                pb = prof ? prof->begin(st) : -1;
                if (e == hipSuccess) e = cg_update_xp<T>(n, k, x, p, r, ld, cs, st);
                if (prof) prof->end(2, pb, k, st);
            }
            if (e != hipSuccess) return fail(e, "cg iteration");
            if (pinned_flag != nullptr && (it % 4) == 3) {
                // non-blocking poll of the number of active columns
                if (pending && hipEventQuery(ev) == hipSuccess) {
                    pending = false;
                    if (*pinned_flag == 0) {
                        ++it;
                        break;
                    }
                }
                if (!pending) {
                    e = hipMemcpyAsync(pinned_flag, cs.flags, sizeof(int), hipMemcpyDeviceToHost, st);
                    if (e == hipSuccess) e = hipEventRecord(ev, st);
                    if (e != hipSuccess) return fail(e, "cg poll");
                    pending = true;
                }
            }
        }
        if (lz && (it > first || !have_x)) {
            e = fold(x, ld, k, first, it, !have_x);
            if (e != hipSuccess) return fail(e, "cg iterate");
        }
        if (total_its) *total_its += it;
        return GCGE_OK;
    }
    // Preconditioned CG (M^-1 = the multigrid V-cycle) on M delta = R, delta
    // from 0; same stopping rule as run().  z is one more n x ld vector.
    int run_pcg(const DevCsr<T> &M, Amg &amg, const double *R, int64_t ldr, const double *rscale, int k, int maxit,
                double rel_tol, T *x, T *r, T *p, T *q, T *z, int64_t ld, CgState<T> cs, int64_t *total_its) {
        hipError_t e = ws.ensure_part(sizeof(double) * (size_t)k * max_row_parts() + 256);
        if (e != hipSuccess) return fail(e, "workspace");
        T *part = (T *)ws.part;
        int nparts = 0;
        const bool lz = lazy(k, ld);
        int first = 0;
        bool have_x = false;
        T *p0 = lz ? slot(0, ld) : p;
        e = cg_init<T>(R, ldr, rscale, k, n, r, p0, lz ? nullptr : x, ld, part, &nparts, cs, st);
        if (e == hipSuccess) e = cg_init_finish<T>(part, nparts, k, cs, st);
        if (e != hipSuccess) return fail(e, "pcg init");
        int rc = amg.apply<T>(r, ld, k, z, ld, part, &nparts, st, err);
        if (rc) return rc;
        e = pcg_rz<T>(part, nparts, k, true, cs, st);
        if (e == hipSuccess) e = copy_cols<T, T>(n, k, z, ld, p0, ld, nullptr, st);
        if (e != hipSuccess) return fail(e, "pcg init");
        bool pending = false;
        int it = 0;
        for (; it < maxit; ++it) {
            const CgState<T> ci = lz ? step_state(cs, it) : cs;
            T *pc = lz ? slot(it, ld) : p;
            int pb = prof ? prof->begin(st) : -1;
            e = cg_spmm<T>(M, pc, q, ld, k, part, &nparts, ci.flags, st);
            if (prof) prof->end(0, pb, k, st);
            if (e == hipSuccess) e = cg_alpha<T>(part, nparts, k, ci, st);
            pb = prof ? prof->begin(st) : -1;
            if (e == hipSuccess) e = cg_update_r<T>(n, k, q, r, ld, part, &nparts, ci, st);
            if (prof) prof->end(1, pb, k, st);
            if (e == hipSuccess) e = cg_beta<T>(part, nparts, k, rel_tol, ci, st);
            if (e != hipSuccess) return fail(e, "pcg iteration");
            pb = prof ? prof->begin(st) : -1;
            rc = amg.apply<T>(r, ld, k, z, ld, part, &nparts, st, err, ci.flags);
            if (prof) prof->end(6, pb, k, st);
            if (rc) return rc;
            e = pcg_rz<T>(part, nparts, k, false, ci, st);
            if (lz) {
                if (e == hipSuccess && it + 1 - first >= hist_slots) {
                    e = fold(x, ld, k, first, it + 1, !have_x);
                    first = it + 1;
                    have_x = true;
                }
                pb = prof ? prof->begin(st) : -1;
                if (e == hipSuccess) e = cg_update_p<T>(n, k, pc, slot(it + 1, ld), z, ld, ci, st);
                if (prof) prof->end(2, pb, k, st);
            } else {
                pb = prof ? prof->begin(st) : -1;
                if (e == hipSuccess) e = cg_update_xp<T>(n, k, x, p, z, ld, cs, st);
                if (prof) prof->end(2, pb, k, st);
            }
            if (e != hipSuccess) return fail(e, "pcg iteration");
            // A preconditioned iteration is long and few are needed: after
            // queuing an iteration, wait for the count of active columns copied
            // after the previous one, so the host stays one iteration ahead and
            // stops right after the last column converges (an iteration queued
            // past that point skips its SpMMs and updates on the device).
            if (pinned_flag != nullptr) {
                if (pending) {
                    e = hipEventSynchronize(ev);
                    if (e != hipSuccess) return fail(e, "pcg poll");
                    pending = false;
                    if (*pinned_flag == 0) {
                        ++it;
                        break;
                    }
                }
                e = hipMemcpyAsync(pinned_flag, cs.flags, sizeof(int), hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipEventRecord(ev, st);
                if (e != hipSuccess) return fail(e, "pcg poll");
                pending = true;
            }
        }
        if (lz && (it > first || !have_x)) {
            e = fold(x, ld, k, first, it, !have_x);
            if (e != hipSuccess) return fail(e, "pcg iterate");
        }
        if (total_its) *total_its += it;
        return GCGE_OK;
    }
    int fail(hipError_t e, const char *what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return hip_status(e);
    }
};

}  // namespace

struct gcge_handle_s {
    Operator op;
    gcge_csr A_user{};
    gcge_csr B_user{};
    const double *d_user = nullptr;
    int nev = 0;
    double tol = 1e-8;
    // options
    int64_t opt_bs = 0, opt_sizex = 0;
    int max_iter = 1000, cg_max_iter = 30, precision = GCGE_PREC_FP64, moving = 0, shift = 1, check = 1;
    int precond = 0, amg_levels = 10, amg_coarse = 512;   // STEP 6 preconditioner (1: multigrid at theta = 0)
    double amg_strength = AMG_STRENGTH;
    Amg amg;
    bool amg_valid = false;
    double amg_setup_ms = 0.0;
    uint64_t seed = 1;
    double cg_rel_tol = 1e-2, orth_tol = 1e-13, drop_tol = 1e-8;
    hipStream_t st = nullptr;
    Workspace ws;
    Stager stg;
    // warm start
    const double *x0 = nullptr;
    int64_t x0_ld = 0;
    int x0_k = 0;
    // buffers (allocated at solve for a configuration)
    Buffers bufs;
    int cfg_bs = -1, cfg_capx = -1, cfg_prec = -1;
    double *Xb[2] = {nullptr, nullptr};
    int64_t ldX = 0;
    double *Xc = nullptr;
    int64_t ldC = 0;
    double *Pb[2] = {nullptr, nullptr};
    double *Wb = nullptr, *AWb = nullptr, *BWb = nullptr, *Rb = nullptr;
    int64_t ldB = 0;
    int64_t ldR = 0;   // R holds 2 ldB columns: after locking c pairs the CG reads R + c
    double *cg64[4] = {nullptr, nullptr, nullptr, nullptr};
    float *cg32[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    void *cgmem = nullptr;
    // inner CG search-direction history (option "cg_history": ring slots,
    // 0 = update the iterate in every step): cghist_slots n x ldB vectors in
    // the CG precision and their alpha rows
    int cg_history = CG_HIST_MAX;
    void *cghist = nullptr, *cghist_alpha = nullptr;
    int cghist_slots = 0, cfg_hist = -1;
    double *mval = nullptr;
    float *mval32 = nullptr;
    double theta_cur = 0.0;
    bool m_valid = false, m32_valid = false;
    int *pinned_flag = nullptr;
    hipEvent_t ev = nullptr;
    int profile = 0;
    KProf prof;
    int dense_eig_opt = 1;
    int orth_alg = 3, orth_block_opt = 0, orth_skip_final = 0;
    DenseEigWork eigw;
    // Rayleigh-Ritz state in device memory (never copied to the host):
    // rr_ab[0] = Abar of the last Rayleigh-Ritz step, rr_ab[1] the one being
    // built; rr_w its Ritz values, rr_xh its coefficient vectors xhat (dim x
    // nwant); rr_ph, rr_a0 = phat and alpha0 = phat^T Abar_old phat of STEP 5;
    // rr_g = [X_u, P, W]^T A W; rr_pt, rr_cf, rr_t, rr_nrm0 = STEP 5 scratch;
    // rr_np = number of phat columns kept.
    double *rr_ab[2] = {nullptr, nullptr};
    double *rr_w = nullptr, *rr_xh = nullptr, *rr_ph = nullptr, *rr_a0 = nullptr, *rr_g = nullptr;
    double *rr_pt = nullptr, *rr_cf = nullptr, *rr_t = nullptr, *rr_nrm0 = nullptr;
    int *rr_np = nullptr;
    int rr_dmax = 0;
    // results of the last solve
    bool have_res = false;         // nev pairs were returned by the last solve
    bool res_converged = false;    // ... and all of them met tol
    std::vector<double> res_lam;   // ascending
    std::vector<int> res_col;      // column of Xc holding the i-th pair
    gcge_stats last{};
    std::string err;

    int fail(int code, const std::string &msg) {
        err = msg;
        return code;
    }
    int hipfail(hipError_t e, const char *what) { return fail(hip_status(e), std::string(what) + ": " + hipGetErrorString(e)); }

    int ensure_buffers(int bs, int capx, int prec, int hist);
    int do_residual(const double *X, int64_t ldx, int k, const double *lam_host, const double *lam_dev, double *R,
                    int64_t ldr, std::vector<double> &rn, std::vector<double> &bn, std::vector<double> *lam_out);
    int do_cg(double theta, const double *R, int64_t ldr, int k, const std::vector<double> &rn, int64_t *cg_its);
    int gram_host(const Segs &X, const double *Y, int64_t ldy, int k, const double *d, std::vector<double> &C);
    int ritz_rotate(const Segs &V, int dim, int nwant, double *Y, int64_t ldy);
    int step5(const Segs &Vold, int dim_old, int nxh_old, int shift, int act_old, int bsa2, double *P, int *launched);
    int solve(double *evals, double *evecs, int64_t ld, gcge_stats *stats);
};

// Ritz pairs of the symmetric dim x dim matrix rr_ab[1] (device, assembled by
// the caller): the nwant smallest eigenvalues into rr_w and their coefficient
// vectors into rr_xh (dim x nwant), and the rotation Y = V xhat.  The
// eigenproblem is solved on the device (dense_eig) unless the option dense_eig
// is 0 or dim exceeds DENSE_EIG_MAX; then Abar goes to the host solver and
// its results come back to rr_w, rr_xh.  Afterwards rr_ab[0] is this Abar.
int gcge_handle_s::ritz_rotate(const Segs &V, int dim, int nwant, double *Y, int64_t ldy) {
    hipError_t e = hipSuccess;
    if (dense_eig_opt && dim <= DENSE_EIG_MAX) {
        e = dense_eig(dim, rr_ab[1], dim, nwant, rr_w, rr_xh, nwant, eigw, ws, st);
        if (e != hipSuccess) return hipfail(e, "dense eigensolve");
    } else {
        std::vector<double> A((size_t)dim * dim), w(dim), xh((size_t)dim * nwant);
        e = stg.download(A.data(), rr_ab[1], sizeof(double) * dim * dim);
        if (e != hipSuccess) return hipfail(e, "download");
        if (sym_eig(dim, A.data(), w.data(), xh.data(), nwant) != 0)
            return fail(GCGE_ERR_INTERNAL, "dense eigensolve did not converge");
        e = stg.upload(rr_w, w.data(), sizeof(double) * nwant);
        if (e == hipSuccess) e = stg.upload(rr_xh, xh.data(), sizeof(double) * dim * nwant);
        if (e != hipSuccess) return hipfail(e, "upload");
    }
    const int pb = prof.begin(st);
    e = gemm(op.n, V, rr_xh, nwant, nwant, 1.0, 0.0, Y, ldy, st);
    prof.end(3, pb, (int64_t)dim * nwant, st);
    if (e != hipSuccess) return hipfail(e, "rotation");
    std::swap(rr_ab[0], rr_ab[1]);
    return GCGE_OK;
}

// STEP 5 on the device: phat from the previous Rayleigh-Ritz step's xhat
// (columns shift .. shift+bsa2-1, the rows of that step's active block act_old
// zeroed, eq. CP_tilde), L2-orthogonalized against xhat twice and among
// itself twice (columns below 1e-10 of their norm dropped), alpha0 = phat^T
// Abar_old phat, and P = V_old phat (bsa2 columns, those past the kept count
// zero).  The kept count is copied to pinned_flag[8] for the host, which reads
// it after the next synchronization.  *launched = the columns of P written (0:
// no P this iteration).
int gcge_handle_s::step5(const Segs &Vold, int dim_old, int nxh_old, int shift, int act_old, int bsa2, double *P,
                         int *launched) {
    *launched = 0;
    const int nn = std::max(0, std::min(bsa2, nxh_old - shift));
    if (nn <= 0 || dim_old <= nxh_old) return GCGE_OK;
    hipError_t e = phat_init(dim_old, nxh_old, rr_xh, shift, act_old, nn, rr_pt, rr_nrm0, st);
    Segs XH;
    XH.add(rr_xh, nxh_old, nxh_old);
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
        e = gram(dim_old, XH, rr_pt, nn, nn, nullptr, rr_cf, nn, ws, st);
        if (e == hipSuccess) e = gemm(dim_old, XH, rr_cf, nn, nn, -1.0, 1.0, rr_pt, nn, st);
    }
    if (e == hipSuccess) e = phat_mgs(dim_old, nn, rr_pt, rr_nrm0, 1e-10, rr_ph, bsa2, rr_np, st);
    Segs AO, PH;
    AO.add(rr_ab[0], dim_old, dim_old);
    PH.add(rr_ph, bsa2, bsa2);
    if (e == hipSuccess) e = gemm(dim_old, AO, rr_ph, bsa2, bsa2, 1.0, 0.0, rr_t, bsa2, st);
    if (e == hipSuccess) e = gram(dim_old, PH, rr_t, bsa2, bsa2, nullptr, rr_a0, bsa2, ws, st);
    const int pb = prof.begin(st);
    if (e == hipSuccess) e = gemm(op.n, Vold, rr_ph, bsa2, bsa2, 1.0, 0.0, P, ldB, st);
    prof.end(4, pb, (int64_t)dim_old * bsa2, st);
    if (e == hipSuccess) e = hipMemcpyAsync(pinned_flag + 8, rr_np, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hipfail(e, "STEP 5");
    *launched = bsa2;
    return GCGE_OK;
}

int gcge_handle_s::ensure_buffers(int bs, int capx, int prec, int hist) {
    if (bs == cfg_bs && capx == cfg_capx && prec == cfg_prec && hist == cfg_hist) return GCGE_OK;
    bufs.release();
    m_valid = m32_valid = false;
    cfg_bs = cfg_capx = cfg_prec = cfg_hist = -1;
    cghist = cghist_alpha = nullptr;
    cghist_slots = 0;
    const int64_t n = op.n;
    ldX = round_up(capx, 4);
    ldC = round_up(nev, 4);
    ldB = round_up(bs, 4);
    ldR = 2 * ldB;
    hipError_t e = hipSuccess;
    auto A = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = bufs.alloc(p, bytes);
    };
    A((void **)&Xb[0], sizeof(double) * n * ldX);
    A((void **)&Xb[1], sizeof(double) * n * ldX);
    A((void **)&Xc, sizeof(double) * n * ldC);
    A((void **)&Pb[0], sizeof(double) * n * ldB);
    A((void **)&Pb[1], sizeof(double) * n * ldB);
    A((void **)&Wb, sizeof(double) * n * ldB);
    A((void **)&AWb, sizeof(double) * n * ldB);
    A((void **)&Rb, sizeof(double) * n * ldR);
    if (op.bkind == GCGE_B_CSR) A((void **)&BWb, sizeof(double) * n * ldB);
    A((void **)&mval, sizeof(double) * std::max<int64_t>(op.nnz, 1));
    if (prec % 2 == GCGE_PREC_FP64) {
        for (int i = 0; i < (prec >= 2 ? 4 : 3); ++i) A((void **)&cg64[i], sizeof(double) * n * ldB);
    } else {
        A((void **)&mval32, sizeof(float) * std::max<int64_t>(op.nnz, 1));
        for (int i = 0; i < (prec >= 2 ? 5 : 4); ++i) A((void **)&cg32[i], sizeof(float) * n * ldB);
    }
    // eight per-column slots, then the counter of the column-parallel
    // alpha / beta kernels (zeroed below; each use leaves it zero)
    A(&cgmem, 8 * sizeof(double) * (ldB + 16) + 64);
    if (e == hipSuccess) e = hipMemset((char *)cgmem + 8 * sizeof(double) * (ldB + 16), 0, 64);
    // Rayleigh-Ritz state: Abar of order at most capx + 2 bs (X_u, P, W)
    const int dmax = capx + 2 * bs + 8;
    const size_t d2 = (size_t)dmax * dmax, db = (size_t)dmax * ldB;
    A((void **)&rr_ab[0], sizeof(double) * d2);
    A((void **)&rr_ab[1], sizeof(double) * d2);
    A((void **)&rr_w, sizeof(double) * (dmax + 32));
    A((void **)&rr_xh, sizeof(double) * d2);
    A((void **)&rr_ph, sizeof(double) * db);
    A((void **)&rr_pt, sizeof(double) * db);
    A((void **)&rr_t, sizeof(double) * db);
    A((void **)&rr_g, sizeof(double) * std::max(d2, db));   // also X0^T A X0 of the initial block
    A((void **)&rr_cf, sizeof(double) * db);
    A((void **)&rr_a0, sizeof(double) * (size_t)ldB * ldB);
    A((void **)&rr_nrm0, sizeof(double) * (ldB + 32));
    A((void **)&rr_np, 64);
    rr_dmax = dmax;
    if (e == hipSuccess && dmax <= DENSE_EIG_MAX) e = eigw.ensure(dmax, dmax);
    if (e == hipSuccess && hist >= 2) {
        // the history takes at most half of the device memory still free
        const size_t elem = (prec % 2 == GCGE_PREC_FP64) ? sizeof(double) : sizeof(float);
        const size_t slot_bytes = elem * (size_t)n * ldB;
        size_t fr = 0, tot = 0;
        int H = 0;
        if (slot_bytes > 0 && hipMemGetInfo(&fr, &tot) == hipSuccess)
            H = (int)std::min<size_t>((size_t)hist, fr / 2 / slot_bytes);
        if (H >= 2) {
            A(&cghist, slot_bytes * H);
            A(&cghist_alpha, elem * 128 * H);
            cghist_slots = H;
        }
    }
    if (e != hipSuccess) {
        bufs.release();
        cghist = cghist_alpha = nullptr;
        cghist_slots = 0;
        return hipfail(e, "buffer allocation");
    }
    cfg_bs = bs;
    cfg_capx = capx;
    cfg_prec = prec;
    cfg_hist = hist;
    return GCGE_OK;
}

int gcge_handle_s::gram_host(const Segs &X, const double *Y, int64_t ldy, int k, const double *d,
                             std::vector<double> &C) {
    const int m = X.total();
    C.assign((size_t)m * k, 0.0);
    if (m == 0 || k == 0) return GCGE_OK;
    hipError_t e = ws.ensure_small(sizeof(double) * (2 * (size_t)m * k + 64));
    if (e != hipSuccess) return hipfail(e, "workspace");
    const int pb = prof.begin(st);
    e = gram(op.n, X, Y, ldy, k, d, ws.small, k, ws, st);
    prof.end(5, pb, (int64_t)m * k, st);
    if (e != hipSuccess) return hipfail(e, "gram");
    e = stg.download(C.data(), ws.small, sizeof(double) * m * k);
    if (e != hipSuccess) return hipfail(e, "download");
    return GCGE_OK;
}

// STEP 4 residuals R = A X - B X diag(lam) of k columns with their norms.
// lam is on the device (lam_dev, e.g. the Ritz values of the last
// Rayleigh-Ritz step) or on the host (lam_host); with lam_out the device values
// come back to the host in the same download as the norms.
int gcge_handle_s::do_residual(const double *X, int64_t ldx, int k, const double *lam_host, const double *lam_dev,
                               double *R, int64_t ldr, std::vector<double> &rn, std::vector<double> &bn,
                               std::vector<double> *lam_out) {
    rn.assign(k, 0.0);
    bn.assign(k, 0.0);
    if (k == 0) return GCGE_OK;
    int nparts = 0;
    hipError_t e = ws.ensure_part(sizeof(double) * 2 * (size_t)k * max_row_parts() + 256);
    if (e == hipSuccess) e = ws.ensure_colvec(sizeof(double) * (4 * k + 64));
    if (e != hipSuccess) return hipfail(e, "workspace");
    double *sig = ws.colvec, *out = ws.colvec + k + 16;
    if (lam_dev != nullptr) sig = const_cast<double *>(lam_dev);
    else e = stg.upload(sig, lam_host, sizeof(double) * k);
    if (e == hipSuccess) e = op.residual(X, ldx, k, sig, R, ldr, ws.part, &nparts, st);
    if (e == hipSuccess) e = colsum<double>(ws.part, nparts, 2 * k, out, st);
    const bool with_lam = lam_out != nullptr && lam_dev != nullptr;
    if (e == hipSuccess && with_lam)
        e = hipMemcpyAsync(out + 2 * k, lam_dev, sizeof(double) * k, hipMemcpyDeviceToDevice, st);
    std::vector<double> h((with_lam ? 3 : 2) * k);
    if (e == hipSuccess) e = stg.download(h.data(), out, sizeof(double) * h.size());
    if (e != hipSuccess) return hipfail(e, "residual");
    for (int j = 0; j < k; ++j) {
        rn[j] = std::sqrt(std::max(h[j], 0.0));
        bn[j] = std::sqrt(std::max(h[k + j], 0.0));
    }
    if (with_lam) {
        lam_out->assign(h.begin() + 2 * k, h.begin() + 3 * k);
        for (double v : *lam_out)
            if (!std::isfinite(v)) return fail(GCGE_ERR_INTERNAL, "dense eigensolve produced a non-finite value");
    }
    return GCGE_OK;
}

int gcge_handle_s::do_cg(double theta, const double *R, int64_t ldr, int k, const std::vector<double> &rn,
                         int64_t *cg_its) {
    const bool mixed = (precision == GCGE_PREC_MIXED);
    hipError_t e = hipSuccess;
    if (!m_valid || theta != theta_cur || (mixed && !m32_valid)) {
        e = op.shifted(theta, mval, mixed ? mval32 : nullptr, st);
        if (e != hipSuccess) return hipfail(e, "shifted operator");
        theta_cur = theta;
        m_valid = true;
        m32_valid = mixed;
    }
    char *cm = (char *)cgmem;
    const size_t slot = sizeof(double) * (ldB + 16);
    if (!mixed) {
        CgState<double> cs{(double *)cm, (double *)(cm + slot), (double *)(cm + 2 * slot), (double *)(cm + 3 * slot),
                           (int *)(cm + 4 * slot), (int *)(cm + 5 * slot), (int *)(cm + 6 * slot)};
        cs.done = (unsigned *)(cm + 8 * slot);
        CgRunner<double> runner{op.n, ws, st, pinned_flag, ev, err, &prof};
        runner.hist = (double *)cghist;
        runner.hist_slots = cghist_slots;
        runner.hist_alpha = (double *)cghist_alpha;
        DevCsr<double> M = op.csr_of(mval);
        if (precond) {
            if (!amg_valid) {
                const auto ta = Clock::now();
                int rc = amg.build(op.A_csr(), amg_levels, amg_coarse, amg_strength, st, err);
                if (rc) return rc;
                amg_valid = true;
                amg_setup_ms = ms_since(ta);
            }
            cs.rz = (double *)(cm + 7 * slot);
            return runner.run_pcg(M, amg, R, ldr, nullptr, k, cg_max_iter, cg_rel_tol, Wb, cg64[0], cg64[1],
                                  cg64[2], cg64[3], ldB, cs, cg_its);
        }
        return runner.run(M, R, ldr, nullptr, k, cg_max_iter, cg_rel_tol, Wb, cg64[0], cg64[1], cg64[2], ldB, cs,
                          cg_its);
    }
    // FP32: right-hand side scaled to unit column norms, delta scaled back on output
    e = ws.ensure_colvec(sizeof(double) * (3 * k + 64));
    if (e != hipSuccess) return hipfail(e, "workspace");
    std::vector<double> sc(k), usc(k);
    for (int j = 0; j < k; ++j) {
        sc[j] = rn[j] > 0.0 ? 1.0 / rn[j] : 0.0;
        usc[j] = rn[j];
    }
    double *dsc = ws.colvec, *dusc = ws.colvec + k + 16;
    e = stg.upload(dsc, sc.data(), sizeof(double) * k);
    if (e == hipSuccess) e = stg.upload(dusc, usc.data(), sizeof(double) * k);
    if (e != hipSuccess) return hipfail(e, "upload");
    CgState<float> cs{(float *)cm, (float *)(cm + slot), (float *)(cm + 2 * slot), (float *)(cm + 3 * slot),
                      (int *)(cm + 4 * slot), (int *)(cm + 5 * slot), (int *)(cm + 6 * slot)};
    cs.done = (unsigned *)(cm + 8 * slot);
    CgRunner<float> runner{op.n, ws, st, pinned_flag, ev, err, &prof};
    runner.hist = (float *)cghist;
    runner.hist_slots = cghist_slots;
    runner.hist_alpha = (float *)cghist_alpha;
    DevCsr<float> M = op.csr_of(mval32);
    int rc;
    if (precond) {
        // FP32 preconditioned CG with the FP32 copy of the V-cycle (the
        // hierarchy is built from the FP64 operator; level 0 is M itself)
        if (!amg_valid) {
            const auto ta = Clock::now();
            rc = amg.build(op.A_csr(), amg_levels, amg_coarse, amg_strength, st, err);
            if (rc) return rc;
            amg_valid = true;
            amg_setup_ms = ms_since(ta);
        }
        amg.set_level0_f32(M);
        cs.rz = (float *)(cm + 7 * slot);
        rc = runner.run_pcg(M, amg, R, ldr, dsc, k, cg_max_iter, cg_rel_tol, cg32[0], cg32[1], cg32[2], cg32[3],
                            cg32[4], ldB, cs, cg_its);
    } else {
        rc = runner.run(M, R, ldr, dsc, k, cg_max_iter, cg_rel_tol, cg32[0], cg32[1], cg32[2], cg32[3], ldB, cs,
                        cg_its);
    }
    if (rc) return rc;
    e = copy_cols<float, double>(op.n, k, cg32[0], ldB, Wb, ldB, dusc, st);
    if (e != hipSuccess) return hipfail(e, "cg output");
    return GCGE_OK;
}

int gcge_handle_s::solve(double *evals, double *evecs, int64_t ldev, gcge_stats *stats_out) {
    have_res = false;
    gcge_stats S;
    std::memset(&S, 0, sizeof(S));
    prof.on = profile != 0;
    prof.marks.clear();
    prof.next = 0;
    const auto T0 = Clock::now();
    const int64_t n = op.n;
    int bs = (int)(opt_bs > 0 ? opt_bs : std::max(1, nev / 5));
    bs = std::min<int64_t>(bs, std::min<int64_t>(nev, n));
    if (bs > 128) return fail(GCGE_ERR_INVALID_ARG, "block_size above 128 is not supported");
    prof.full_cols = bs;
    const bool mv = moving && nev > 2 * bs;
    int64_t sx = opt_sizex > 0 ? opt_sizex : std::min<int64_t>(nev + 3 * (int64_t)bs, n);
    sx = std::max<int64_t>(sx, nev);
    sx = std::min<int64_t>(sx, n);
    const int sizeX = (int)sx;
    const int nx0 = mv ? (int)std::min<int64_t>(3 * (int64_t)bs, n) : sizeX;
    if (x0_k > nx0) return fail(GCGE_ERR_INVALID_ARG, "more initial vectors than the initial block holds");
    const int hist = (cg_history >= 2 && cg_max_iter >= 1) ? std::min(cg_history, cg_max_iter + 1) : 0;
    int rc = ensure_buffers(bs, nx0, precision + 2 * precond, hist);
    if (rc) return rc;
    stg.st = st;
    hipError_t e;
    if (!pinned_flag) {
        e = hipHostMalloc((void **)&pinned_flag, 64, hipHostMallocDefault);
        if (e != hipSuccess) return hipfail(e, "pinned flag");
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return hipfail(e, "event");
    }
    // small-matrix workspace sized for the largest Abar and Gram once
    {
        const size_t dmax = (size_t)nx0 + 2 * bs + 8;
        e = ws.ensure_small(sizeof(double) * (2 * std::max(dmax * dmax, (size_t)nev * nev) + 1024));
        // Gram partials for any shape, so that nothing is reallocated while work is queued
        if (e == hipSuccess) e = ws.ensure_part(gram_part_bytes_max());
        if (e != hipSuccess) return hipfail(e, "workspace");
    }
    const BOp bop = op.bop();
    const double *dW = (op.bkind == GCGE_B_DIAG) ? op.dg : nullptr;   // Gram weight for B
    OrthOptions oo;
    oo.orth_tol = orth_tol;
    oo.drop_tol = drop_tol;
    oo.algorithm = orth_alg;
    oo.mbo_block = orth_block_opt;
    oo.skip_final = orth_skip_final != 0;
    OrthStats ostat;

    // ---------------- STEPs 1-3, first pass: random block, orthogonalize, Rayleigh-Ritz
    e = fill_random(n, nx0, 0, seed, Xb[0], ldX, st);
    if (e == hipSuccess && x0_k > 0) e = copy_cols<double, double>(n, x0_k, x0, x0_ld, Xb[0], ldX, nullptr, st);
    if (e != hipSuccess) return hipfail(e, "initial block");
    int k0 = 0;
    rc = orth_block(n, bop, Segs{}, Xb[0], ldX, nx0, Xb[1], ldX, oo, ws, stg, st, &k0, &ostat, err);
    if (rc) return rc;
    if (k0 == 0) return fail(GCGE_ERR_NOT_SPD, "the initial block has no direction of positive B-norm");
    for (int c0 = 0; c0 < k0; c0 += 128) {
        const int kk = std::min(128, k0 - c0);
        e = spmm<double>(op.A_csr(), nullptr, nullptr, nullptr, 0, 0, Xb[0] + c0, ldX, kk, Xb[1] + c0, ldX, nullptr,
                         0, nullptr, nullptr, st);
        if (e != hipSuccess) return hipfail(e, "A X");
    }
    S.spmm_columns += k0;
    {
        Segs X0;
        X0.add(Xb[0], ldX, k0);
        const int pb = prof.begin(st);
        e = gram(n, X0, Xb[1], ldX, k0, nullptr, rr_g, k0, ws, st);
        prof.end(5, pb, (int64_t)k0 * k0, st);
        // Abar = X0^T A X0, symmetrized (all of it is "the W block")
        if (e == hipSuccess) e = assemble_abar(k0, 0, 0, k0, nullptr, nullptr, 0, rr_g, rr_ab[1], st);
        if (e != hipSuccess) return hipfail(e, "initial Rayleigh-Ritz");
        rc = ritz_rotate(X0, k0, k0, Xb[1], ldX);
        if (rc) return rc;
    }
    int cur = 1, pc = 0;
    int64_t off = 0;
    int nx = k0;
    int woff = 0;   // Ritz values of the window: rr_w + woff .. (locked ones are skipped)
    Segs Vold;
    Vold.add(Xb[0], ldX, k0);
    int dim_old = k0, nxh_old = k0, act_old = 0;
    int np = 0, nw = 0;
    int ell = 0;
    std::vector<double> lam_lock(nev, 0.0);
    S.time_ms[0] = ms_since(T0);
    bool converged = false;
    std::vector<double> rn, bn, lamv;

    for (int it = 0; it < max_iter; ++it) {
        S.iterations = it + 1;
        // ---------------- STEP 4: convergence of the active block, locking
        auto t4 = Clock::now();
        int bsa = std::min({bs, nev - ell, nx});
        if (bsa <= 0) return fail(GCGE_ERR_INTERNAL, "empty active block");
        double *Xu = Xb[cur] + off;
        rc = do_residual(Xu, ldX, bsa, nullptr, rr_w + woff, Rb, ldR, rn, bn, &lamv);
        if (rc) return rc;
        S.spmm_columns += bsa;
        int c = 0;
        while (c < bsa && rn[c] <= tol * std::fabs(lamv[c]) * bn[c]) ++c;
        if (c > 0) {
            e = copy_cols<double, double>(n, c, Xu, ldX, Xc + ell, ldC, nullptr, st);
            if (e != hipSuccess) return hipfail(e, "lock");
            for (int j = 0; j < c; ++j) lam_lock[ell + j] = lamv[j];
            ell += c;
        }
        S.time_ms[3] += ms_since(t4);
        if (ell >= nev) {
            converged = true;
            break;
        }
        off += c;
        nx -= c;
        woff += c;
        Xu = Xb[cur] + off;
        const int bsa2 = std::min({bs, nev - ell, nx});
        if (bsa2 <= 0) return fail(GCGE_ERR_INTERNAL, "no unconverged vectors left in the window");

        // ---------------- STEP 5: the next P, on the device (its kept count is read after STEP 6)
        auto t5 = Clock::now();
        int p_launched = 0;
        rc = step5(Vold, dim_old, nxh_old, c, act_old, bsa2, Pb[1 - pc], &p_launched);
        if (rc) return rc;
        S.time_ms[4] += ms_since(t5);

        // residuals of the shifted active block: the first bsa - c are those of
        // STEP 4 (columns c .. bsa-1 of R, which the CG reads from R + c); only
        // the columns entering the block are computed, into R + bsa
        const double *Rcur = Rb + c;
        if (c > 0) {
            auto t4b = Clock::now();
            rn.erase(rn.begin(), rn.begin() + c);
            bn.erase(bn.begin(), bn.begin() + c);
            const int have = bsa - c, nnew = bsa2 - have;
            if (nnew > 0) {
                std::vector<double> rn2, bn2;
                rc = do_residual(Xu + have, ldX, nnew, nullptr, rr_w + woff + have, Rb + bsa, ldR, rn2, bn2, nullptr);
                if (rc) return rc;
                rn.insert(rn.end(), rn2.begin(), rn2.end());
                bn.insert(bn.end(), bn2.begin(), bn2.end());
                S.spmm_columns += nnew;
            }
            rn.resize(bsa2);
            bn.resize(bsa2);
            S.time_ms[3] += ms_since(t4b);
        }

        // ---------------- STEP 6: inner CG with the dynamic shift
        auto t6 = Clock::now();
        double theta = 0.0;
        if (shift && !precond && ell > 0) theta = *std::max_element(lam_lock.begin(), lam_lock.begin() + ell);
        int64_t cgi = 0;
        rc = do_cg(theta, Rcur, ldR, bsa2, rn, &cgi);
        if (rc) return rc;
        S.cg_iterations += cgi;
        S.spmm_columns += cgi * bsa2;
        e = stg.sync();
        if (e != hipSuccess) return hipfail(e, "sync");
        S.time_ms[5] += ms_since(t6);
        np = 0;
        if (p_launched > 0) {
            np = pinned_flag[8];
            if (np < 0 || np > p_launched) return fail(GCGE_ERR_INTERNAL, "inconsistent STEP 5 column count");
            pc = 1 - pc;
        }

        // ---------------- STEP 2: B-orthogonalize W against [X_c, X_u, P], Algorithm 3
        auto t2 = Clock::now();
        Segs Q;
        Q.add(Xc, ldC, ell);
        Q.add(Xu, ldX, nx);
        Q.add(Pb[pc], ldB, np);
        rc = orth_block(n, bop, Q, Wb, ldB, bsa2, BWb, ldB, oo, ws, stg, st, &nw, &ostat, err);
        if (rc) return rc;
        S.time_ms[1] += ms_since(t2);

        // ---------------- STEP 3: Rayleigh-Ritz with the structured Abar, on the device
        auto t3 = Clock::now();
        if (nw > 0) {
            e = spmm<double>(op.A_csr(), nullptr, nullptr, nullptr, 0, 0, Wb, ldB, nw, AWb, ldB, nullptr, 0, nullptr, nullptr, st);
            if (e != hipSuccess) return hipfail(e, "A W");
            S.spmm_columns += nw;
        }
        Segs Vu;
        Vu.add(Xu, ldX, nx);
        Vu.add(Pb[pc], ldB, np);
        Vu.add(Wb, ldB, nw);
        const int dim = nx + np + nw;
        if (dim > rr_dmax) return fail(GCGE_ERR_INTERNAL, "Rayleigh-Ritz order above its buffers");
        if (nw > 0) {
            const int pb = prof.begin(st);
            e = gram(n, Vu, AWb, ldB, nw, nullptr, rr_g, nw, ws, st);
            prof.end(5, pb, (int64_t)dim * nw, st);
            if (e != hipSuccess) return hipfail(e, "gram");
        }
        e = assemble_abar(dim, nx, np, nw, rr_w + woff, rr_a0, bsa2, rr_g, rr_ab[1], st);
        if (e != hipSuccess) return hipfail(e, "Abar");
        const bool move = mv && nx <= bs;
        const int nwant = move ? dim : nx;
        rc = ritz_rotate(Vu, dim, nwant, Xb[1 - cur], ldX);
        if (rc) return rc;
        if (move) S.moves++;
        Vold = Vu;
        dim_old = dim;
        nxh_old = nwant;
        act_old = bsa2;
        cur = 1 - cur;
        off = 0;
        woff = 0;
        nx = nwant;
        e = stg.sync();
        if (e != hipSuccess) return hipfail(e, "sync");
        S.time_ms[2] += ms_since(t3);
    }

    // ---------------- outputs
    auto tf = Clock::now();
    int nout = ell;
    if (!converged) {
        // fill the remaining pairs with the current approximations
        const int extra = std::min(nev - ell, nx);
        if (extra > 0) {
            e = copy_cols<double, double>(n, extra, Xb[cur] + off, ldX, Xc + ell, ldC, nullptr, st);
            if (e == hipSuccess) e = stg.download(lam_lock.data() + ell, rr_w + woff, sizeof(double) * extra);
            if (e != hipSuccess) return hipfail(e, "output");
        }
        nout = ell + extra;
    }
    std::vector<int> ord(nout);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return lam_lock[a] < lam_lock[b]; });
    res_lam.assign(nev, std::nan(""));
    res_col.assign(nev, -1);
    for (int i = 0; i < nout; ++i) {
        res_lam[i] = lam_lock[ord[i]];
        res_col[i] = ord[i];
    }
    if (evals) std::memcpy(evals, res_lam.data(), sizeof(double) * nev);
    if (evecs && nout > 0) {
        e = ws.ensure_colvec(sizeof(int) * (nout + 64));
        if (e == hipSuccess) e = stg.upload(ws.colvec, ord.data(), sizeof(int) * nout);
        if (e == hipSuccess) e = gather_cols(n, nout, Xc, ldC, (const int *)ws.colvec, evecs, ldev, st);
        if (e != hipSuccess) return hipfail(e, "output");
    }
    S.nconv = ell;
    S.max_rel_residual = std::nan("");
    S.orth_error = std::nan("");
    if (check && nout > 0) {
        // explicit residuals of the returned pairs and B-orthonormality
        double *tmpR = Xb[1 - cur];
        const int chunk = (int)std::min<int64_t>(128, ldX);
        double mr = 0.0;
        for (int c0 = 0; c0 < nout; c0 += chunk) {
            const int kk = std::min(chunk, nout - c0);
            rc = do_residual(Xc + c0, ldC, kk, lam_lock.data() + c0, nullptr, tmpR, ldX, rn, bn, nullptr);
            if (rc) return rc;
            for (int j = 0; j < kk; ++j) mr = std::max(mr, rn[j] / (std::fabs(lam_lock[c0 + j]) * bn[j]));
        }
        S.max_rel_residual = mr;
        double oe = 0.0;
        Segs XC;
        XC.add(Xc, ldC, nout);
        for (int c0 = 0; c0 < nout; c0 += chunk) {
            const int kk = std::min(chunk, nout - c0);
            std::vector<double> C;
            if (op.bkind == GCGE_B_CSR) {
                e = bop_apply(bop, n, Xc + c0, ldC, kk, tmpR, ldX, st);
                if (e != hipSuccess) return hipfail(e, "B X");
                rc = gram_host(XC, tmpR, ldX, kk, nullptr, C);
            } else {
                rc = gram_host(XC, Xc + c0, ldC, kk, dW, C);
            }
            if (rc) return rc;
            for (int i = 0; i < nout; ++i)
                for (int j = 0; j < kk; ++j)
                    oe = std::max(oe, std::fabs(C[(size_t)i * kk + j] - (i == c0 + j ? 1.0 : 0.0)));
        }
        S.orth_error = oe;
    }
    e = stg.sync();
    if (e != hipSuccess) return hipfail(e, "sync");
    S.time_ms[6] = ms_since(tf);
    S.time_ms[7] = ms_since(T0);
    prof.finish(S);
    have_res = nout == nev;
    res_converged = converged;
    last = S;
    if (stats_out) *stats_out = S;
    return converged ? GCGE_OK : GCGE_NOT_CONVERGED;
}

// =================================================================== C ABI

#define GCGE_CATCH(h)                                                        \
    catch (const std::bad_alloc &) {                                         \
        if (h) (h)->err = "host out of memory";                              \
        return GCGE_ERR_OOM;                                                 \
    }                                                                        \
    catch (...) {                                                            \
        if (h) (h)->err = "internal error";                                  \
        return GCGE_ERR_INTERNAL;                                            \
    }

namespace gcge {
void set_thread_error(const std::string &msg) { g_thread_err = msg; }
}  // namespace gcge

static bool csr_ok(const gcge_csr *A) {
    return A && A->n >= 1 && A->nnz >= 0 && A->rowptr && (A->nnz == 0 || (A->colind && A->val)) &&
           A->nnz <= INT32_MAX;
}

extern "C" int gcge_create(const gcge_csr *A, int b_kind, const void *B, int nev, double tol, gcge_handle *out) {
    if (!out) {
        g_thread_err = "out is NULL";
        return GCGE_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (!csr_ok(A) || nev < 1 || nev > A->n || !(tol > 0.0) ||
        (b_kind != GCGE_B_IDENTITY && b_kind != GCGE_B_DIAG && b_kind != GCGE_B_CSR) ||
        (b_kind != GCGE_B_IDENTITY && B == nullptr) || (b_kind == GCGE_B_CSR && !csr_ok((const gcge_csr *)B))) {
        g_thread_err = "gcge_create: invalid argument";
        return GCGE_ERR_INVALID_ARG;
    }
    gcge_handle h = nullptr;
    try {
        h = new gcge_handle_s();
        h->A_user = *A;
        if (b_kind == GCGE_B_CSR) h->B_user = *(const gcge_csr *)B;
        if (b_kind == GCGE_B_DIAG) h->d_user = (const double *)B;
        h->nev = nev;
        h->tol = tol;
        std::string err;
        int rc = h->op.build(A, b_kind, B, h->st, err);
        if (!rc) rc = h->op.check_b_positive(h->st, err);
        if (rc) {
            g_thread_err = "gcge_create: " + err;
            h->op.destroy();
            delete h;
            return rc;
        }
    } catch (...) {
        g_thread_err = "gcge_create: host allocation failed";
        if (h) {
            h->op.destroy();
            delete h;
        }
        return GCGE_ERR_OOM;
    }
    *out = h;
    return GCGE_OK;
}

extern "C" int gcge_set_option_i(gcge_handle h, const char *key, int64_t v) {
    if (!h || !key) return GCGE_ERR_INVALID_ARG;
    const std::string k(key);
    auto bad = [&]() { return h->fail(GCGE_ERR_INVALID_ARG, "bad value for option " + k); };
    if (k == "block_size") { if (v < 0 || v > 128) return bad(); h->opt_bs = v; }
    else if (k == "size_x") { if (v < 0 || v > h->op.n) return bad(); h->opt_sizex = v; }
    else if (k == "max_iter") { if (v < 1 || v > 1000000) return bad(); h->max_iter = (int)v; }
    else if (k == "cg_max_iter") { if (v < 0 || v > 100000) return bad(); h->cg_max_iter = (int)v; }
    else if (k == "precision") { if (v != GCGE_PREC_FP64 && v != GCGE_PREC_MIXED) return bad(); h->precision = (int)v; }
    else if (k == "moving") { if (v != 0 && v != 1) return bad(); h->moving = (int)v; }
    else if (k == "shift") { if (v != 0 && v != 1) return bad(); h->shift = (int)v; }
    else if (k == "seed") { h->seed = (uint64_t)v; }
    else if (k == "check") { if (v != 0 && v != 1) return bad(); h->check = (int)v; }
    else if (k == "profile") { if (v != 0 && v != 1) return bad(); h->profile = (int)v; }
    else if (k == "cg_history") { if (v != 0 && (v < 2 || v > CG_HIST_MAX)) return bad(); h->cg_history = (int)v; }
    else if (k == "dense_eig") { if (v != 0 && v != 1) return bad(); h->dense_eig_opt = (int)v; }
    else if (k == "orth") { if (v != 2 && v != 3) return bad(); h->orth_alg = (int)v; }
    else if (k == "orth_block") { if (v < 0 || v > 100000) return bad(); h->orth_block_opt = (int)v; }
    else if (k == "orth_skip_final") { if (v != 0 && v != 1) return bad(); h->orth_skip_final = (int)v; }
    else if (k == "precond") { if (v != 0 && v != 1) return bad(); h->precond = (int)v; }
    else if (k == "amg_levels") {
        if (v < 1 || v > AMG_MAX_LEVELS) return bad();
        h->amg_levels = (int)v;
        h->amg_valid = false;
    } else if (k == "amg_coarse") {
        if (v < 1 || v > AMG_COARSE_LIMIT) return bad();
        h->amg_coarse = (int)v;
        h->amg_valid = false;
    }
    else return h->fail(GCGE_ERR_INVALID_ARG, "unknown option " + k);
    return GCGE_OK;
}

extern "C" int gcge_set_option_d(gcge_handle h, const char *key, double v) {
    if (!h || !key) return GCGE_ERR_INVALID_ARG;
    const std::string k(key);
    const bool zero_ok = (k == "cg_rel_tol" || k == "amg_strength");   // cg_rel_tol 0: fixed CG length
    if (!std::isfinite(v) || v < 0.0 || (v == 0.0 && !zero_ok))
        return h->fail(GCGE_ERR_INVALID_ARG, "bad value for option " + k);
    if (k == "tol") h->tol = v;
    else if (k == "cg_rel_tol") h->cg_rel_tol = v;
    else if (k == "orth_tol") h->orth_tol = v;
    else if (k == "drop_tol") h->drop_tol = v;
    else if (k == "amg_strength") {
        if (v >= 1.0) return h->fail(GCGE_ERR_INVALID_ARG, "bad value for option " + k);
        h->amg_strength = v;
        h->amg_valid = false;
    }
    else return h->fail(GCGE_ERR_INVALID_ARG, "unknown option " + k);
    return GCGE_OK;
}

extern "C" int gcge_set_stream(gcge_handle h, void *stream) {
    if (!h) return GCGE_ERR_INVALID_ARG;
    h->st = (hipStream_t)stream;
    h->stg.st = h->st;
    return GCGE_OK;
}

extern "C" int gcge_set_initial_vectors(gcge_handle h, const double *X0, int64_t ld, int k) {
    if (!h || k < 0 || (k > 0 && (!X0 || ld < k))) return GCGE_ERR_INVALID_ARG;
    h->x0 = X0;
    h->x0_ld = ld;
    h->x0_k = k;
    return GCGE_OK;
}

extern "C" int gcge_solve(gcge_handle h, double *evals, double *evecs, int64_t ld, gcge_stats *stats) {
    if (!h) return GCGE_ERR_INVALID_ARG;
    if (evecs && ld < h->nev) return h->fail(GCGE_ERR_INVALID_ARG, "ld < nev");
    try {
        h->stg.st = h->st;
        return h->solve(evals, evecs, ld, stats);
    }
    GCGE_CATCH(h)
}

extern "C" int gcge_update_values(gcge_handle h, const double *a_val, const void *b_val) {
    if (!h) return GCGE_ERR_INVALID_ARG;
    h->m_valid = h->m32_valid = false;
    h->amg_valid = false;
    h->have_res = false;
    std::string err;
    int rc = h->op.set_values(a_val, b_val, h->st, err);
    if (!rc && b_val) rc = h->op.check_b_positive(h->st, err);
    if (rc) h->err = err;
    return rc;
}

extern "C" int gcge_eig_grad(gcge_handle h, const double *g, double *gA, double *gB) {
    if (!h || !g || !gA) return GCGE_ERR_INVALID_ARG;
    if (!h->have_res) return h->fail(GCGE_ERR_INVALID_ARG, "no solution available (call gcge_solve first)");
    const int nev = h->nev;
    if (nev > 256) return h->fail(GCGE_ERR_INVALID_ARG, "gradients support nev <= 256");
    try {
        // weights per column of the locked block
        std::vector<double> wA(nev, 0.0), wB(nev, 0.0);
        for (int i = 0; i < nev; ++i) {
            wA[h->res_col[i]] = g[i];
            wB[h->res_col[i]] = -g[i] * h->res_lam[i];
        }
        hipError_t e = h->ws.ensure_colvec(sizeof(double) * (2 * nev + 64));
        if (e != hipSuccess) return h->hipfail(e, "workspace");
        h->stg.st = h->st;
        double *dA = h->ws.colvec, *dB = h->ws.colvec + nev + 16;
        e = h->stg.upload(dA, wA.data(), sizeof(double) * nev);
        if (e == hipSuccess) e = h->stg.upload(dB, wB.data(), sizeof(double) * nev);
        if (e == hipSuccess)
            e = pattern_grad(h->op.n, h->A_user.rowptr, h->A_user.colind, h->Xc, h->ldC, nev, dA, gA, h->st);
        if (e == hipSuccess && gB) {
            if (h->op.bkind == GCGE_B_CSR)
                e = pattern_grad(h->op.n, h->B_user.rowptr, h->B_user.colind, h->Xc, h->ldC, nev, dB, gB, h->st);
            else if (h->op.bkind == GCGE_B_DIAG)
                e = diag_grad(h->op.n, h->Xc, h->ldC, nev, dB, gB, h->st);
        }
        if (e == hipSuccess) e = h->stg.sync();
        if (e != hipSuccess) return h->hipfail(e, "gradient");
        if (!h->res_converged) {
            h->err = "the last solve did not converge: the gradient formula assumes exact eigenpairs";
            return GCGE_NOT_CONVERGED;
        }
        return GCGE_OK;
    }
    GCGE_CATCH(h)
}

extern "C" void gcge_destroy(gcge_handle h) {
    if (!h) return;
    if (h->st) (void)hipStreamSynchronize(h->st);
    else (void)hipDeviceSynchronize();
    h->bufs.release();
    h->amg.release();
    h->op.destroy();
    h->ws.release();
    h->stg.release();
    if (h->pinned_flag) (void)hipHostFree(h->pinned_flag);
    if (h->ev) (void)hipEventDestroy(h->ev);
    h->prof.release();
    h->eigw.release();
    delete h;
}

extern "C" const char *gcge_last_error(gcge_handle h) {
    if (!h) return g_thread_err.c_str();
    return h->err.c_str();
}

// ============================================================ step entries

namespace {

struct StepCtx {
    std::mutex mu;
    Workspace ws;
    Stager stg;
    DenseEigWork eig;
};

StepCtx &step_ctx() {
    static StepCtx *c = new StepCtx();   // never destroyed: lives until process exit
    return *c;
}

int step_fail(int code, const std::string &msg) {
    g_thread_err = msg;
    return code;
}
int step_hip(hipError_t e, const char *what) {
    return step_fail(hip_status(e), std::string(what) + ": " + hipGetErrorString(e));
}

DevCsr<double> to_dev(const gcge_csr *A) { return DevCsr<double>{A->n, A->nnz, A->rowptr, A->colind, A->val}; }

}  // namespace

extern "C" int gcge_spmm(const gcge_csr *A, const double *X, int64_t ldx, int k, double *Y, int64_t ldy,
                         void *stream) {
    if (!csr_ok(A) || k < 0 || (k > 0 && (!X || !Y || ldx < k || ldy < k)))
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_spmm: invalid argument");
    hipStream_t st = (hipStream_t)stream;
    for (int c0 = 0; c0 < k; c0 += 128) {
        const int kk = std::min(128, k - c0);
        Affine<double> exact;   // Y = 0 - (-1) A X: the affine epilogue writes only the k columns
        exact.ws = -1.0;
        exact.exact = true;
        hipError_t e = spmm_affine<double>(to_dev(A), X + c0, ldx, kk, Y + c0, ldy, exact, st);
        if (e != hipSuccess) return step_hip(e, "gcge_spmm");
    }
    return GCGE_OK;
}

extern "C" int gcge_spmm_f32(int64_t n, const int32_t *rowptr, const int32_t *colind, const float *val,
                             const float *X, int64_t ldx, int k, float *Y, int64_t ldy, void *stream) {
    if (n < 1 || !rowptr || k < 0 || (k > 0 && (!X || !Y || ldx < k || ldy < k)))
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_spmm_f32: invalid argument");
    hipStream_t st = (hipStream_t)stream;
    DevCsr<float> A{n, 0, rowptr, colind, val};
    for (int c0 = 0; c0 < k; c0 += 128) {
        const int kk = std::min(128, k - c0);
        Affine<float> exact;   // Y = 0 - (-1) A X: the affine epilogue writes only the k columns
        exact.ws = -1.0f;
        exact.exact = true;
        hipError_t e = spmm_affine<float>(A, X + c0, ldx, kk, Y + c0, ldy, exact, st);
        if (e != hipSuccess) return step_hip(e, "gcge_spmm_f32");
    }
    return GCGE_OK;
}

static int build_step_operator(const gcge_csr *A, int b_kind, const void *B, hipStream_t st, Operator &op) {
    if (!csr_ok(A) || (b_kind != GCGE_B_IDENTITY && b_kind != GCGE_B_DIAG && b_kind != GCGE_B_CSR) ||
        (b_kind != GCGE_B_IDENTITY && !B) || (b_kind == GCGE_B_CSR && !csr_ok((const gcge_csr *)B)))
        return step_fail(GCGE_ERR_INVALID_ARG, "invalid operator arguments");
    std::string err;
    int rc = op.build(A, b_kind, B, st, err);
    if (rc) return step_fail(rc, err);
    return GCGE_OK;
}

static int shifted_or_residual(const gcge_csr *A, int b_kind, const void *B, const double *sigma, const double *X,
                               int64_t ldx, int k, double *Y, int64_t ldy, double *rnorm, double *bxnorm,
                               void *stream) {
    if (k < 0 || (k > 0 && (!sigma || !X || !Y || ldx < k || ldy < k)))
        return step_fail(GCGE_ERR_INVALID_ARG, "invalid argument");
    if (k == 0) return GCGE_OK;
    hipStream_t st = (hipStream_t)stream;
    StepCtx &C = step_ctx();
    std::lock_guard<std::mutex> lk(C.mu);
    C.stg.st = st;
    Operator op;
    int rc = build_step_operator(A, b_kind, B, st, op);
    if (rc) return rc;
    hipError_t e = hipSuccess;
    for (int c0 = 0; c0 < k && e == hipSuccess; c0 += 128) {
        const int kk = std::min(128, k - c0);
        int nparts = 0;
        e = C.ws.ensure_part(sizeof(double) * 2 * (size_t)kk * max_row_parts() + 256);
        if (e == hipSuccess) e = C.ws.ensure_colvec(sizeof(double) * (3 * kk + 64));
        if (e != hipSuccess) break;
        double *sig = C.ws.colvec, *out = C.ws.colvec + kk + 16;
        e = C.stg.upload(sig, sigma + c0, sizeof(double) * kk);
        if (e == hipSuccess) e = op.residual(X + c0, ldx, kk, sig, Y + c0, ldy, C.ws.part, &nparts, st);
        if (e == hipSuccess && rnorm) {
            std::vector<double> h(2 * kk);
            e = colsum<double>(C.ws.part, nparts, 2 * kk, out, st);
            if (e == hipSuccess) e = C.stg.download(h.data(), out, sizeof(double) * 2 * kk);
            for (int j = 0; j < kk && e == hipSuccess; ++j) {
                rnorm[c0 + j] = std::sqrt(std::max(h[j], 0.0));
                if (bxnorm) bxnorm[c0 + j] = std::sqrt(std::max(h[kk + j], 0.0));
            }
        }
    }
    if (e == hipSuccess) e = C.stg.sync();
    op.destroy();
    if (e != hipSuccess) return step_hip(e, "shifted spmm");
    return GCGE_OK;
}

extern "C" int gcge_shifted_spmm(const gcge_csr *A, int b_kind, const void *B, const double *sigma, const double *X,
                                 int64_t ldx, int k, double *Y, int64_t ldy, void *stream) {
    try {
        return shifted_or_residual(A, b_kind, B, sigma, X, ldx, k, Y, ldy, nullptr, nullptr, stream);
    } catch (...) {
        return step_fail(GCGE_ERR_INTERNAL, "gcge_shifted_spmm: internal error");
    }
}

extern "C" int gcge_residual(const gcge_csr *A, int b_kind, const void *B, const double *lam, const double *X,
                             int64_t ldx, int k, double *R, int64_t ldr, double *rnorm, double *bxnorm, void *stream) {
    if (!rnorm || !bxnorm) return step_fail(GCGE_ERR_INVALID_ARG, "gcge_residual: norms are required");
    try {
        return shifted_or_residual(A, b_kind, B, lam, X, ldx, k, R, ldr, rnorm, bxnorm, stream);
    } catch (...) {
        return step_fail(GCGE_ERR_INTERNAL, "gcge_residual: internal error");
    }
}

extern "C" int gcge_gram(int64_t n, const double *X, int64_t ldx, int m, const double *Y, int64_t ldy, int k,
                         const double *d, double *Cout, void *stream) {
    if (n < 0 || m < 0 || k < 0 || (m > 0 && (!X || ldx < m)) || (k > 0 && (!Y || ldy < k)) || (m * k > 0 && !Cout))
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_gram: invalid argument");
    if (m == 0 || k == 0) return GCGE_OK;
    if (m > 48 * 64) return step_fail(GCGE_ERR_INVALID_ARG, "gcge_gram: m above 3072 is not supported");
    if (n == 0) {
        std::memset(Cout, 0, sizeof(double) * m * k);
        return GCGE_OK;
    }
    try {
        hipStream_t st = (hipStream_t)stream;
        StepCtx &C = step_ctx();
        std::lock_guard<std::mutex> lk(C.mu);
        C.stg.st = st;
        hipError_t e = C.ws.ensure_small(sizeof(double) * ((size_t)m * k + 64));
        Segs XS;
        XS.add(X, ldx, m);
        if (e == hipSuccess) e = gram(n, XS, Y, ldy, k, d, C.ws.small, k, C.ws, st);
        if (e == hipSuccess) e = C.stg.download(Cout, C.ws.small, sizeof(double) * m * k);
        if (e != hipSuccess) return step_hip(e, "gcge_gram");
        return GCGE_OK;
    } catch (...) {
        return step_fail(GCGE_ERR_INTERNAL, "gcge_gram: internal error");
    }
}

extern "C" int gcge_gemm_update(int64_t n, const double *X, int64_t ldx, int m, const double *S, int k, double alpha,
                                double beta, double *Y, int64_t ldy, void *stream) {
    if (n < 0 || m < 0 || k < 0 || (m > 0 && (!X || ldx < m)) || (k > 0 && (!Y || ldy < k)) || (m * k > 0 && !S))
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_gemm_update: invalid argument");
    if (n == 0 || k == 0) return GCGE_OK;
    // in-place use is only defined for a row transform of at most 64 columns:
    // row i of Y may overlap row i of X only, so with equal strides the
    // columns of X and of Y, offset by off doubles, must fit in one row
    const char *xb = (const char *)X, *xe = (const char *)(X + (n - 1) * ldx + m);
    const char *yb = (const char *)Y, *ye = (const char *)(Y + (n - 1) * ldy + k);
    const bool overlap = m > 0 && !(ye <= xb || xe <= yb);
    if (overlap) {
        const std::ptrdiff_t db = yb - xb;
        const bool whole = db % (std::ptrdiff_t)sizeof(double) == 0;
        const int64_t off = db / (std::ptrdiff_t)sizeof(double);
        const bool row_local = whole && ldx == ldy && std::max<int64_t>(m, off + k) - std::min<int64_t>(0, off) <= ldx;
        if (k > 64 || !row_local)
            return step_fail(GCGE_ERR_INVALID_ARG, "gcge_gemm_update: overlapping X and Y must be a row transform "
                                                   "(equal ld, row i of Y within row i of X's stride, k <= 64)");
    }
    try {
        hipStream_t st = (hipStream_t)stream;
        StepCtx &C = step_ctx();
        std::lock_guard<std::mutex> lk(C.mu);
        C.stg.st = st;
        hipError_t e = C.ws.ensure_small(sizeof(double) * ((size_t)std::max(m, 1) * k + 64));
        if (e == hipSuccess && m > 0) e = C.stg.upload(C.ws.small, S, sizeof(double) * m * k);
        Segs XS;
        XS.add(X, ldx, m);
        if (e == hipSuccess) e = gemm(n, XS, C.ws.small, k, k, alpha, beta, Y, ldy, st);
        if (e == hipSuccess) e = C.stg.sync();
        if (e != hipSuccess) return step_hip(e, "gcge_gemm_update");
        return GCGE_OK;
    } catch (...) {
        return step_fail(GCGE_ERR_INTERNAL, "gcge_gemm_update: internal error");
    }
}

extern "C" int gcge_cg(const gcge_csr *A, int b_kind, const void *B, double theta, const double *R, int64_t ldr, int k,
                       int maxit, double rel_tol, int precision, double *delta, int64_t ldd, int *its, void *stream) {
    if (k < 0 || k > 128 || maxit < 0 || !(rel_tol >= 0.0) ||
        (precision != GCGE_PREC_FP64 && precision != GCGE_PREC_MIXED) || (k > 0 && (!R || !delta || ldr < k || ldd < k)))
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_cg: invalid argument");
    if (k == 0) return GCGE_OK;
    try {
        hipStream_t st = (hipStream_t)stream;
        StepCtx &C = step_ctx();
        std::lock_guard<std::mutex> lk(C.mu);
        C.stg.st = st;
        Operator op;
        int rc = build_step_operator(A, b_kind, B, st, op);
        if (rc) return rc;
        const int64_t n = op.n;
        const int64_t ld = round_up(k, 4);
        Buffers bufs;
        hipError_t e = hipSuccess;
        double *m64 = nullptr;
        float *m32 = nullptr;
        void *vecs = nullptr, *cm = nullptr;
        const bool mixed = precision == GCGE_PREC_MIXED;
        e = bufs.alloc((void **)&m64, sizeof(double) * std::max<int64_t>(op.nnz, 1));
        if (e == hipSuccess && mixed) e = bufs.alloc((void **)&m32, sizeof(float) * std::max<int64_t>(op.nnz, 1));
        if (e == hipSuccess) e = bufs.alloc(&vecs, (mixed ? sizeof(float) : sizeof(double)) * 4 * n * ld);
        if (e == hipSuccess) e = bufs.alloc(&cm, 8 * sizeof(double) * (ld + 16) + 64);
        if (e == hipSuccess) e = op.shifted(theta, m64, m32, st);
        std::string err;
        if (e == hipSuccess) {
            const size_t slot = sizeof(double) * (ld + 16);
            char *c8 = (char *)cm;
            unsigned *done = (unsigned *)(c8 + 8 * slot);   // counter of the column-parallel alpha / beta
            e = hipMemsetAsync(done, 0, 64, st);
            if (e == hipSuccess && !mixed) {
                double *v = (double *)vecs;
                CgState<double> cs{(double *)c8, (double *)(c8 + slot), (double *)(c8 + 2 * slot),
                                   (double *)(c8 + 3 * slot), (int *)(c8 + 4 * slot), (int *)(c8 + 5 * slot),
                                   (int *)(c8 + 6 * slot)};
                cs.done = done;
                CgRunner<double> runner{n, C.ws, st, nullptr, nullptr, err};
                DevCsr<double> M = op.csr_of(m64);
                rc = runner.run(M, R, ldr, nullptr, k, maxit, rel_tol, v, v + n * ld, v + 2 * n * ld, v + 3 * n * ld, ld, cs,
                                nullptr);
                if (!rc) e = copy_cols<double, double>(n, k, v, ld, delta, ldd, nullptr, st);
                if (!rc && e == hipSuccess && its) e = C.stg.download(its, cs.its, sizeof(int) * k);
            } else if (e == hipSuccess) {
                float *v = (float *)vecs;
                // RHS scaled to unit columns; delta scaled back
                std::vector<double> rn(k), bn(k), sc(k);
                (void)bn;
                e = C.ws.ensure_colvec(sizeof(double) * (3 * k + 64));
                if (e == hipSuccess) {
                    Segs RS;
                    RS.add(R, ldr, k);
                    e = C.ws.ensure_small(sizeof(double) * ((size_t)k * k + 64));
                    if (e == hipSuccess) e = gram(n, RS, R, ldr, k, nullptr, C.ws.small, k, C.ws, st);
                    std::vector<double> G((size_t)k * k);
                    if (e == hipSuccess) e = C.stg.download(G.data(), C.ws.small, sizeof(double) * k * k);
                    for (int j = 0; j < k; ++j) {
                        rn[j] = std::sqrt(std::max(G[(size_t)j * k + j], 0.0));
                        sc[j] = rn[j] > 0 ? 1.0 / rn[j] : 0.0;
                    }
                }
                double *dsc = C.ws.colvec, *dusc = C.ws.colvec + k + 16;
                if (e == hipSuccess) e = C.stg.upload(dsc, sc.data(), sizeof(double) * k);
                if (e == hipSuccess) e = C.stg.upload(dusc, rn.data(), sizeof(double) * k);
                if (e == hipSuccess) {
                    CgState<float> cs{(float *)c8, (float *)(c8 + slot), (float *)(c8 + 2 * slot),
                                      (float *)(c8 + 3 * slot), (int *)(c8 + 4 * slot), (int *)(c8 + 5 * slot),
                                      (int *)(c8 + 6 * slot)};
                    cs.done = done;
                    CgRunner<float> runner{n, C.ws, st, nullptr, nullptr, err};
                    DevCsr<float> M = op.csr_of(m32);
                    rc = runner.run(M, R, ldr, dsc, k, maxit, rel_tol, v, v + n * ld, v + 2 * n * ld, v + 3 * n * ld,
                                    ld, cs, nullptr);
                    if (!rc) e = copy_cols<float, double>(n, k, v, ld, delta, ldd, dusc, st);
                    if (!rc && e == hipSuccess && its) e = C.stg.download(its, cs.its, sizeof(int) * k);
                }
            }
        }
        if (e == hipSuccess) e = C.stg.sync();
        bufs.release();
        op.destroy();
        if (rc) return step_fail(rc, err);
        if (e != hipSuccess) return step_hip(e, "gcge_cg");
        return GCGE_OK;
    } catch (...) {
        return step_fail(GCGE_ERR_INTERNAL, "gcge_cg: internal error");
    }
}

struct gcge_amg_s {
    Amg amg;
    std::mutex mu;
    std::string err;
};

extern "C" int gcge_amg_create(const gcge_csr *A, int max_levels, int coarse_max, double strength, void *stream,
                               gcge_amg *out) {
    if (!out) return step_fail(GCGE_ERR_INVALID_ARG, "gcge_amg_create: out is null");
    *out = nullptr;
    if (!A || !csr_ok(A) || max_levels < 1 || max_levels > AMG_MAX_LEVELS || coarse_max < 1 ||
        coarse_max > AMG_COARSE_LIMIT || !(strength >= 0.0) || strength >= 1.0)
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_amg_create: invalid argument");
    try {
        gcge_amg_s *h = new gcge_amg_s;
        const int rc = h->amg.build(to_dev(A), max_levels, coarse_max, strength, (hipStream_t)stream, h->err);
        if (rc) {
            const std::string m = h->err;
            delete h;
            return step_fail(rc, m);
        }
        *out = h;
        return GCGE_OK;
    } catch (...) {
        return step_fail(GCGE_ERR_INTERNAL, "gcge_amg_create: internal error");
    }
}

extern "C" int gcge_amg_levels(gcge_amg h, int *nlevels, int64_t *rows, int64_t *nnz, int cap) {
    if (!h || !nlevels || cap < 0 || (cap > 0 && (!rows || !nnz)))
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_amg_levels: invalid argument");
    const int nl = (int)h->amg.lv.size();
    *nlevels = nl;
    for (int l = 0; l < std::min(nl, cap); ++l) {
        rows[l] = h->amg.rows[l];
        nnz[l] = h->amg.nnz[l];
    }
    return GCGE_OK;
}

extern "C" int gcge_amg_aggregates(gcge_amg h, int level, int32_t *agg) {
    if (!h || !agg || level < 0 || level >= (int)h->amg.agg.size())
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_amg_aggregates: invalid argument");
    std::memcpy(agg, h->amg.agg[level].data(), sizeof(int32_t) * h->amg.agg[level].size());
    return GCGE_OK;
}

extern "C" int gcge_amg_apply(gcge_amg h, const double *B, int64_t ldb, int k, double *Y, int64_t ldy, void *stream) {
    if (!h || k < 0 || k > 128 || (k > 0 && (!B || !Y || ldb < k || ldy < k)))
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_amg_apply: invalid argument");
    if (k == 0) return GCGE_OK;
    try {
        std::lock_guard<std::mutex> lk(h->mu);
        hipStream_t st = (hipStream_t)stream;
        const int rc = h->amg.apply<double>(B, ldb, k, Y, ldy, nullptr, nullptr, st, h->err, nullptr, true);
        if (rc) return step_fail(rc, h->err);
        return GCGE_OK;
    } catch (...) {
        return step_fail(GCGE_ERR_INTERNAL, "gcge_amg_apply: internal error");
    }
}

extern "C" void gcge_amg_destroy(gcge_amg h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    delete h;
}

extern "C" int gcge_pcg(const gcge_csr *A, gcge_amg M, const double *R, int64_t ldr, int k, int maxit,
                        double rel_tol, double *delta, int64_t ldd, int *its, void *stream) {
    if (!M || k < 0 || k > 128 || maxit < 0 || !(rel_tol >= 0.0) || (k > 0 && (!R || !delta || ldr < k || ldd < k)))
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_pcg: invalid argument");
    if (!A || !csr_ok(A) || A->n != M->amg.rows[0])
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_pcg: A does not match the hierarchy");
    if (k == 0) return GCGE_OK;
    try {
        hipStream_t st = (hipStream_t)stream;
        StepCtx &C = step_ctx();
        std::lock_guard<std::mutex> lk(C.mu);
        std::lock_guard<std::mutex> lk2(M->mu);
        C.stg.st = st;
        Operator op;
        int rc = build_step_operator(A, GCGE_B_IDENTITY, nullptr, st, op);
        if (rc) return rc;
        const int64_t n = op.n;
        const int64_t ld = round_up(k, 4);
        Buffers bufs;
        void *vecs = nullptr, *cm = nullptr;
        double *m64 = nullptr;
        hipError_t e = bufs.alloc((void **)&m64, sizeof(double) * std::max<int64_t>(op.nnz, 1));
        if (e == hipSuccess) e = bufs.alloc(&vecs, sizeof(double) * 5 * n * ld);
        if (e == hipSuccess) e = bufs.alloc(&cm, 8 * sizeof(double) * (ld + 16) + 64);
        if (e == hipSuccess) e = op.shifted(0.0, m64, nullptr, st);
        std::string err;
        if (e == hipSuccess) {
            const size_t slot = sizeof(double) * (ld + 16);
            char *c8 = (char *)cm;
            double *v = (double *)vecs;
            CgState<double> cs{(double *)c8, (double *)(c8 + slot), (double *)(c8 + 2 * slot),
                               (double *)(c8 + 3 * slot), (int *)(c8 + 4 * slot), (int *)(c8 + 5 * slot),
                               (int *)(c8 + 6 * slot), (double *)(c8 + 7 * slot)};
            cs.done = (unsigned *)(c8 + 8 * slot);
            e = hipMemsetAsync(cs.done, 0, 64, st);
            CgRunner<double> runner{n, C.ws, st, nullptr, nullptr, err};
            if (e == hipSuccess)
                rc = runner.run_pcg(op.csr_of(m64), M->amg, R, ldr, nullptr, k, maxit, rel_tol, v, v + n * ld,
                                    v + 2 * n * ld, v + 3 * n * ld, v + 4 * n * ld, ld, cs, nullptr);
            if (!rc && e == hipSuccess) e = copy_cols<double, double>(n, k, v, ld, delta, ldd, nullptr, st);
            if (!rc && e == hipSuccess && its) e = C.stg.download(its, cs.its, sizeof(int) * k);
        }
        if (e == hipSuccess) e = C.stg.sync();
        bufs.release();
        op.destroy();
        if (rc) return step_fail(rc, err);
        if (e != hipSuccess) return step_hip(e, "gcge_pcg");
        return GCGE_OK;
    } catch (...) {
        return step_fail(GCGE_ERR_INTERNAL, "gcge_pcg: internal error");
    }
}

static int orth_entry(int64_t n, int b_kind, const void *B, const double *Q, int64_t ldq, int mq, double *W,
                      int64_t ldw, int k, int *kept, void *stream, const OrthOptions &oo) {
    if (n < 1 || k < 0 || mq < 0 || !kept || (k > 0 && (!W || ldw < k)) || (mq > 0 && (!Q || ldq < mq)) ||
        (b_kind != GCGE_B_IDENTITY && b_kind != GCGE_B_DIAG && b_kind != GCGE_B_CSR) ||
        (b_kind != GCGE_B_IDENTITY && !B) || (b_kind == GCGE_B_CSR && !csr_ok((const gcge_csr *)B)))
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_orth: invalid argument");
    *kept = 0;
    if (k == 0) return GCGE_OK;
    try {
        hipStream_t st = (hipStream_t)stream;
        StepCtx &C = step_ctx();
        std::lock_guard<std::mutex> lk(C.mu);
        C.stg.st = st;
        BOp bop;
        bop.kind = b_kind;
        if (b_kind == GCGE_B_DIAG) bop.dg = (const double *)B;
        if (b_kind == GCGE_B_CSR) bop.csr = to_dev((const gcge_csr *)B);
        Buffers bufs;
        double *BW = nullptr;
        const int64_t ldbw = round_up(k, 4);
        hipError_t e = hipSuccess;
        if (b_kind == GCGE_B_CSR) e = bufs.alloc((void **)&BW, sizeof(double) * n * ldbw);
        if (e != hipSuccess) return step_hip(e, "gcge_orth");
        Segs QS;
        QS.add(Q, ldq, mq);
        std::string err;
        int rc = orth_block(n, bop, QS, W, ldw, k, BW, ldbw, oo, C.ws, C.stg, st, kept, nullptr, err);
        if (!rc) e = C.stg.sync();
        bufs.release();
        if (rc) return step_fail(rc, err);
        if (e != hipSuccess) return step_hip(e, "gcge_orth");
        return GCGE_OK;
    } catch (...) {
        return step_fail(GCGE_ERR_INTERNAL, "gcge_orth: internal error");
    }
}

extern "C" int gcge_orth(int64_t n, int b_kind, const void *B, const double *Q, int64_t ldq, int mq, double *W,
                         int64_t ldw, int k, int *kept, void *stream) {
    OrthOptions oo;
    return orth_entry(n, b_kind, B, Q, ldq, mq, W, ldw, k, kept, stream, oo);
}

extern "C" int gcge_orth_mbo(int64_t n, int b_kind, const void *B, const double *Q, int64_t ldq, int mq, double *W,
                             int64_t ldw, int k, int block, int *kept, void *stream) {
    if (block < 0) return step_fail(GCGE_ERR_INVALID_ARG, "gcge_orth_mbo: invalid argument");
    OrthOptions oo;
    oo.algorithm = 2;
    oo.mbo_block = block;
    return orth_entry(n, b_kind, B, Q, ldq, mq, W, ldw, k, kept, stream, oo);
}

extern "C" int gcge_small_eigh(int n, double *a, double *w, double *z, int nwant) {
    if (n < 0 || (n > 0 && (!a || !w)) || nwant < 0 || nwant > n)
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_small_eigh: invalid argument");
    try {
        if (sym_eig(n, a, w, z, nwant) != 0) return step_fail(GCGE_ERR_INTERNAL, "QL iteration did not converge");
        return GCGE_OK;
    } catch (...) {
        return step_fail(GCGE_ERR_OOM, "gcge_small_eigh: host allocation failed");
    }
}

extern "C" int gcge_dense_eig(int n, const double *a, int64_t lda, int nwant, double *w, double *x, int64_t ldx,
                              void *stream) {
    if (n < 1 || n > DENSE_EIG_MAX || nwant < 1 || nwant > n || !a || !w || !x || lda < n || ldx < nwant)
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_dense_eig: invalid argument");
    StepCtx &C = step_ctx();
    std::lock_guard<std::mutex> lk(C.mu);
    const hipStream_t st = (hipStream_t)stream;
    hipError_t e = dense_eig(n, a, lda, nwant, w, x, ldx, C.eig, C.ws, st);
    if (e != hipSuccess) return step_hip(e, "gcge_dense_eig");
    return GCGE_OK;
}

extern "C" int gcge_p_hat(int dim, int nx, const double *xhat, int shift, int n_old, int n_new, double drop_tol,
                          double *phat, int *np) {
    if (dim < 0 || nx < 0 || nx > dim || shift < 0 || n_old < 0 || n_new < 0 || !np || (dim * n_new > 0 && !phat) ||
        (dim * nx > 0 && !xhat) || !(drop_tol >= 0.0))
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_p_hat: invalid argument");
    try {
        *np = p_hat(dim, nx, xhat, shift, n_old, n_new, drop_tol, phat);
        return GCGE_OK;
    } catch (...) {
        return step_fail(GCGE_ERR_OOM, "gcge_p_hat: host allocation failed");
    }
}

extern "C" int gcge_pattern_grad(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colind,
                                 const double *X, int64_t ldx, int nev, const double *wts, double *gval,
                                 void *stream) {
    if (n < 1 || nnz < 0 || nev < 0 || nev > 256 || !rowptr || (nnz > 0 && (!colind || !gval)) ||
        (nev > 0 && (!X || ldx < nev || !wts)))
        return step_fail(GCGE_ERR_INVALID_ARG, "gcge_pattern_grad: invalid argument");
    try {
        hipStream_t st = (hipStream_t)stream;
        StepCtx &C = step_ctx();
        std::lock_guard<std::mutex> lk(C.mu);
        C.stg.st = st;
        hipError_t e = C.ws.ensure_colvec(sizeof(double) * (nev + 64));
        if (e == hipSuccess && nev > 0) e = C.stg.upload(C.ws.colvec, wts, sizeof(double) * nev);
        if (e == hipSuccess) e = pattern_grad(n, rowptr, colind, X, ldx, nev, C.ws.colvec, gval, st);
        if (e == hipSuccess) e = C.stg.sync();
        if (e != hipSuccess) return step_hip(e, "gcge_pattern_grad");
        return GCGE_OK;
    } catch (...) {
        return step_fail(GCGE_ERR_INTERNAL, "gcge_pattern_grad: internal error");
    }
}
