// Internal interfaces between the HIP kernels (kernels.hip), the host dense
// linear algebra (dense.cpp) and the solver driver (solver.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace gcge {

// A contiguous range of columns of a row-major block: column j of the segment
// is p[i * ld + j], i = 0 .. n-1, j = 0 .. ncol-1.
struct Seg {
    const double *p;
    int64_t ld;
    int ncol;
};

// Up to MAX_SEG segments read as one block (their columns concatenated), e.g.
// V_u = [X_u, P, W] or [X_c, X_u, P].
constexpr int MAX_SEG = 4;
struct Segs {
    Seg s[MAX_SEG];
    int nseg = 0;
    int total() const {
        int t = 0;
        for (int i = 0; i < nseg; ++i) t += s[i].ncol;
        return t;
    }
    void add(const double *p, int64_t ld, int ncol) {
        if (ncol > 0) s[nseg++] = Seg{p, ld, ncol};
    }
};

// Sparse matrix in CSR form on the device (int32 indices).  uorder, when not
// null, is the order in which the SpMM visits the 64-row units of the matrix
// (a permutation of 0 .. ceil(n/64)-1; the data stay in natural order).
template <typename T>
struct DevCsr {
    int64_t n = 0, nnz = 0;
    const int32_t *rowptr = nullptr;
    const int32_t *colind = nullptr;
    const T *val = nullptr;
    const int32_t *uorder = nullptr;
};

// SpMM traversal order of 64-row units for a pattern (rowptr/colind on the
// host), or an empty vector when natural order is kept.  *plane receives the
// detected coupling distance (0 if none).
std::vector<int32_t> spmm_unit_order(int64_t n, const int32_t *rowptr, const int32_t *colind, int64_t *plane);

// Grow-only device scratch used by the reductions.
struct Workspace {
    double *part = nullptr;      // partial sums (also used as float)
    size_t part_bytes = 0;
    double *small = nullptr;     // small dense matrices (Gram results, coefficient blocks)
    size_t small_bytes = 0;
    double *colvec = nullptr;    // per-column scalars
    size_t colvec_bytes = 0;
    int *iflags = nullptr;       // CG counters
    double *pinned = nullptr;    // pinned host staging (hipHostMalloc)
    size_t pinned_bytes = 0;
    char *orth = nullptr;        // STEP 2 device state: coefficient blocks and flags
    size_t orth_bytes = 0;
    hipError_t ensure_part(size_t bytes);
    hipError_t ensure_orth(size_t bytes);
    hipError_t ensure_small(size_t bytes);
    hipError_t ensure_colvec(size_t bytes);
    hipError_t ensure_pinned(size_t bytes);
    hipError_t ensure_flags();
    void release();
};

// Text returned by gcge_last_error(NULL) on the calling thread.
void set_thread_error(const std::string &msg);

// ------------------------------------------------------------------ launches
// All launches are asynchronous on `st`.

// Upper bound on the number of work-groups (partials per column) a
// row-streaming kernel launches: partial buffers are sized with it.
int max_row_parts();

// Y = M X with M = A (mode 0), M = A - sigma_j diag(dg) (mode 1, dg == nullptr:
// identity), or M = A - sigma_j B on the values vb of a shared pattern (mode 2).
// red = 0: none; red = 1: partial sums of y^2 and (Bx)^2 per column into part
// (layout [2][k][nparts]); red = 2: partial sums of z_j . y_j (layout [k][nparts]).
// *nparts receives the number of partials per column (the launch's grid).
// Operands of the affine SpMM epilogue: row i of the output is
// z_i + w_i (b_i - (A x)_i) with w_i = ws * w[i] (ws when w is null); a null b
// or z reads as zero.  The multigrid V-cycle uses it for the residual
// (z = 0, w = 1), the damped Jacobi sweep (z = x, w = omega / a_ii) and the
// coarse-grid correction (A = P, b = 0, z = x, w = -1, in place).
// With exact, only the k columns of each output row are written (outputs
// owned by a caller); otherwise padding columns up to round_up(k, 16 / sizeof(T))
// may be written too (the library's own blocks), which keeps 16-byte stores.
template <typename T>
struct Affine {
    const T *b = nullptr;
    int64_t ldb = 0;
    const T *z = nullptr;
    int64_t ldz = 0;
    const T *w = nullptr;
    T ws = T(1);
    bool exact = false;
};
// With zdot != nullptr the SpMM also writes partials of the column dots
// y . zdot (part[c * np + g], np in *nparts), as the RED = 2 products do.
// With skip != nullptr the kernel does nothing when skip[0] == 0 (device flag).
template <typename T>
hipError_t spmm_affine(const DevCsr<T> &A, const T *X, int64_t ldx, int k, T *Y, int64_t ldy, const Affine<T> &af,
                       hipStream_t st, const T *zdot = nullptr, int64_t ldzdot = 0, T *part = nullptr,
                       int *nparts = nullptr, const int *skip = nullptr);

template <typename T>
hipError_t spmm(const DevCsr<T> &A, const T *vb, const T *dg, const T *sigma, int mode, int red,
                const T *X, int64_t ldx, int k, T *Y, int64_t ldy, const T *Z, int64_t ldz, T *part,
                int *nparts, hipStream_t st);

// out[j] = sum_p part[j * nparts + p] (fixed order); count = number of column vectors.
template <typename T>
hipError_t colsum(const T *part, int nparts, int k, double *out, hipStream_t st);

// CG state, one entry per column; all device arrays of length k.
template <typename T>
struct CgState {
    T *rr, *rr0, *alpha, *beta;
    int *active, *its, *flags;   // flags[0] = columns still iterating, flags[1] = columns updated this iteration
    T *rz = nullptr;             // preconditioned CG: r . z per column (alpha = rz / pq, beta = rz_new / rz)
    unsigned *done = nullptr;    // zeroed counter: alpha and beta then run one work-group per column
};

template <typename T>
hipError_t cg_init(const double *R, int64_t ldr, const double *rscale, int k, int64_t n, T *r, T *p,
                   T *x, int64_t ld, T *part, int *nparts, CgState<T> cs, hipStream_t st);
template <typename T>
hipError_t cg_init_finish(const T *part, int nparts, int k, CgState<T> cs, hipStream_t st);
template <typename T>
hipError_t cg_alpha(const T *part, int nparts, int k, CgState<T> cs, hipStream_t st);
template <typename T>
hipError_t cg_update_r(int64_t n, int k, const T *q, T *r, int64_t ld, T *part, int *nparts, CgState<T> cs,
                       hipStream_t st);
template <typename T>
hipError_t cg_beta(const T *part, int nparts, int k, double rel_tol, CgState<T> cs, hipStream_t st);
template <typename T>
hipError_t cg_update_xp(int64_t n, int k, T *x, T *p, const T *r, int64_t ld, CgState<T> cs, hipStream_t st);
// Search-direction history (k_cg_update_p_flat, k_cg_fold in kernels.hip):
// cg_hist_ok tells whether a ring of H slots of n x ld vectors can be used
// for k columns (2 <= H <= 32, the flat 16-byte layout); cg_update_p writes
// pn = s + beta p; cg_fold adds sum_j alpha_j p_j over steps first ..
// first+count-1 to x (x = that sum when init), slot j mod H of hist (stride
// sstride elements), alpha_j row j mod H of ar (stride astride).
constexpr int CG_HIST_MAX = 32;
template <typename T>
bool cg_hist_ok(int64_t n, int k, int64_t ld, int H);
template <typename T>
hipError_t cg_update_p(int64_t n, int k, const T *p, T *pn, const T *s, int64_t ld, CgState<T> cs,
                       hipStream_t st);
template <typename T>
hipError_t cg_fold(int64_t n, int k, T *x, int64_t ld, const T *hist, int64_t sstride, int H, const T *ar,
                   int astride, int first, int count, bool init, hipStream_t st);
// Y = diag(d) X (n x k row-major).
template <typename T>
hipError_t scale_rows(int64_t n, int k, const T *d, const T *X, int64_t ldx, T *Y, int64_t ldy, hipStream_t st);
// Preconditioned CG: rz[c] = sum of the partials (init: beta = 0), or, for the
// columns updated this iteration, beta = rz_new / rz and rz = rz_new.
template <typename T>
hipError_t pcg_rz(const T *part, int nparts, int k, bool init, CgState<T> cs, hipStream_t st);
// Partials of the column dots x[:, c] . y[:, c] (part[c * np + g], np in *nparts).
template <typename T>
hipError_t coldot_part(int64_t n, int k, const T *X, int64_t ldx, const T *Y, int64_t ldy, T *part, int *nparts,
                       hipStream_t st);
// SpMM of the CG iteration (q = M p with partial p.q), skipped when flags[0] == 0.
template <typename T>
hipError_t cg_spmm(const DevCsr<T> &M, const T *p, T *q, int64_t ld, int k, T *part, int *nparts,
                   const int *flags, hipStream_t st);

// Device gates: the launches below that take `const int *go` do nothing
// when go != nullptr and *go == 0 (a flag written by an earlier kernel on the
// stream), so that a host-enqueued sequence can skip work decided on the GPU.

// C (m x k, row-major, ldc) = X^T diag(d) Y with X given as segments.
hipError_t gram(int64_t n, const Segs &X, const double *Y, int64_t ldy, int k, const double *d, double *C,
                int64_t ldc, Workspace &ws, hipStream_t st, const int *go = nullptr);
// Bytes of per-chunk partials gram() needs at most, for any shape.
size_t gram_part_bytes_max();
// The same product with the per-chunk partial tiles in the caller's device
// buffer part (part_bytes): when it holds fewer chunks than gram() would use,
// each work-group takes a longer chunk of rows (the summation order then
// differs from gram()'s).  With need != nullptr, *need receives the bytes of
// partials used, and a null part only plans (nothing is launched).
// hipErrorInvalidValue when not even one chunk fits or X has too many tiles.
hipError_t gram_into(int64_t n, const Segs &X, const double *Y, int64_t ldy, int k, const double *d, double *C,
                     int64_t ldc, double *part, size_t part_bytes, size_t *need, hipStream_t st,
                     const int *go = nullptr);

// Y = alpha * X S + beta * Y; X segments (m = total columns), S device row-major
// (m x lds), Y n x k.
hipError_t gemm(int64_t n, const Segs &X, const double *S, int64_t lds, int k, double alpha, double beta,
                double *Y, int64_t ldy, hipStream_t st, const int *go = nullptr);

// Y[:, j] = scale[j] * X[:, j] (scale == nullptr: copy) with type conversion.
template <typename TI, typename TO>
hipError_t copy_cols(int64_t n, int k, const TI *X, int64_t ldx, TO *Y, int64_t ldy, const double *scale,
                     hipStream_t st, const int *go = nullptr);

// ------------------------------------------------ STEP 2 decisions on the device
// The pass loops of Algorithm 3 (and of Algorithm 2 and the deflation against
// [X, P]) are enqueued in full by the host; their "repeat until small" tests
// and the drop decisions run on the device and gate the later launches, so
// STEP 2 needs no host round trip until the kept count at its end.  A dropped
// direction becomes a zero column in place; orth_finish moves the kept
// columns to the front once.
//
// Flag layout (ints): [0] kept count, [1] nonzero once a direction was
// dropped, [ORTH_ALIVE + j] column j alive (j < k), then one (go, upd) pair
// per pass loop: go = the loop's next pass runs, upd = the current pass's
// update is applied.
constexpr int ORTH_ALIVE = 4;
inline int *orth_loop(int *ints, int k, int loop) { return ints + ORTH_ALIVE + k + 2 * loop; }
// kept = 0, dropped = 0, alive[j] = 1, every loop's go = upd = 1.
hipError_t orth_init(int *ints, int k, int nloops, hipStream_t st);
// scale[j] = 1 / sqrt(G[j][j]) for alive columns with G[j][j] > thr (finite),
// else 0 and the column is marked dead (dropped set if it was alive).  Skipped
// when go != nullptr and *go == 0 (scale is then left as is; callers gate the
// scaling with the same flag).
hipError_t orth_norm_scale(const double *G, int ldg, int k, double thr, int *ints, double *scale, const int *go,
                           hipStream_t st);
// The stopping test of a pass on its coefficient block R (rows x cols, ldr):
// small = max |R| <= tol.  loop[1] (upd) = !(allow_skip && small); loop[0]
// (go) = 0 when allow_break && small.  When loop[0] is already 0 the pass is
// off: upd = 0.
hipError_t orth_pass_test(const double *R, int rows, int cols, int ldr, double tol, int allow_skip, int allow_break,
                          int *loop, hipStream_t st);
// One leaf pass of Algorithm 3 (one work-group): Jacobi eigendecomposition
// M = Q Lam Q^T of the leaf Gram (kl <= 16, ldm = kl), directions with
// Lam <= drop_tol (or not finite) dropped, S (kl x kl, lds = kl) = the kept
// columns of Q Lam^{-1/2} in ascending order of Lam, zero columns after them;
// alive flags of the leaf's columns (alive = ints + ORTH_ALIVE + s) set to the
// first kk; dev = max |Lam - 1| over the kept.  upd = 0 and go = 0 when
// skip_final and nothing was dropped and dev <= orth_tol; else upd = 1 and
// go = 0 when dev <= orth_tol or kk = 0.  Off (upd = 0) when go was 0.
hipError_t orth_leaf(const double *M, int kl, double drop_tol, double orth_tol, int skip_final, int *ints, int s,
                     double *S, int *loop, hipStream_t st);
// Algorithm 2, one column w against the kept columns U of its block:
// c = [U, w]^T B w (nu + 1 entries); state[0] = c[nu] on pass 0 (the squared
// B-norm before the projection), state[1] = c[nu] - sum_{i<nu} c_i^2 (after it).
hipError_t orth_mbo_coef(const double *c, int nu, int pass, double *state, hipStream_t st);
// keep = state[0] > 0, state[1] finite and > drop_tol: scale = 1/sqrt(state[1])
// or 0 with the column marked dead.
hipError_t orth_mbo_keep(const double *state, double drop_tol, int *ints, int j, double *scale, hipStream_t st);
// ints[0] = number of alive columns; when a direction was dropped, the alive
// columns of W (n x k, ldw) move to the front in order, in place.
hipError_t orth_finish(int64_t n, double *W, int64_t ldw, int k, int *ints, hipStream_t st);

// ------------------------------- STEP 5 and the STEP 3 assembly on the device
// ptilde (dim x nn, ld nn) = columns shift .. shift+nn-1 of xhat (dim x nx,
// ld nx) with rows 0 .. n_old-1 zeroed (eq. CP_tilde); nrm0[j] = its column norms.
hipError_t phat_init(int dim, int nx, const double *xhat, int shift, int n_old, int nn, double *pt, double *nrm0,
                     hipStream_t st);
// Gram-Schmidt (twice) among the columns of pt, dropping those whose norm falls
// to drop_tol * nrm0[j] or below: phat (dim x n_new, ld n_new) holds the kept
// columns first and zeros after them; *np (device) their count.  dim <= 16384,
// nn <= n_new <= 128.
hipError_t phat_mgs(int dim, int nn, const double *pt, const double *nrm0, double drop_tol, double *phat, int n_new,
                    int *np, hipStream_t st);
// The structured Abar (dim x dim, ld dim) of Section 3.2 from lam (nx Ritz
// values), alpha0 (np x np block of a0, ld lda0, symmetrized) and
// G = [X_u, P, W]^T A W (dim x nw, ld nw).
hipError_t assemble_abar(int dim, int nx, int np, int nw, const double *lam, const double *a0, int lda0,
                         const double *G, double *Ab, hipStream_t st);

// Move columns [src, src+cnt) to [dst, dst+cnt), dst < src, in place.
hipError_t shift_cols_left(int64_t n, double *X, int64_t ld, int dst, int src, int cnt, hipStream_t st);

// Y[:, j] = X[:, perm[j]] (perm device int[k]).
hipError_t gather_cols(int64_t n, int k, const double *X, int64_t ldx, const int *perm, double *Y, int64_t ldy,
                       hipStream_t st);

// Entry (i, j) = 2 u - 1 with u the SplitMix64 draw (col0 + j) * n + i of stream seed.
hipError_t fill_random(int64_t n, int k, int col0, uint64_t seed, double *X, int64_t ld, hipStream_t st);

// Shifted operator values on the union pattern: m = a - theta * b (b == nullptr:
// m = a, then m[dpos[i]] -= theta * dg[i] when dg != nullptr); m32 = float(m).
hipError_t shift_values(int64_t nnz, const double *a, const double *b, int64_t n, const int32_t *dpos,
                        const double *dg, double theta, double *m, float *m32, hipStream_t st);

// *out = the first row i whose B diagonal is missing, not positive or not
// finite: dg[i] (dg != nullptr, diagonal B) or b[dpos[i]] (CSR B on the union
// pattern, dpos[i] < 0 when the row stores no diagonal); n when there is none.
hipError_t first_nonpositive_diag(int64_t n, const int32_t *dpos, const double *b, const double *dg, int *out,
                                  hipStream_t st);

// gval[e] = sum_i w[i] X[r_e, i] X[c_e, i].
hipError_t pattern_grad(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *X, int64_t ldx,
                        int nev, const double *w, double *gval, hipStream_t st);

// gd[i] = sum_j w[j] X[i, j]^2.
hipError_t diag_grad(int64_t n, const double *X, int64_t ldx, int nev, const double *w, double *gd,
                     hipStream_t st);

// ------------------------------------------------------------ device dense
// Largest matrix order of the device eigensolver (LDS per work-group).
constexpr int DENSE_EIG_MAX = 768;

// Grow-only device scratch of dense_eig.
struct DenseEigWork {
    double *buf = nullptr;
    size_t cap = 0;   // doubles
    hipError_t ensure(int n, int nwant);
    void release();
};

// The nwant smallest eigenpairs of the symmetric n x n matrix A (device,
// row-major, lda; not modified): w (device, ascending) and X (device, n x
// nwant row-major, ldx) with X^T X = I.  Asynchronous on st.
hipError_t dense_eig(int n, const double *A, int64_t lda, int nwant, double *w, double *X, int64_t ldx,
                     DenseEigWork &dw, Workspace &ws, hipStream_t st);

// ------------------------------------------------------- multigrid (STEP 6)
// Smoothed-aggregation algebraic multigrid for the STEP 6 systems at theta = 0
// (Section 2 suggests an algebraic multigrid preconditioner there).  The
// hierarchy is built on the host; the V-cycle runs on the device.
struct AmgLevel {
    int64_t n = 0;
    DevCsr<double> A, P, R;   // level operator, prolongator (n x n_next), restriction P^T
    double *w = nullptr;      // omega / a_ii of the damped Jacobi sweep
    DevCsr<float> A32, P32, R32;   // FP32 copies for the V-cycle of the mixed-precision inner solve
    float *w32 = nullptr;
};
struct Amg {
    std::vector<AmgLevel> lv;                 // the last level is solved with cinv
    double *cinv = nullptr;                   // dense inverse of the coarsest operator (row-major)
    std::vector<void *> owned;                // device arrays of the hierarchy
    std::vector<std::vector<int32_t>> agg;    // aggregate of each row, per coarsened level
    std::vector<int64_t> rows, nnz;
    std::vector<double> omega, rho;
    double *work = nullptr;                   // V-cycle vectors for up to kcap columns
    size_t work_bytes = 0;
    int kcap = 0;
    int64_t ldw = 0;
    // A0: device CSR of the level-0 operator (borrowed; must outlive the hierarchy).
    int build(const DevCsr<double> &A0, int max_levels, int coarse_max, double strength, hipStream_t st,
              std::string &err);
    // y = V(b) for k <= 128 columns (b and y n x k row-major, 16-byte aligned
    // rows when ldb, ldy are even).  With part != nullptr the last kernel also
    // writes per-work-group partials of the column dots b . y (part[c * np + g],
    // np in *nparts).
    // With skip != nullptr every SpMM of the cycle is skipped on the device
    // when skip[0] == 0 (the CG's count of active columns).
    // T = float runs the cycle on the FP32 copies (the coarsest solve in FP64);
    // it needs the FP32 level-0 operator from set_level0_f32.
    // exact_out: y is caller-owned, its padding columns are not written.
    template <typename T>
    int apply(const T *b, int64_t ldb, int k, T *y, int64_t ldy, T *part, int *nparts, hipStream_t st,
              std::string &err, const int *skip = nullptr, bool exact_out = false);
    void set_level0_f32(const DevCsr<float> &A32) { if (!lv.empty()) lv[0].A32 = A32; }
    void release();
    ~Amg() { release(); }
};
constexpr int AMG_MAX_LEVELS = 16;
constexpr int64_t AMG_COARSE_LIMIT = 4096;   // largest coarsest level (dense inverse)
constexpr int64_t AMG_MAX_ROW_FILL = 400;    // a level denser than this is not coarsened further
constexpr double AMG_STRENGTH = 0.02;        // default strength threshold at the finest level

// ------------------------------------------------------------- host dense
// Symmetric eigensolver: a (n x n, row-major, destroyed), w ascending, z (n x
// nwant row-major) eigenvectors of the nwant smallest eigenvalues.  Returns 0
// or -1 when the QL iteration does not converge.
int sym_eig(int n, double *a, double *w, double *z, int nwant);

// Cyclic Jacobi for tiny matrices (n <= 64): a row-major destroyed, w ascending,
// v row-major n x n eigenvectors as columns.
int jacobi_small(int n, double *a, double *w, double *v);

// STEP 5 coefficients (row-major dim x n_new output, returns number of columns kept).
int p_hat(int dim, int nx, const double *xhat, int shift, int n_old, int n_new, double drop_tol, double *phat);

// C (m x n row-major) = A^T B with A (k x m), B (k x n) row-major.
void matmul_tn(int k, int m, int n, const double *A, const double *B, double *C);
// C (m x n row-major) = A B with A (m x k), B (k x n) row-major.
void matmul_nn(int m, int k, int n, const double *A, const double *B, double *C);

}  // namespace gcge
