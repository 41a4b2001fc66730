/*
 * gcge.h -- C ABI of the MI355X (gfx950) GCG eigensolver library, libgcge.so.
 *
 * The library computes the nev smallest eigenpairs of the generalized
 * symmetric eigenproblem  A x = lambda B x  (A symmetric, B symmetric
 * positive definite; paper Section 2, the eigenvalue problem) with the GCG
 * algorithm (paper Section 2, Algorithm 1) and the implementing techniques of
 * Section 3: recursive SVD-based B-orthogonalization (Algorithm 3), the
 * reduced Rayleigh-Ritz problem with structured Abar and locking
 * (Section 3.2), the dynamic shift of the inner CG (Section 3.2, STEP 6) and
 * the moving mechanism (Section 3.3).  Paper: Y. Li, Z. Wang, H. Xie, "GCGE:
 * A package for solving large scale eigenvalue problems by parallel block
 * damping inverse power method", arXiv 2111.06552.
 *
 * Conventions shared by every entry point:
 *  - Dense blocks of vectors are ROW-MAJOR: entry (i, j) of an n x k block with
 *    leading dimension ld is at ptr[i * ld + j]; ld >= k.
 *  - Sparse matrices are CSR with int32 row pointers and column indices, the
 *    columns of each row sorted and unique, values float64 (float32 for the
 *    *_f32 entry points).
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary CPU memory.  The caller owns every buffer it
 *    passes and keeps it alive until the call returns (until gcge_destroy
 *    for the matrices given to gcge_create).
 *  - stream arguments are hipStream_t values passed as void* (NULL = the
 *    default stream).  Device results are ordered on that stream; entry points
 *    that return host results synchronize the stream before returning.
 *  - Every function returns a status code (GCGE_OK = 0; negative = error, no
 *    output is valid; GCGE_NOT_CONVERGED = 1 = outputs hold the best
 *    approximations).  No C++ exception crosses the ABI.  A description of the
 *    last error of a handle is returned by gcge_last_error, of a handle-free
 *    call by gcge_last_error(NULL) (per thread).
 */
#ifndef GCGE_H
#define GCGE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GCGE_OK 0
#define GCGE_NOT_CONVERGED 1
#define GCGE_ERR_INVALID_ARG (-1)
#define GCGE_ERR_NOT_SPD (-2)
#define GCGE_ERR_OOM (-3)
#define GCGE_ERR_HIP (-4)
#define GCGE_ERR_INTERNAL (-5)

/* Kind of the B matrix. */
#define GCGE_B_IDENTITY 0 /* B = I; the B argument is NULL                          */
#define GCGE_B_DIAG 1     /* B = diag(d); the B argument is a device double[n]      */
#define GCGE_B_CSR 2      /* B sparse; the B argument is a const gcge_csr* (device) */

/* Precision of the inner CG (option "precision"). */
#define GCGE_PREC_FP64 0  /* everything in FP64                                      */
#define GCGE_PREC_MIXED 1 /* inner CG and its SpMM in FP32 with FP32 accumulation;   */
                          /* residuals, orthogonalization, Rayleigh-Ritz in FP64     */

typedef struct gcge_handle_s *gcge_handle;

/* Square CSR matrix; all three arrays are device memory, borrowed. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int32_t *rowptr; /* [n+1], rowptr[0] = 0, rowptr[n] = nnz */
    const int32_t *colind; /* [nnz] */
    const double *val;     /* [nnz] */
} gcge_csr;

/* Solver statistics of the last gcge_solve. */
typedef struct {
    int32_t iterations;      /* GCG iterations (Algorithm 1 loop passes)                 */
    int32_t nconv;           /* converged (locked) pairs                                 */
    int32_t moves;           /* moving-mechanism moves (Section 3.3)                     */
    int32_t reserved0;
    int64_t cg_iterations;   /* inner CG iterations summed over GCG iterations           */
    int64_t spmm_columns;    /* columns pushed through a sparse product (work measure)   */
    double time_ms[8];       /* wall time per step: 0 init (STEPs 1-3 first pass),
                                1 STEP 2 (orthogonalization of W), 2 STEP 3 (Rayleigh-Ritz:
                                AW, Abar, small eigensolve, rotation), 3 STEP 4 (residuals,
                                locking), 4 STEP 5 (P block), 5 STEP 6 (inner CG),
                                6 final check, 7 total                                    */
    double max_rel_residual; /* max over returned pairs of ||Ax - lam Bx|| / (|lam| ||Bx||) */
    double orth_error;       /* max |X^T B X - I| over the returned vectors               */
    /* With option "profile" = 1: device time (HIP events on the solver stream
     * around each launch) summed per kernel class, the number of launches and
     * the summed column count of the launches (for the GEMMs and Grams: the
     * product of the two column counts).  Classes: 0 CG SpMM (q = (A - theta
     * B) p with p.q), 1 CG residual update (r -= alpha q with r.r), 2 CG
     * iterate and direction update (x += alpha p, p = r + beta p; with a
     * search-direction history only p_new = r + beta p), 3 Ritz rotation (V_u
     * xhat), 4 P block (V_u phat), 5 Gram products of the solver driver
     * (initial and Rayleigh-Ritz), 6 the multigrid V-cycle of the
     * preconditioned CG, 7 the CG iterate formed from the history (x = sum_i
     * alpha_i p_i; columns = block width times the n-vectors it moves: the
     * terms read, x written, and x read when it already held earlier terms). */
    double prof_ms[8];
    int64_t prof_launches[8];
    int64_t prof_columns[8];
    /* The part of classes 0-2 whose launches span a full block (block_size
     * columns); entry 3 is unused (zero). */
    double prof_full_ms[4];
    int64_t prof_full_launches[4];
} gcge_stats;

/* ------------------------------------------------------------------ solver */

/* Create a solver for the nev smallest eigenpairs of (A, B) with relative
 * residual tolerance tol: a pair converges when
 * ||A x - lam B x||_2 / (|lam| ||B x||_2) <= tol.  A (and B for
 * GCGE_B_CSR, B the vector d for GCGE_B_DIAG) are borrowed device memory.
 * The library copies the values it needs (union pattern of A and B, shifted
 * operator, FP32 copies) at creation; the borrowed arrays are read again only
 * by gcge_eig_grad (patterns).  Errors: INVALID_ARG (n < 1, nev < 1,
 * nev > n, tol <= 0, nnz < 0, a pointer NULL), NOT_SPD (a diagonal entry of
 * B that is not positive, not finite, or, for CSR B, not stored: B cannot be
 * positive definite; a B with a positive diagonal is not tested further), OOM,
 * HIP. */
int gcge_create(const gcge_csr *A, int b_kind, const void *B, int nev, double tol, gcge_handle *out);

/* Integer options (defaults in brackets; paper defaults cited):
 *  "block_size"   [max(1, nev/5)]  |P| = |W| = blockSize (Section 3.2, item (2))
 *  "size_x"       [min(nev + 3*block_size, n)]  sizeX (Section 3.2, remark on sizeX)
 *  "max_iter"     [1000]  GCG iterations before GCGE_NOT_CONVERGED
 *  "cg_max_iter"  [30]    inner CG iterations (Section 4.1)
 *  "cg_history"   [32]    0, or 2 .. 32: the inner CG keeps up to min(cg_history,
 *                         cg_max_iter + 1) search directions in device memory (n x
 *                         block_size each, in the CG precision; at most half of the free
 *                         device memory, else fewer slots, else none) and forms the
 *                         correction as sum_i alpha_i p_i when they are used up and at
 *                         the end, in place of an update of it in every CG step: the
 *                         same result to the bit with two fewer passes over an n x
 *                         block_size block per step.  0 updates it in every step.
 *  "precision"    [GCGE_PREC_FP64]
 *  "moving"       [0]     moving mechanism, maxProjDim = 5*block_size (Section 3.3)
 *  "shift"        [1]     dynamic shift theta = largest converged eigenvalue (Section 3.2, STEP 6);
 *                         0 keeps theta = 0
 *  "seed"         [1]     SplitMix64 seed of the random initial block
 *  "check"        [1]     compute max_rel_residual and orth_error at the end
 *  "profile"      [0]     time the launches of the main kernel classes with HIP events
 *                         (fields prof_* of gcge_stats)
 *  "orth"         [3]     STEP 2 orthogonalization: 3 RecursiveOrthSVD (Algorithm 3), 2 modified
 *                         block orthogonalization (Algorithm 2, gcge_orth_mbo)
 *  "orth_block"   [0]     block size of Algorithm 2 (0: min(m/4, 200), Section 3.1)
 *  "orth_skip_final" [0]  1: in Algorithm 3 and the deflation of W against [X, P], a pass
 *                         loop stops at the first pass whose R (or Lambda - I) meets
 *                         orth_tol without applying that pass's update (Algorithm 3 as
 *                         printed applies it); the basis then meets the orth_tol test
 *                         itself, one product fewer per loop
 *  "dense_eig"    [1]     small Rayleigh-Ritz eigenproblem on the device (gcge_dense_eig)
 *                         when its order is at most 768; 0 solves it on the host
 *                         (gcge_small_eigh)
 *  "precond"      [0]     1: STEP 6 runs preconditioned CG with the algebraic multigrid
 *                         V-cycle of A (gcge_amg_create) and theta = 0, as Section 2
 *                         suggests for discretized PDE operators.  With precision MIXED
 *                         the PCG and the V-cycle run in FP32 (FP32 copies of the
 *                         levels; the coarsest solve stays FP64).  The hierarchy is built
 *                         at the first STEP 6 (its time counts in time_ms[5]) and again
 *                         after gcge_update_values; a setup failure (e.g. an operator the
 *                         aggregation cannot coarsen) is returned by gcge_solve.
 *  "amg_levels"   [10]    level limit of that hierarchy (1 .. 16)
 *  "amg_coarse"   [512]   rows at or below which a level is the coarsest (1 .. 4096)
 * (double option "amg_strength" [0.02]: the strength threshold of the hierarchy)
 * Unknown keys or out-of-range values return INVALID_ARG. */
int gcge_set_option_i(gcge_handle h, const char *key, int64_t value);

/* Double options: "tol", "cg_rel_tol" [1e-2] (Section 4.1; 0 runs cg_max_iter
 * iterations on every column), "orth_tol" [1e-13]
 * (the "small enough" tests of Algorithm 3), "drop_tol" [1e-8] (eigenvalue of a
 * leaf Gram of unit-B-norm columns at or below which a direction counts as
 * linearly dependent and is dropped). */
int gcge_set_option_d(gcge_handle h, const char *key, double value);

/* Stream on which the solver enqueues all its work (hipStream_t as void*). */
int gcge_set_stream(gcge_handle h, void *stream);

/* Warm start: the first k columns of the initial block are copied from the
 * device block X0 (n x k, row-major, leading dimension ld) at the next
 * gcge_solve; k = 0 clears it.  k must not exceed sizeX. */
int gcge_set_initial_vectors(gcge_handle h, const double *X0, int64_t ld, int k);

/* Run the GCG iteration.  evals: host double[nev], ascending.  evecs: device,
 * n x nev row-major with leading dimension ld >= nev, B-orthonormal columns
 * (may be NULL).  stats may be NULL.  Returns GCGE_OK, GCGE_NOT_CONVERGED
 * (max_iter reached; outputs hold the current approximations), NOT_SPD (the
 * initial block has no positive B-norm direction), or an error. */
int gcge_solve(gcge_handle h, double *evals, double *evecs, int64_t ld, gcge_stats *stats);

/* Replace the values of A (and of B: a device double[nnzB] for CSR, or the
 * device diagonal for DIAG; NULL keeps B) keeping the sparsity patterns.
 * NOT_SPD as gcge_create for the new B (the handle then holds the new values
 * and gcge_solve must not be called before valid ones are set). */
int gcge_update_values(gcge_handle h, const double *a_val, const void *b_val);

/* Eigenvalue gradients of L = sum_i g[i] lambda_i for the pairs of the last
 * successful gcge_solve, with respect to every stored nonzero of A and B:
 * dlambda_i/dA_jk = x_i[j] x_i[k], dlambda_i/dB_jk = -lambda_i x_i[j] x_i[k]
 * for B-normalized x_i (well separated eigenvalues).  g: host double[nev].
 * gA: device double[nnzA].  gB: device double[nnzB] (CSR B) or double[n]
 * (diagonal B) or NULL.  Each stored entry is an independent variable; for a
 * symmetric perturbation of a_jk and a_kj add both entries.  Returns
 * GCGE_NOT_CONVERGED (gradients still written) when the last solve ended at
 * max_iter: the formula holds for exact eigenpairs only. */
int gcge_eig_grad(gcge_handle h, const double *g, double *gA, double *gB);

void gcge_destroy(gcge_handle h);

/* Text of the last error of h (h = NULL: of the calling thread's last
 * handle-free call).  Valid until the next call on h / on the thread. */
const char *gcge_last_error(gcge_handle h);

/* --------------------------------------------------------- step entry points
 * Each step of one GCG iteration is exported on its own, with explicit
 * device buffers, so that it can be checked against an independent
 * implementation.  They are enqueued on `stream` and use a per-process
 * workspace (allocated on first use, guarded by a mutex: calls from several
 * threads are serialized). */

/* Y = A X (CSR times a block of k vectors; Section 3.4, the product of the
 * matrix with a multi-vector).  X: n x k (ldx), Y: n x k (ldy), device, no
 * overlap.  k >= 0.  Only the k columns of each row of Y are written. */
int gcge_spmm(const gcge_csr *A, const double *X, int64_t ldx, int k, double *Y, int64_t ldy, void *stream);

/* FP32 variant used by the mixed-precision inner CG: values, X and Y float,
 * FP32 accumulation. */
int gcge_spmm_f32(int64_t n, const int32_t *rowptr, const int32_t *colind, const float *val,
                  const float *X, int64_t ldx, int k, float *Y, int64_t ldy, void *stream);

/* Column j of Y is (A - sigma[j] B) x_j; sigma: host double[k].  This is the
 * operator of STEP 6 (sigma_j = theta) and of the STEP 4 residual
 * (sigma_j = lambda_j).  For GCGE_B_CSR, B's pattern may differ from A's.
 * Like the solver's internal blocks, an odd k with an even ldy and 16-byte
 * aligned rows may also overwrite column k of each row of Y (padding). */
int gcge_shifted_spmm(const gcge_csr *A, int b_kind, const void *B, const double *sigma,
                      const double *X, int64_t ldx, int k, double *Y, int64_t ldy, void *stream);

/* STEP 4: R = A X - B X diag(lam) and per-column norms rnorm[j] = ||r_j||_2,
 * bxnorm[j] = ||B x_j||_2.  lam, rnorm, bxnorm: host double[k].  Padding as
 * gcge_shifted_spmm. */
int gcge_residual(const gcge_csr *A, int b_kind, const void *B, const double *lam,
                  const double *X, int64_t ldx, int k, double *R, int64_t ldr,
                  double *rnorm, double *bxnorm, void *stream);

/* Block inner product C = X^T diag(d) Y (d NULL: identity): X n x m (ldx),
 * Y n x k (ldy), d device double[n] or NULL; C host double[m*k] row-major
 * (C[i*k + j] = x_i^T D y_j).  Summation order is fixed (bitwise
 * reproducible). */
int gcge_gram(int64_t n, const double *X, int64_t ldx, int m, const double *Y, int64_t ldy, int k,
              const double *d, double *C, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the block
 * inner product of gcge_gram with no allocation and no host synchronization.
 * C is DEVICE memory here, double[m*k] row-major (C[i*k + j] = x_i^T D y_j),
 * written asynchronously on stream; the other arguments are those of
 * gcge_gram.  The kernels are gcge_gram's; their per-chunk partial tiles live
 * in a library-owned device array of GCGE_NOALLOC_SCRATCH_BYTES (each device
 * the library runs on holds its own until the process ends), not in the
 * workspace gcge_gram grows.  When that array holds fewer chunks than
 * gcge_gram would use, each work-group sums a longer chunk of rows, so the
 * result can differ from gcge_gram's in the last bits (it is still fixed for
 * fixed sizes).  Every call on one device uses that device's array: calls
 * that overlap in time on one device (several streams or threads) race and
 * must be serialized by the caller.  Nothing in the array has to start at
 * zero.  INVALID_ARG when m > 3072, or when one chunk of the m x k partial
 * tiles (ceil(m/64) * ceil(k/64) tiles of 32 KiB for m or k above 32) does
 * not fit the array; HIP on a launch failure. */
#define GCGE_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int gcge_gram_noalloc(int64_t n, const double *X, int64_t ldx, int m, const double *Y, int64_t ldy, int k,
                      const double *d, double *C, void *stream);

/* Y = alpha X S + beta Y with S host double[m*k] row-major (S[i*k + j]):
 * the dense multi-vector linear combination of the Ritz rotation
 * X_new = V xhat (Section 3.2) and of the orthogonalization updates.  X, Y
 * device; if Y overlaps X then k <= 64 and the rows of Y must be the rows of
 * X (in-place row transform). */
int gcge_gemm_update(int64_t n, const double *X, int64_t ldx, int m, const double *S, int k,
                     double alpha, double beta, double *Y, int64_t ldy, void *stream);

/* STEP 6: column-wise CG on (A - theta B) delta_j = r_j from delta = 0, per
 * column stopping at ||res|| <= rel_tol ||r_j||, after maxit iterations, or
 * when p^T (A - theta B) p <= 0.  precision GCGE_PREC_MIXED runs it in FP32
 * (the right-hand side is scaled by 1/||r_j|| on entry and delta scaled back
 * on exit).  R: device n x k (ldr); delta: device n x k (ldd);
 * its: host int[k] (iterations per column) or NULL. */
int gcge_cg(const gcge_csr *A, int b_kind, const void *B, double theta, const double *R, int64_t ldr,
            int k, int maxit, double rel_tol, int precision, double *delta, int64_t ldd, int *its,
            void *stream);

/* STEP 2 for a block W (n x k, ldw, device, overwritten): B-orthogonalize W
 * against the B-orthonormal block Q (n x mq, ldq; Q may be NULL with mq = 0)
 * by repeated block Gram-Schmidt, then orthonormalize it with
 * RecursiveOrthSVD (Algorithm 3, leaf size c = min(k, 16)).  Linearly
 * dependent columns are dropped and later columns move forward; *kept
 * receives the number of output columns (host int). */
int gcge_orth(int64_t n, int b_kind, const void *B, const double *Q, int64_t ldq, int mq,
              double *W, int64_t ldw, int k, int *kept, void *stream);

/* STEP 2 with the modified block orthogonalization of Algorithm 2 (Section
 * 3.1) in place of Algorithm 3: after the same deflation against Q, the
 * columns are taken in blocks of `block` (0: min(k/4, 200)); inside a block
 * each column is B-orthogonalized against the block's kept columns by
 * Gram-Schmidt (two passes) and normalized, or dropped when its squared
 * B-norm falls to drop_tol (1e-8) of its value before; then the block is
 * deflated from all later columns (repeated until the coefficients are
 * small).  Arguments and results as gcge_orth. */
int gcge_orth_mbo(int64_t n, int b_kind, const void *B, const double *Q, int64_t ldq, int mq,
                  double *W, int64_t ldw, int k, int block, int *kept, void *stream);

/* Host-only dense symmetric eigensolver used for the Rayleigh-Ritz problem
 * (the paper calls LAPACK dsyevx; this is the library's own Householder
 * tridiagonalization + implicit QL).  a: host n x n row-major symmetric
 * (destroyed); w: host double[n] ascending; z: host n x nwant row-major, the
 * eigenvectors of the nwant smallest eigenvalues as columns (may be NULL). */
int gcge_small_eigh(int n, double *a, double *w, double *z, int nwant);

/* Device dense symmetric eigensolver of the Rayleigh-Ritz problem (the paper
 * calls LAPACK dsyevx on the host): Householder tridiagonalization,
 * multisection for the eigenvalues, inverse iteration (clusters
 * Gram-Schmidt-orthogonalized) and back-transformation, then Newton-Schulz
 * re-orthonormalization of the eigenvectors.  a: device n x n row-major
 * symmetric (lda, not modified); w: device double[nwant], the nwant smallest
 * eigenvalues ascending; x: device n x nwant row-major (ldx), the matching
 * orthonormal eigenvectors as columns.  1 <= nwant <= n <= 768 (INVALID_ARG
 * otherwise).  Asynchronous on stream. */
int gcge_dense_eig(int n, const double *a, int64_t lda, int nwant, double *w, double *x, int64_t ldx,
                   void *stream);

/* Host-only STEP 5: coefficients phat of the next P block from the Ritz
 * coefficient vectors xhat (dim x nx, row-major): columns shift ..
 * shift+n_new-1 of xhat with rows 0 .. n_old-1 zeroed (eq. CP_tilde), L2
 * orthogonalized against xhat and among themselves (twice each); columns
 * whose norm falls below drop_tol times their initial norm are dropped.
 * phat: host dim x n_new row-major (first *np columns valid). */
int gcge_p_hat(int dim, int nx, const double *xhat, int shift, int n_old, int n_new,
               double drop_tol, double *phat, int *np);

/* ------------------------------------------------- STEP 6 preconditioner */

/* Algebraic multigrid preconditioner of the STEP 6 systems.  Section 2
 * suggests algebraic multigrid as the preconditioner of STEP 6 with theta = 0
 * when A discretizes a PDE; the paper does not fix the method, so this is
 * smoothed aggregation (Vanek, Mandel, Brezina 1996):
 *   strength   |a_ij| >= eps_l sqrt(a_ii a_jj), eps_l = strength * 2^-l at level l
 *              (0 <= strength < 1; 0.02 suits 7- and 27-point stencils);
 *   aggregates rows in order: a row whose strong neighbours are all free
 *              seeds an aggregate with them; a row left joins the aggregate
 *              of its strongest already aggregated neighbour (first in column
 *              order among those within a relative 1e-8 of the largest);
 *   transfer   P = (I - omega D^-1 A) P_t with P_t the normalized aggregate
 *              indicators, omega = 4/(3 rho), rho = max_i sum_j |a_ij| / a_ii;
 *              R = P^T, next level R A P;
 *   coarsest   at most coarse_max rows, the level limit, or no coarsening:
 *              inverted densely (at most 4096 rows, INVALID_ARG otherwise);
 *   V-cycle    one damped Jacobi sweep (omega D^-1) before and after the
 *              coarse correction, from a zero guess: symmetric positive
 *              definite for SPD A.
 */
typedef struct gcge_amg_s *gcge_amg;

/* Build the hierarchy of the SPD matrix A (device CSR, borrowed: the level-0
 * operator is read from it at every gcge_amg_apply / gcge_pcg, so it must
 * stay alive and unchanged until gcge_amg_destroy).  The setup runs on the
 * host (A is copied down once); the coarse levels live in device memory owned
 * by the handle.  max_levels in 1 .. 16, coarse_max in 1 .. 4096, strength
 * in [0, 1).  Errors:
 * INVALID_ARG, NOT_SPD (a non-positive diagonal entry, or a coarsest level
 * that is not positive definite), OOM, HIP. */
int gcge_amg_create(const gcge_csr *A, int max_levels, int coarse_max, double strength, void *stream,
                    gcge_amg *out);

/* Number of levels (the last one is the dense coarsest level) and, for the
 * first min(levels, cap), the rows and stored entries of each level operator
 * (host arrays). */
int gcge_amg_levels(gcge_amg h, int *nlevels, int64_t *rows, int64_t *nnz, int cap);

/* Aggregate index of every row of level `level` (0 .. levels - 2) into the
 * host array agg[rows(level)]. */
int gcge_amg_aggregates(gcge_amg h, int level, int32_t *agg);

/* Y = V(B): one V-cycle applied to the k <= 128 columns of B (device, n x k
 * row-major, ldb) into Y (device, ldy).  Calls on one handle are serialized
 * (the work vectors belong to the handle).  Asynchronous on stream. */
int gcge_amg_apply(gcge_amg h, const double *B, int64_t ldb, int k, double *Y, int64_t ldy, void *stream);

/* STEP 6 with preconditioning: column-wise preconditioned CG on A delta = R
 * (theta = 0) from delta = 0 with M^-1 = the V-cycle of h (built from A);
 * a column stops when ||r|| <= rel_tol ||r_0||, after maxit iterations, or
 * when p^T A p <= 0.  Arguments as gcge_cg (FP64 only). */
int gcge_pcg(const gcge_csr *A, gcge_amg h, const double *R, int64_t ldr, int k, int maxit, double rel_tol,
             double *delta, int64_t ldd, int *its, void *stream);

/* Release the hierarchy (synchronizes the device first). */
void gcge_amg_destroy(gcge_amg h);

/* Eigenvalue-gradient kernel: gval[e] = sum_i wts[i] X[r_e, i] X[c_e, i] over
 * the stored entries e = (r_e, c_e) of the pattern (rowptr, colind) (device),
 * X device n x nev (ldx), wts host double[nev], gval device double[nnz]. */
int gcge_pattern_grad(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colind,
                      const double *X, int64_t ldx, int nev, const double *wts, double *gval,
                      void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GCGE_H */
