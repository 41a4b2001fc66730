// Operator setup shared by the solver and the step entry points: the union
// sparsity pattern of A and B, their values on it, the diagonal positions, and
// the shifted operator A - theta B used by the inner CG (STEP 6).
#pragma once

#include <string>

#include "gcge.h"
#include "internal.h"

namespace gcge {

// Pinned staging for host <-> device transfers of small matrices on one
// stream.  Uploads take consecutive slices of a pinned ring; every download
// synchronizes the stream, after which the ring is reused from its start.
struct Stager {
    char *ring = nullptr;
    size_t cap = 0, off = 0;
    hipStream_t st = nullptr;
    hipError_t upload(void *dst, const void *src, size_t bytes);
    hipError_t download(void *dst, const void *src, size_t bytes);
    hipError_t sync();
    void release();
};

// How B acts: identity, diagonal (device vector) or CSR.
struct BOp {
    int kind = GCGE_B_IDENTITY;
    const double *dg = nullptr;   // GCGE_B_DIAG
    DevCsr<double> csr;           // GCGE_B_CSR
};

struct Operator {
    int64_t n = 0, nnz = 0;
    int bkind = GCGE_B_IDENTITY;
    int32_t *rowptr = nullptr, *colind = nullptr;   // union pattern (device, owned)
    double *a = nullptr;                            // A on the union pattern
    double *b = nullptr;                            // B on the union pattern (CSR B)
    double *dg = nullptr;                           // diagonal of B (DIAG B), own copy
    int32_t *dpos = nullptr;                        // position of (i, i) in the union pattern (-1: none)
    int64_t nnzA = 0, nnzB = 0;
    // host copies of the user patterns' position maps into the union pattern
    int32_t *mapA = nullptr, *mapB = nullptr;       // device int32[nnzA], [nnzB]
    bool same_pattern = true;                       // union pattern == A's pattern (and B's for CSR)
    int32_t *uorder = nullptr;                      // SpMM unit order (device) or null
    int64_t plane = 0;                              // coupling distance behind the order

    // Build from user (device) arrays.  Returns a GCGE status; err gets a message.
    int build(const gcge_csr *A, int b_kind, const void *B, hipStream_t st, std::string &err);
    // Replace values keeping the patterns.
    int set_values(const double *a_val, const void *b_val, hipStream_t st, std::string &err);
    // GCGE_ERR_NOT_SPD when a diagonal entry of B is missing, not positive or
    // not finite (B cannot then be positive definite, Section 2); the solver
    // checks its B, the product entry points take any B.
    int check_b_positive(hipStream_t st, std::string &err) const;
    void destroy();

    DevCsr<double> A_csr() const { return DevCsr<double>{n, nnz, rowptr, colind, a, uorder}; }
    template <typename T>
    DevCsr<T> csr_of(const T *val) const { return DevCsr<T>{n, nnz, rowptr, colind, val, uorder}; }
    BOp bop() const {
        BOp o;
        o.kind = bkind;
        o.dg = dg;
        o.csr = DevCsr<double>{n, nnz, rowptr, colind, b, uorder};
        return o;
    }
    // m = A - theta B on the union pattern, and m32 = float(m) when m32 != nullptr.
    hipError_t shifted(double theta, double *m, float *m32, hipStream_t st) const;
    // Y = B X
    hipError_t apply_b(const double *X, int64_t ldx, int k, double *Y, int64_t ldy, hipStream_t st) const;
    // R = A X - B X diag(sigma) with partial sums of r^2 and (Bx)^2 (sigma device);
    // *nparts receives the number of partials per column.
    hipError_t residual(const double *X, int64_t ldx, int k, const double *sigma, double *R, int64_t ldr,
                        double *part, int *nparts, hipStream_t st) const;
};

// Y = B X for a B operator.
hipError_t bop_apply(const BOp &B, int64_t n, const double *X, int64_t ldx, int k, double *Y, int64_t ldy,
                     hipStream_t st);

// STEP 2 machinery.  Statistics of one orthogonalization.
struct OrthStats {
    int grams = 0;
    int dropped = 0;
};

struct OrthOptions {
    double orth_tol = 1e-13;
    double drop_tol = 1e-8;
    int max_pass = 3;
    int algorithm = 3;   // 3: RecursiveOrthSVD (Algorithm 3); 2: modified block orthogonalization (Algorithm 2)
    int mbo_block = 0;   // block size b of Algorithm 2 (0: min(m/4, 200))
    // Algorithm 3 and the deflation against Q: stop a pass loop as soon as a
    // pass's R (or Lambda - I) meets orth_tol, without applying that pass's
    // update (the paper's listing applies it; the result then meets the
    // stopping test itself rather than its square)
    bool skip_final = false;
};

// B-orthonormalize the n x k block W (ld) against the B-orthonormal block Q
// and within itself (Algorithm 3, or Algorithm 2 when opt.algorithm == 2).  BW: n x k scratch (used for CSR B).  On
// success *kept holds the number of output columns (W compacted).
int orth_block(int64_t n, const BOp &B, const Segs &Q, double *W, int64_t ldw, int k, double *BW, int64_t ldbw,
               const OrthOptions &opt, Workspace &ws, Stager &stg, hipStream_t st, int *kept, OrthStats *os,
               std::string &err);

}  // namespace gcge
