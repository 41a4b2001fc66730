"""Oracle functions (test infrastructure only; see the package docstring).

Notation follows the paper: the pencil (A, B) with A symmetric and B symmetric
positive definite (Section 2, the eigenvalue problem A x = lambda B x); the
subspace V = [X, P, W] with V^T B V = I; X = [X_c, X_n, X_n~] (converged,
active block of blockSize columns, remaining), Section 3.2.

B is described by ``(bkind, B)``: ``("identity", None)``, ``("diag", d)`` with
d a float64 vector, or ``("csr", Csr)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "csrc", f) for f in ("jacobi.c", "sparse.c")]
_SO = os.path.join(_HERE, "_build", "liboracle.so")
_lock = threading.Lock()
_lib = None

# Parity status of each oracle function: what pins it (tests/test_oracle_pins.py).
PINS = {
    "jacobi_eigh": "closed-form 1D/2D Laplacian spectra; diagonal and 2x2 exact cases; "
                   "A V = V diag(w), V^T V = I; brute force vs numpy.linalg.eigh (test-only)",
    "cholesky": "L L^T = B; triangular structure; known factor of a constructed matrix",
    "pencil_eigs": "Q1 FEM closed form (constant kappa); 2D/3D Laplacian closed forms; "
                   "Courant-Fischer sandwich for random diagonal B; residual and B-orthonormality",
    "spmm": "dense matrix product on small operators; Laplacian applied to its closed-form eigenvectors",
    "gram": "explicit small cases; B-weighted inner products vs dense B",
    "residual": "zero residual on closed-form eigenpairs; dense recomputation",
    "cg_columnwise": "Remark rem:shift one-step closed form; n-step termination on SPD n x n; "
                     "correction form equals the initial-guess form (same iterates up to shift)",
    "deflate": "[X,P]^T B W = 0, unit B-norms, each output column parallel to (I - Q Q^T B) w_j; "
               "a column inside span(Q) is dropped",
    "recursive_orth_svd": "W^T B W = I, span preservation, dependent-column drop, "
                          "m/4 - 1 Gram count for c = 16 (Section 3.1 count)",
    "modified_block_orth": "W^T B W = I, X0^T B W = 0, span preservation, m + m/b - 1 count (Section 3.1)",
    "assemble_abar": "equals the explicit V_u^T A V_u on a random pencil after one exact GCG step",
    "p_hat": "hand-derived coefficients of two small cases (the zeroed rows and the column window of eq. "
             "CP_tilde both matter); [xhat, phat]^T [xhat, phat] = I; rank loss on a complete xhat",
    "eig_grad": "central finite differences of pencil_eigs on small random pencils",
    "lanczos.lanczos_eigs": "closed-form 2D/3D Laplacian and Q1 spectra with their multiplicities (a "
                            "block of 8 holds the sixfold clusters); the dense Jacobi oracle on diagonal-B and "
                            "variable-coefficient pencils (eigenvalues and eigenvectors); B-orthonormality and "
                            "explicit residuals",
    "lanczos.csr_spmm": "dense matrix product",
    "lanczos.csr_cg": "numpy.linalg.solve on SPD systems; zero right-hand side; breakdown on an indefinite matrix",
    "amg.aggregate": "hand-derived aggregates of the 1D Laplacian and of small graphs (strongest-link "
                     "rule, tie margin, weak links); partition of the rows",
    "amg.amg_setup": "hand-derived smoothed prolongator column (1D); P_t^T P_t = I; the V-cycle checks below",
    "amg.amg_vcycle": "one level equals numpy.linalg.solve; symmetric positive definite; error "
                      "propagation I - V A contracts (spectral radius < 0.7) on 2D/3D stencils",
    "amg.pcg_columnwise": "exact preconditioner converges in one step to numpy.linalg.solve; solves "
                          "A x = r to 1e-10; far fewer iterations than plain CG",
}


# ---------------------------------------------------------------------------
# dense kernels
# ---------------------------------------------------------------------------

def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        need = (not os.path.exists(_SO)) or os.path.getmtime(_SO) < max(os.path.getmtime(f) for f in _SRCS)
        if need:
            build()
        lib = ctypes.CDLL(_SO)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.oracle_jacobi_eigh.restype = ctypes.c_int
        lib.oracle_jacobi_eigh.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int]
        lib.oracle_spmm.restype = None
        lib.oracle_spmm.argtypes = [i64, vp, vp, vp, ctypes.c_int, vp, vp]
        lib.oracle_cg.restype = ctypes.c_int
        lib.oracle_cg.argtypes = [i64, vp, vp, vp, ctypes.c_int, vp, vp, ctypes.c_double, ctypes.c_int, vp]
        _lib = lib
        return lib


def build():
    """Compile the oracle's C part (gcc, OpenMP) into oracle/_build."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, *_SRCS, "-lm"])
    os.replace(tmp, _SO)


def jacobi_eigh(C, max_sweeps: int = 100):
    """All eigenpairs of the symmetric matrix C by cyclic Jacobi rotations.

    Returns (w, V): eigenvalues ascending and orthonormal eigenvectors as the
    columns of V.  (The paper computes the Rayleigh-Ritz eigenpairs with
    LAPACK's dsyevx, Section 3.2; the oracle uses its own Jacobi instead.)
    """
    C = np.array(C, dtype=np.float64, order="C", copy=True)
    n = C.shape[0]
    if n == 0:
        return np.zeros(0), np.zeros((0, 0))
    C = 0.5 * (C + C.T)
    C = np.ascontiguousarray(C)
    V = np.zeros((n, n))
    lib = _load()
    rc = lib.oracle_jacobi_eigh(n, C.ctypes.data, V.ctypes.data, max_sweeps)
    if rc < 0:
        raise RuntimeError("Jacobi did not converge in %d sweeps" % max_sweeps)
    w = np.diag(C).copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]


def cholesky(B):
    """Lower-triangular L with L L^T = B (B symmetric positive definite),
    column by column."""
    B = np.array(B, dtype=np.float64)
    n = B.shape[0]
    L = np.zeros_like(B)
    for j in range(n):
        s = B[j, j] - L[j, :j] @ L[j, :j]
        if s <= 0.0:
            raise np.linalg.LinAlgError("matrix is not positive definite")
        L[j, j] = np.sqrt(s)
        L[j + 1:, j] = (B[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def solve_lower(L, X):
    """L^{-1} X by forward substitution."""
    X = np.array(X, dtype=np.float64)
    Y = np.zeros_like(X)
    for i in range(L.shape[0]):
        Y[i] = (X[i] - L[i, :i] @ Y[:i]) / L[i, i]
    return Y


def solve_lower_t(L, X):
    """L^{-T} X by back substitution."""
    X = np.array(X, dtype=np.float64)
    Y = np.zeros_like(X)
    n = L.shape[0]
    for i in range(n - 1, -1, -1):
        Y[i] = (X[i] - L[i + 1:, i] @ Y[i + 1:]) / L[i, i]
    return Y


# ---------------------------------------------------------------------------
# sparse operators (Section 3.4: the only user operation GCG needs is the
# product of the matrix with a block of vectors)
# ---------------------------------------------------------------------------

def spmm(A, X):
    """Y = A X for CSR A (n x n) and dense X (n x k): y_i = sum_e a_e x_{col(e)}."""
    X = np.asarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    n, k = A.n, X.shape[1]
    Y = np.zeros((n, k))
    counts = np.diff(A.rowptr.astype(np.int64))
    nonempty = counts > 0
    if A.nnz:
        contrib = A.val[:, None] * X[A.colind.astype(np.int64)]
        starts = A.rowptr[:-1].astype(np.int64)[nonempty]
        Y[nonempty] = np.add.reduceat(contrib, starts, axis=0)
    return Y[:, 0] if squeeze else Y


def spmm_rows(A, X, rows):
    """Rows ``rows`` of A X, one row at a time (for sampled checks at full size)."""
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros((len(rows), X.shape[1]))
    for t, i in enumerate(rows):
        a, b = int(A.rowptr[i]), int(A.rowptr[i + 1])
        for e in range(a, b):
            out[t] += A.val[e] * X[int(A.colind[e])]
    return out


def apply_b(bkind, B, X):
    """B X for B = identity, diagonal or CSR."""
    X = np.asarray(X, dtype=np.float64)
    if bkind == "identity":
        return X.copy()
    if bkind == "diag":
        return (B[:, None] * X) if X.ndim == 2 else B * X
    return spmm(B, X)


def dense_b(bkind, B, n):
    if bkind == "identity":
        return np.eye(n)
    if bkind == "diag":
        return np.diag(B)
    return B.to_dense()


def shifted_spmm(A, bkind, B, X, sigma):
    """Column j of the result is (A - sigma_j B) x_j (STEP 6's operator A - theta B
    for a common sigma; STEP 4's residual for sigma_j = lambda_j)."""
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (X.shape[1],))
    return spmm(A, X) - apply_b(bkind, B, X) * sigma[None, :]


def gram(X, Y, d=None):
    """C = X^T diag(d) Y (d=None: identity); the block inner product of Section 3.4."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    if d is not None:
        Y = np.asarray(d)[:, None] * Y
    return X.T @ Y


def b_gram(bkind, B, X, Y):
    """X^T B Y."""
    return X.T @ apply_b(bkind, B, Y)


# ---------------------------------------------------------------------------
# STEP 4: residuals and the convergence test
# ---------------------------------------------------------------------------

def residual(A, bkind, B, X, lam):
    """R = A X - B X diag(lam) with per-column norms ||r_j|| and ||B x_j||.

    The convergence measure is ||A x - lambda B x|| / (|lambda| ||B x||)
    (the relative residual used for the solver's tolerance; the paper's
    Section 4 states ||Ax - lambda x||/||x|| for standard problems and
    ||Ax - lambda Bx||/(lambda ||B^{1/2} x||) for the FEM pencil)."""
    lam = np.asarray(lam, dtype=np.float64)
    BX = apply_b(bkind, B, X)
    R = spmm(A, X) - BX * lam[None, :]
    rn = np.sqrt(np.sum(R * R, axis=0))
    bn = np.sqrt(np.sum(BX * BX, axis=0))
    return R, rn, bn


def relative_residuals(A, bkind, B, X, lam):
    _, rn, bn = residual(A, bkind, B, X, lam)
    lam = np.asarray(lam, dtype=np.float64)
    return rn / (np.abs(lam) * bn)


def converged_prefix(rel, tol):
    """Length of the leading run of converged pairs (locking keeps only a
    consecutive prefix, Section 3.2 STEP 4)."""
    c = 0
    for r in rel:
        if r <= tol:
            c += 1
        else:
            break
    return c


# ---------------------------------------------------------------------------
# STEP 6: inexact shifted CG, column by column
# ---------------------------------------------------------------------------

def cg_columnwise(A, bkind, B, theta, R, maxit=30, rel_tol=1e-2, x0=None):
    """Conjugate gradients on (A - theta B) x_j = r_j for each column j.

    Starts from x0 (default 0); each column stops when its residual norm is at
    most rel_tol times the initial one, after ``maxit`` iterations, or when
    p^T (A - theta B) p <= 0 (the shifted matrix need not be positive
    definite, Section 3.2 STEP 6).  The paper's default is a 1% reduction or 30
    iterations (Section 4.1).  Returns (x, iterations per column).
    """
    R = np.asarray(R, dtype=np.float64)
    n, k = R.shape
    X = np.zeros((n, k)) if x0 is None else np.array(x0, dtype=np.float64)
    its = np.zeros(k, dtype=np.int64)

    def op(v):
        return shifted_spmm(A, bkind, B, v[:, None], theta)[:, 0]

    for j in range(k):
        x = X[:, j].copy()
        r = R[:, j] - (op(x) if x0 is not None else 0.0)
        p = r.copy()
        rr = r @ r
        rr0 = rr
        it = 0
        while it < maxit and rr > rel_tol * rel_tol * rr0:
            q = op(p)
            pq = p @ q
            if pq <= 0.0:
                break
            alpha = rr / pq
            x = x + alpha * p
            r = r - alpha * q
            rr_new = r @ r
            beta = rr_new / rr
            p = r + beta * p
            rr = rr_new
            it += 1
        X[:, j] = x
        its[j] = it
    return X, its


# ---------------------------------------------------------------------------
# STEP 2: B-orthogonalization
# ---------------------------------------------------------------------------

def deflate(W, Q, bkind, B, tol=1e-13, max_pass=3, drop_tol=1e-8, skip_final=False):
    """Remove from W its B-components along the B-orthonormal block Q:
    repeat R = Q^T B W, W <- W - Q R until max|R| <= tol (at most max_pass
    passes).  This is the top split of the recursive orthogonalization, where
    the left part [X, P] is already B-orthonormal (Section 3.2 STEP 6, last
    paragraph; Algorithm 3), and the first loop of Algorithm 2.

    The columns of W are first scaled to unit B-norm.  A column whose squared
    B-norm falls to drop_tol or below in the first pass lay in span(Q): it is
    linearly dependent and dropped (later columns move forward); the others are
    rescaled to unit B-norm.  Returns (W_out, passes).

    skip_final (an option, not the paper's listing): from the second pass on,
    stop as soon as max|R| <= tol without applying that pass's update; W then
    meets the stopping test itself.  passes counts the applied updates."""
    W = np.array(W, dtype=np.float64)
    passes = 0
    if Q.shape[1] == 0 or W.shape[1] == 0:
        return W, passes
    nrm = np.sqrt(np.maximum(np.sum(W * apply_b(bkind, B, W), axis=0), 0.0))
    W = W[:, nrm > 0] / nrm[nrm > 0][None, :]
    for p in range(max_pass):
        Rm = b_gram(bkind, B, Q, W)
        if skip_final and p > 0 and np.max(np.abs(Rm)) <= tol:
            break
        W = W - Q @ Rm
        passes += 1
        if p == 0:
            nu2 = np.sum(W * apply_b(bkind, B, W), axis=0)
            keep = nu2 > drop_tol
            W = W[:, keep] / np.sqrt(nu2[keep])[None, :]
            if W.shape[1] == 0:
                break
        elif np.max(np.abs(Rm)) <= tol:
            break
    return W, passes


def recursive_orth_svd(X, bkind, B, c=None, leaf_tol=1e-13, int_tol=1e-13, max_pass=3,
                       drop_tol=1e-8, leaf_passes=None, int_passes=None, counters=None, skip_final=False):
    """RecursiveOrthSVD (Algorithm 3) of the columns of X in the B inner product.

    Columns [s, e) with e - s <= c are a leaf: repeat M = X^T B X, M = Q Lam Q^T,
    X <- X Q Lam^{-1/2} until max|Lam - I| <= leaf_tol.  Otherwise split at
    s + length // 2, orthogonalize the left half, repeat R = (B X1)^T X2,
    X2 <- X2 - X1 R until max|R| <= int_tol, then orthogonalize the right half.
    c defaults to min(m, 16).  The columns are first scaled to unit B-norm;
    directions with Lam <= drop_tol are then linearly dependent and are
    dropped; later columns move forward into their place.  (An exact duplicate
    inside one leaf shows up as an eigenvalue at the rounding floor of M,
    about 1e-16 ||M||, so the threshold has to sit well above it: 1e-8, a
    remaining B-norm of 1e-4 of the unit input.)

    ``leaf_passes`` / ``int_passes`` force fixed pass counts (used to check the
    paper's count of global reductions).  ``counters['gram']`` counts Gram
    products (the global reductions of the distributed version).

    skip_final (an option, not the paper's listing, which applies the update of
    the last pass): a leaf pass whose Lam already meets leaf_tol with nothing
    dropped, or a node pass whose R meets int_tol, ends its loop without
    applying its update.  ``counters['update']`` counts applied updates.

    Returns (X_out, kept) with X_out of shape (n, kept).
    """
    X = np.array(X, dtype=np.float64)
    m = X.shape[1]
    if counters is None:
        counters = {}
    counters.setdefault("gram", 0)
    counters.setdefault("update", 0)
    if m == 0:
        return X, 0
    # "eigenvalues close to zero" is judged on the unit-normalized input:
    # scale every column to unit B-norm first (exact zero columns are dropped)
    nrm = np.sqrt(np.maximum(np.sum(X * apply_b(bkind, B, X), axis=0), 0.0))
    X = X[:, nrm > 0] / nrm[nrm > 0][None, :]
    m = X.shape[1]
    if m == 0:
        return X, 0
    if c is None:
        c = min(m, 16)

    def rec(s, e):
        length = e - s
        if length <= c:
            k = length
            npass = 0
            while True:
                blk = X[:, s:s + k]
                M = b_gram(bkind, B, blk, blk)
                counters["gram"] += 1
                lam, Qm = jacobi_eigh(M)
                keep = lam > drop_tol
                kk = int(np.sum(keep))
                if skip_final and leaf_passes is None and kk == k and np.max(np.abs(lam - 1.0)) <= leaf_tol:
                    break
                X[:, s:s + kk] = blk @ (Qm[:, keep] / np.sqrt(lam[keep])[None, :])
                counters["update"] += 1
                k = kk
                npass += 1
                if leaf_passes is not None:
                    if npass >= leaf_passes:
                        break
                elif k == 0 or np.max(np.abs(lam[keep] - 1.0)) <= leaf_tol or npass >= max_pass:
                    break
            return k
        s1, e1 = s, s + length // 2
        s2, e2 = e1, e
        k1 = rec(s1, e1)
        if k1 > 0:
            npass = 0
            while True:
                X1 = X[:, s1:s1 + k1]
                X2 = X[:, s2:e2]
                Rm = apply_b(bkind, B, X1).T @ X2
                counters["gram"] += 1
                if skip_final and int_passes is None and np.max(np.abs(Rm)) <= int_tol:
                    break
                X[:, s2:e2] = X2 - X1 @ Rm
                counters["update"] += 1
                npass += 1
                if int_passes is not None:
                    if npass >= int_passes:
                        break
                elif np.max(np.abs(Rm)) <= int_tol or npass >= max_pass:
                    break
        k2 = rec(s2, e2)
        if k1 < e1 - s1:
            X[:, s1 + k1:s1 + k1 + k2] = X[:, s2:s2 + k2].copy()
        return k1 + k2

    kept = rec(0, m)
    return X[:, :kept].copy(), kept


def modified_block_orth(X, X0, bkind, B, b=None, tol=1e-13, max_pass=3, drop_tol=1e-4, counters=None):
    """Modified block orthogonalization (Algorithm 2): deflate the B-orthonormal
    X0 from X (repeated), then for blocks X_1..X_l of b columns: orthogonalize
    X_k by modified Gram-Schmidt, then deflate X_k from the later blocks
    (repeated).  b defaults to min(m/4, 200).  A column whose B-norm after
    orthogonalization is at most drop_tol times its B-norm on entry (after the
    X0 deflation) is linearly dependent and is dropped (later columns move
    forward).  The default drop_tol = 1e-4 is the threshold of the
    recursive orthogonalization in squared form (a squared B-norm of 1e-8 of
    the unit input; see recursive_orth_svd).  Returns (X_out, kept)."""
    X = np.array(X, dtype=np.float64)
    m = X.shape[1]
    if counters is None:
        counters = {}
    counters.setdefault("gram", 0)
    if X0 is not None and X0.shape[1] > 0:
        for _ in range(max_pass):
            Rm = b_gram(bkind, B, X0, X)
            counters["gram"] += 1
            X = X - X0 @ Rm
            if np.max(np.abs(Rm)) <= tol:
                break
    if m == 0:
        return X, 0
    if b is None:
        b = max(1, min(m // 4, 200))
    cols = [X[:, j].copy() for j in range(m)]
    # a column's B-norm on entry: the reference of the dependence test, so that a
    # column reduced to rounding by the deflation of earlier blocks is dropped
    norms_in = [np.sqrt(max(c @ apply_b(bkind, B, c), 0.0)) for c in cols]
    out = []
    k = 0
    while k < len(cols):
        blk = cols[k:k + b]
        kept_blk = []
        for jb, v in enumerate(blk):
            nrm0 = norms_in[k + jb]
            for _ in range(2):
                for u in kept_blk:
                    v = v - u * (u @ apply_b(bkind, B, v))
            nrm = np.sqrt(max(v @ apply_b(bkind, B, v), 0.0))
            counters["gram"] += 1
            if nrm0 > 0 and nrm > drop_tol * nrm0:
                kept_blk.append(v / nrm)
        out.extend(kept_blk)
        rest = cols[k + b:]
        if rest and kept_blk:
            Xk = np.stack(kept_blk, axis=1)
            Xr = np.stack(rest, axis=1)
            for _ in range(max_pass):
                Rm = apply_b(bkind, B, Xk).T @ Xr
                counters["gram"] += 1
                Xr = Xr - Xk @ Rm
                if np.max(np.abs(Rm)) <= tol:
                    break
            cols = cols[:k + b] + [Xr[:, j].copy() for j in range(Xr.shape[1])]
        k += b
    if not out:
        return np.zeros((X.shape[0], 0)), 0
    Xo = np.stack(out, axis=1)
    return Xo, Xo.shape[1]


# ---------------------------------------------------------------------------
# STEP 3 and STEP 5: the reduced Rayleigh-Ritz problem and the P block
# ---------------------------------------------------------------------------

def assemble_abar(lam_u, alpha0, G, nx, np_, nw):
    """Abar over V_u = [X_u, P, W] with the structure of Section 3.2:
    X_u^T A X_u = diag(lam_u), X_u^T A P = 0, P^T A P = alpha0 = phat^T Abar_old phat,
    and the last block column [alpha1; alpha2; alpha3] = [X_u, P, W]^T A W = G
    (alpha3 symmetrized)."""
    dim = nx + np_ + nw
    Ab = np.zeros((dim, dim))
    Ab[np.arange(nx), np.arange(nx)] = lam_u
    if np_:
        Ab[nx:nx + np_, nx:nx + np_] = alpha0
    if nw:
        Ab[:, nx + np_:] = G
        Ab[nx + np_:, :] = G.T
        a3 = G[nx + np_:, :]
        Ab[nx + np_:, nx + np_:] = 0.5 * (a3 + a3.T)
    return Ab


def rayleigh_ritz(Abar, nwant):
    """The nwant smallest eigenpairs of Abar (Section 3.2 STEP 3)."""
    w, V = jacobi_eigh(Abar)
    return w[:nwant], V[:, :nwant]


def p_hat(xhat, shift, n_old, n_new, drop_tol=1e-10):
    """STEP 5 coefficients of the next P block.

    ptilde = columns shift .. shift+n_new-1 of xhat (the next active block) with
    the rows of the current active block X_n (rows 0 .. n_old-1 of V_u) set to
    zero (eq. CP_tilde); then ptilde is orthogonalized in the L2 inner product
    against all columns of xhat and among itself (classical Gram-Schmidt against
    xhat and modified Gram-Schmidt within, each twice).  A column whose norm
    drops below drop_tol times its norm before orthogonalization is dropped.
    Returns phat with [xhat, phat]^T [xhat, phat] = I (eq. Equality_Cpx).
    """
    xhat = np.asarray(xhat, dtype=np.float64)
    dim = xhat.shape[0]
    pt = xhat[:, shift:shift + n_new].copy()
    pt[:n_old, :] = 0.0
    nrm0 = np.sqrt(np.sum(pt * pt, axis=0))
    for _ in range(2):
        pt = pt - xhat @ (xhat.T @ pt)
    cols = []
    for j in range(pt.shape[1]):
        v = pt[:, j].copy()
        for _ in range(2):
            for u in cols:
                v = v - u * (u @ v)
        nrm = np.sqrt(v @ v)
        if nrm0[j] > 0 and nrm > drop_tol * nrm0[j]:
            cols.append(v / nrm)
    if not cols:
        return np.zeros((dim, 0))
    return np.stack(cols, axis=1)


# ---------------------------------------------------------------------------
# the definition: the nev smallest eigenpairs of the pencil
# ---------------------------------------------------------------------------

def pencil_eigs(A, bkind, B, nev=None):
    """The smallest nev eigenpairs of A x = lambda B x (Section 2), from the
    plain definition: reduce to a standard problem (B = I: C = A; B = D:
    C = D^{-1/2} A D^{-1/2}; general B: Cholesky B = L L^T, C = L^{-1} A L^{-T})
    and diagonalize C densely by Jacobi.  Returns (lam, X) with X^T B X = I."""
    n = A.n
    Ad = A.to_dense()
    if bkind == "identity":
        w, Y = jacobi_eigh(Ad)
        X = Y
    elif bkind == "diag":
        s = 1.0 / np.sqrt(np.asarray(B, dtype=np.float64))
        C = s[:, None] * Ad * s[None, :]
        w, Y = jacobi_eigh(C)
        X = s[:, None] * Y
    else:
        L = cholesky(B.to_dense())
        C = solve_lower(L, solve_lower(L, Ad).T)
        w, Y = jacobi_eigh(C)
        X = solve_lower_t(L, Y)
    if nev is None:
        nev = n
    return w[:nev], X[:, :nev]


# ---------------------------------------------------------------------------
# eigenvalue gradients
# ---------------------------------------------------------------------------

def eig_grad(A, X, lam, g, kind="A"):
    """Gradient of sum_i g_i lambda_i with respect to each stored nonzero of A
    (kind="A") or of a CSR B with A's argument giving B's pattern (kind="B"),
    for B-normalized eigenvectors X of well-separated eigenvalues:
    d lambda_i / d a_jk = x_i[j] x_i[k],  d lambda_i / d b_jk = -lambda_i x_i[j] x_i[k]."""
    X = np.asarray(X, dtype=np.float64)
    w = np.asarray(g, dtype=np.float64)
    if kind == "B":
        w = -w * np.asarray(lam, dtype=np.float64)
    rows = A.row_of_entry()
    cols = A.colind.astype(np.int64)
    return np.sum(X[rows] * X[cols] * w[None, :], axis=1)


def eig_grad_diag(X, lam, g):
    """Gradient of sum_i g_i lambda_i with respect to a diagonal B: -sum_i g_i lambda_i x_i[j]^2."""
    X = np.asarray(X, dtype=np.float64)
    w = -np.asarray(g, dtype=np.float64) * np.asarray(lam, dtype=np.float64)
    return np.sum(X * X * w[None, :], axis=1)



__all__ = [
    "build", "jacobi_eigh", "cholesky", "solve_lower", "solve_lower_t", "spmm", "spmm_rows", "apply_b",
    "dense_b", "shifted_spmm", "gram", "b_gram", "residual", "relative_residuals", "converged_prefix",
    "cg_columnwise", "deflate", "recursive_orth_svd", "modified_block_orth", "assemble_abar",
    "rayleigh_ritz", "p_hat", "pencil_eigs", "eig_grad", "eig_grad_diag",
]
