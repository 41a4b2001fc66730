"""Reference eigensolver for pencils too large for the dense oracle
(test infrastructure only; see the package docstring).

It computes what GCG approximates, the nev smallest eigenpairs of
A x = lambda B x (Section 2, the eigenvalue problem) with A and B symmetric
positive definite, by a different method: block Lanczos with full
reorthogonalization (Golub & Underwood 1977; Parlett, "The Symmetric
Eigenvalue Problem", chapter 13) on the shift-and-invert operator
K = A^{-1} B at shift zero (Ericsson & Ruhe 1980).  K is self-adjoint in the
B inner product and has the eigenvalues mu = 1 / lambda, so the smallest
lambda are its largest and best separated eigenvalues and the Krylov space
stays small.  One step, with blocks of b columns and Q_0 a seeded random block
made B-orthonormal:

1. W = A^{-1} (B Q_j) by conjugate gradients to a relative residual inner_tol
   (``oracle_cg`` in ``csrc/sparse.c``);
2. two classical Gram-Schmidt passes against every block so far in the B
   inner product: H = Q^T B W, W <- W - Q H (twice); the diagonal block of the
   band matrix T is Q_j^T B W, summed over both passes and symmetrized;
3. W = Q_{j+1} R_j, B-orthonormal, by the Cholesky factor of W^T B W (twice);
   R_j and R_j^T are the off-diagonal blocks of T.

Every ``check_every`` steps the band matrix T is diagonalized with the Jacobi
oracle.  Once the Lanczos residual estimates ||R_j s_last|| / mu of the nev
largest Ritz values are small, the Ritz vectors y = Q s are formed,
lambda = y^T A y / y^T B y, and the explicit relative residual
||A y - lambda B y|| / (|lambda| ||B y||) is computed; the run ends when it is
at most max(tol, floor_i) for every wanted pair.  floor_i is the rounding
floor of a stored vector: entries of y carry relative errors of about
sqrt(m) eps (m the Krylov dimension, from the orthogonalization sums), which
A multiplies by up to ||A||_inf, so the relative residual of y cannot fall
below about sqrt(m) eps ||A||_inf ||B^-1|| / |lambda_i| (above 1e-12 for the
larger eigenvalues of the 64^3 and 48^3 operators, whose ||A||_inf is
1e5); the gate is 16 times that.  Such noise lies along the eigenvectors of
the largest eigenvalues and tilts y by only about sqrt(m) eps, far less than
residual / gap.  The block size must exceed the largest eigenvalue
multiplicity among the wanted pairs (6 for the 3D stencils).

Sparse products use ``oracle_spmm`` (plain CSR row loop, OpenMP over rows);
dense products of the reorthogonalization are matrix products (the only
library primitive); the factorizations are the oracle's own Cholesky and
Jacobi.  Nothing here is shared with the GPU library.
"""
from __future__ import annotations

import time

import numpy as np

from . import core
from .core import cholesky, jacobi_eigh, solve_lower


def _ptr(a):
    return a.ctypes.data


class _Csr:
    """Contiguous int32 / float64 arrays of a CSR matrix for the C kernels."""

    def __init__(self, M):
        self.n = int(M.n)
        self.rowptr = np.ascontiguousarray(M.rowptr, dtype=np.int32)
        self.colind = np.ascontiguousarray(M.colind, dtype=np.int32)
        self.val = np.ascontiguousarray(M.val, dtype=np.float64)


def csr_spmm(M, X):
    """Y = M X for a CSR matrix M and a dense block X (n x k)."""
    lib = core._load()
    Mc = M if isinstance(M, _Csr) else _Csr(M)
    X = np.ascontiguousarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None].copy()
    Y = np.empty_like(X)
    lib.oracle_spmm(Mc.n, _ptr(Mc.rowptr), _ptr(Mc.colind), _ptr(Mc.val), X.shape[1], _ptr(X), _ptr(Y))
    return Y[:, 0] if squeeze else Y


def csr_cg(M, Bm, tol, maxit):
    """Column-wise conjugate gradients on M X = Bm from X = 0 (M SPD).
    Returns (X, iterations per column)."""
    lib = core._load()
    Mc = M if isinstance(M, _Csr) else _Csr(M)
    Bm = np.ascontiguousarray(Bm, dtype=np.float64)
    X = np.empty_like(Bm)
    its = np.zeros(Bm.shape[1], dtype=np.int32)
    rc = lib.oracle_cg(Mc.n, _ptr(Mc.rowptr), _ptr(Mc.colind), _ptr(Mc.val), Bm.shape[1], _ptr(Bm), _ptr(X),
                       float(tol), int(maxit), _ptr(its))
    if rc == -1:
        raise np.linalg.LinAlgError("conjugate gradients met p^T A p <= 0: A is not positive definite")
    if rc != 0:
        raise MemoryError("oracle_cg: allocation failed")
    return X, its


def _b_apply(bkind, B, Bc, X):
    if bkind == "identity":
        return X
    if bkind == "diag":
        return np.asarray(B)[:, None] * X
    return csr_spmm(Bc, X)


def _b_orthonormalize(W, bkind, B, Bc):
    """W = Q R with Q^T B Q = I (Cholesky of the Gram matrix, twice)."""
    b = W.shape[1]
    R = np.eye(b)
    for _ in range(2):
        BW = _b_apply(bkind, B, Bc, W)
        G = W.T @ BW
        L = cholesky(0.5 * (G + G.T))
        W = solve_lower(L, W.T).T          # W L^{-T}
        R = L.T @ R
    return np.ascontiguousarray(W), R


def lanczos_eigs(A, bkind, B, nev, block=8, seed=1, tol=1e-12, inner_tol=1e-14, inner_maxit=50000,
                 max_steps=None, check_every=4, verbose=False):
    """The nev smallest eigenpairs of A x = lambda B x (A, B SPD; B as in the
    other oracle functions: ("identity", None), ("diag", d), ("csr", Csr)).

    Returns (lam, X, info): lam ascending, X (n x nev) with X^T B X = I, and
    info with the number of Lanczos steps, the Krylov dimension, the summed CG
    iterations, the largest explicit relative residual and the wall time.
    Raises RuntimeError when max_steps pass without convergence."""
    t0 = time.time()
    n = int(A.n)
    b = int(block)
    if nev < 1 or nev > n:
        raise ValueError("nev out of range")
    if max_steps is None:
        max_steps = max(8, min((n - 1) // b, 4 * (nev // b + 1) + 60))
    Ac = _Csr(A)
    Bc = _Csr(B) if bkind == "csr" else None
    # ||A||_inf and a bound of ||B^-1|| for the rounding floor of the residual gate
    a_inf = float(np.max(np.add.reduceat(np.abs(Ac.val), Ac.rowptr[:-1]))) if A.nnz else 0.0
    if bkind == "identity":
        binv = 1.0
    elif bkind == "diag":
        binv = 1.0 / float(np.min(B))
    else:
        diag = Bc.val[np.repeat(np.arange(n), np.diff(Bc.rowptr)) == Bc.colind]
        binv = 1.0 / float(np.min(diag))
    # seeded start: uniform(-1, 1) keyed by (seed, col * n + row)
    import workloads as wl
    Q0, _ = _b_orthonormalize(wl.initial_block(seed, n, b), bkind, B, Bc)
    mmax = (max_steps + 1) * b
    Q = np.zeros((n, mmax))
    BQ = Q if bkind == "identity" else np.zeros((n, mmax))
    Q[:, :b] = Q0
    if bkind != "identity":
        BQ[:, :b] = _b_apply(bkind, B, Bc, Q0)
    T = np.zeros((mmax, mmax))
    cg_its = 0
    for j in range(max_steps):
        c0, c1 = j * b, (j + 1) * b
        W, its = csr_cg(Ac, BQ[:, c0:c1], inner_tol, inner_maxit)
        cg_its += int(its.sum())
        D = np.zeros((b, b))
        for _ in range(2):
            H = BQ[:, :c1].T @ W
            W = W - Q[:, :c1] @ H
            D += H[c0:c1]
        T[c0:c1, c0:c1] = 0.5 * (D + D.T)
        Qn, R = _b_orthonormalize(W, bkind, B, Bc)
        Q[:, c1:c1 + b] = Qn
        if bkind != "identity":
            BQ[:, c1:c1 + b] = _b_apply(bkind, B, Bc, Qn)
        T[c1:c1 + b, c0:c1] = R
        T[c0:c1, c1:c1 + b] = R.T
        m = c1
        if m < nev + b or ((j + 1) % check_every != 0 and j + 1 != max_steps):
            continue
        mu, S = jacobi_eigh(T[:m, :m])
        mu, S = mu[::-1], S[:, ::-1]              # largest mu = smallest lambda first
        est = np.linalg.norm(R @ S[m - b:m, :nev], axis=0) / np.abs(mu[:nev])
        if verbose:
            print(f"[lanczos] step {j + 1}: dim {m}, cg its {cg_its}, max est {est.max():.2e}, "
                  f"{time.time() - t0:.1f} s", flush=True)
        if est.max() > 1e-2 * tol:
            continue
        Y = Q[:, :m] @ S[:, :nev]
        AY = csr_spmm(Ac, Y)
        BY = _b_apply(bkind, B, Bc, Y)
        lam = np.sum(Y * AY, axis=0) / np.sum(Y * BY, axis=0)
        res = np.linalg.norm(AY - BY * lam[None, :], axis=0) / (np.abs(lam) * np.linalg.norm(BY, axis=0))
        gate = np.maximum(tol, 16.0 * np.sqrt(m) * np.finfo(float).eps * a_inf * binv / np.abs(lam))
        if verbose:
            print(f"[lanczos]   explicit max relative residual {res.max():.2e}, max residual / gate "
                  f"{np.max(res / gate):.2f}", flush=True)
        if np.all(res <= gate):
            order = np.argsort(lam, kind="stable")
            info = dict(steps=j + 1, dim=m, cg_iterations=cg_its, max_rel_residual=float(res.max()),
                        max_gate=float(gate.max()), seconds=time.time() - t0)
            return lam[order], Y[:, order], info
    raise RuntimeError(f"block Lanczos did not reach {tol} in {max_steps} steps")


__all__ = ["lanczos_eigs", "csr_spmm", "csr_cg"]
