"""Oracle for the preconditioned inner solve (test infrastructure only).

Section 2 suggests algebraic multigrid as the preconditioner of the STEP 6
linear systems when A comes from a PDE discretization, with the shift theta
set to 0.  The paper does not fix which AMG; this oracle (and the library)
use smoothed aggregation (Vanek, Mandel and Brezina, Computing 56, 1996) with
the choices below, so that both sides compute the same preconditioner:

* strength of connection at level l: j != i is strong for row i when
  |a_ij| >= eps_l * sqrt(|a_ii a_jj|), eps_l = eps_0 * 0.5**l with eps_0 =
  0.02 by default (the 27-point Q1 stiffness couples a row to each neighbour
  by about 1/30 of its diagonal, below the 0.08 of the textbook Laplacian
  setting);
* greedy aggregation in row order, two phases:
  1. a row whose strong neighbours are all unaggregated starts an aggregate
     with them (a row without strong neighbours becomes a singleton);
  2. every row left joins the phase-1 aggregate of its strongest neighbour
     among the rows aggregated in phase 1 (scanning neighbours in column
     order, a later one wins only if |a_ij| exceeds the best by a relative
     1e-8, so rounding-level differences never change the choice).  A row
     left after phase 1 was blocked by a strong neighbour aggregated in
     phase 1, so it always has one;
* tentative prolongator: P_t[i, agg(i)] = 1 / sqrt(|agg(i)|) (the constant
  vector on each aggregate, normalized);
* rho_l = max_i sum_j |a_ij| / a_ii (Gershgorin bound of D^-1 A),
  omega_l = 4 / (3 rho_l);
* smoothed prolongator P = (I - omega_l D^-1 A) P_t, restriction R = P^T,
  Galerkin coarse operator A_{l+1} = R A P;
* a level is the last one when it has at most ``coarse_max`` rows, when
  ``max_levels`` levels exist, when it stores more than ``MAX_ROW_FILL``
  (400) entries per row, or when aggregation would keep more than half of its
  rows; the last level is solved exactly (Cholesky);
* symmetric V-cycle: one damped-Jacobi sweep (weight omega_l D^-1) before
  and after the coarse correction, starting from zero.

The V-cycle is a symmetric positive definite operator, so it can precondition
CG; ``pcg_columnwise`` is preconditioned CG column by column with the same
stopping rule as the unpreconditioned STEP 6 solver.

Parity status: see ``PINS`` in ``oracle.core`` (entries ``amg_*`` and
``pcg_columnwise``).
"""
from __future__ import annotations

import numpy as np

from .core import cholesky, solve_lower, solve_lower_t, spmm

STRENGTH_EPS0 = 0.02
TIE_REL = 1e-8
MAX_ROW_FILL = 400


class SparseRows:
    """Minimal CSR container (rows x cols) for the hierarchy; same fields as
    the workload Csr plus the column count."""

    def __init__(self, rowptr, colind, val, ncols):
        self.rowptr = np.asarray(rowptr, dtype=np.int64)
        self.colind = np.asarray(colind, dtype=np.int64)
        self.val = np.asarray(val, dtype=np.float64)
        self.n = len(self.rowptr) - 1
        self.ncols = int(ncols)

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    def to_dense(self):
        D = np.zeros((self.n, self.ncols))
        for i in range(self.n):
            for e in range(self.rowptr[i], self.rowptr[i + 1]):
                D[i, self.colind[e]] += self.val[e]
        return D


def _rows(A):
    rp = np.asarray(A.rowptr, dtype=np.int64)
    ci = np.asarray(A.colind, dtype=np.int64)
    va = np.asarray(A.val, dtype=np.float64)
    return rp, ci, va


def _diag(A):
    rp, ci, va = _rows(A)
    d = np.zeros(A.n)
    for i in range(A.n):
        for e in range(rp[i], rp[i + 1]):
            if ci[e] == i:
                d[i] = va[e]
    return d


def strong_neighbours(A, eps):
    """For each row i, the list of (j, |a_ij|) with j != i strongly connected."""
    rp, ci, va = _rows(A)
    d = _diag(A)
    out = []
    for i in range(A.n):
        row = []
        for e in range(rp[i], rp[i + 1]):
            j = int(ci[e])
            if j != i and abs(va[e]) >= eps * np.sqrt(abs(d[i] * d[j])):
                row.append((j, abs(va[e])))
        out.append(row)
    return out


def aggregate(A, eps):
    """Greedy two-phase aggregation; returns (agg per row, number of aggregates)."""
    n = A.n
    S = strong_neighbours(A, eps)
    agg = np.full(n, -1, dtype=np.int64)
    nagg = 0
    # phase 1: a row whose strong neighbourhood is untouched seeds an aggregate
    for i in range(n):
        if agg[i] >= 0:
            continue
        if all(agg[j] < 0 for j, _ in S[i]):
            agg[i] = nagg
            for j, _ in S[i]:
                agg[j] = nagg
            nagg += 1
    phase1 = agg.copy()
    # phase 2: attach to the strongest phase-1-aggregated neighbour
    for i in range(n):
        if agg[i] >= 0:
            continue
        best, best_a = -1, -1.0
        for j, a in S[i]:
            if phase1[j] < 0:
                continue
            if best < 0 or a > best_a * (1.0 + TIE_REL):
                best, best_a = j, a
        if best >= 0:
            agg[i] = phase1[best]
    assert np.all(agg >= 0)
    return agg, nagg


def tentative_p(agg, nagg):
    """P_t (n x nagg): 1/sqrt(size) on (i, agg(i))."""
    n = len(agg)
    size = np.bincount(agg, minlength=nagg).astype(np.float64)
    return SparseRows(np.arange(n + 1), agg, 1.0 / np.sqrt(size[agg]), nagg)


def gershgorin_rho(A):
    """max_i sum_j |a_ij| / a_ii: an upper bound of the spectral radius of D^-1 A."""
    rp, ci, va = _rows(A)
    d = _diag(A)
    rho = 0.0
    for i in range(A.n):
        s = np.sum(np.abs(va[rp[i]:rp[i + 1]]))
        rho = max(rho, s / abs(d[i]))
    return rho


def dense_of(A):
    """Dense copy of a CSR operator (workload Csr or SparseRows)."""
    ncols = getattr(A, "ncols", A.n)
    rp, ci, va = _rows(A)
    D = np.zeros((A.n, ncols))
    for i in range(A.n):
        for e in range(rp[i], rp[i + 1]):
            D[i, ci[e]] += va[e]
    return D


def _from_dense(D):
    rp = [0]
    ci, va = [], []
    for i in range(D.shape[0]):
        nz = np.nonzero(D[i])[0]
        ci.extend(nz.tolist())
        va.extend(D[i, nz].tolist())
        rp.append(len(ci))
    return SparseRows(rp, ci, va, D.shape[1])


def amg_setup(A, coarse_max=512, max_levels=10, strength=STRENGTH_EPS0):
    """Smoothed-aggregation hierarchy of A (dense products: small sizes only).

    Returns a list of level dicts: ``A`` (CSR of the level operator), ``Ad``
    (dense), ``dinv`` (1/a_ii), ``omega``, ``agg``, ``P`` and ``R`` (dense, for
    every level but the last) and ``L`` (Cholesky factor, last level only).
    """
    levels = []
    cur = A
    lev = 0
    while True:
        Ad = dense_of(cur)
        d = np.diag(Ad).copy()
        if np.any(d <= 0):
            raise ValueError("AMG needs a positive diagonal")
        L = {"A": cur, "Ad": Ad, "dinv": 1.0 / d, "n": cur.n}
        last = cur.n <= coarse_max or lev == max_levels - 1 or cur.nnz > MAX_ROW_FILL * cur.n
        if not last:
            agg, nagg = aggregate(cur, strength * 0.5 ** lev)
            if 2 * nagg > cur.n:
                last = True
        if last:
            L["L"] = cholesky(Ad)
            levels.append(L)
            return levels
        rho = gershgorin_rho(cur)
        omega = 4.0 / (3.0 * rho)
        Pt = dense_of(tentative_p(agg, nagg))
        P = Pt - omega * (L["dinv"][:, None] * (Ad @ Pt))
        L.update(agg=agg, nagg=nagg, omega=omega, rho=rho, Pt=Pt, P=P, R=P.T.copy())
        levels.append(L)
        cur = _from_dense(P.T @ Ad @ P)
        lev += 1


def amg_vcycle(H, b, level=0):
    """x = V(b): the symmetric V-cycle of the hierarchy H applied to b (n x k)."""
    b = np.asarray(b, dtype=np.float64)
    L = H[level]
    if "L" in L:
        return solve_lower_t(L["L"], solve_lower(L["L"], b))
    w = (L["omega"] * L["dinv"])[:, None] if b.ndim == 2 else L["omega"] * L["dinv"]
    x = w * b                                   # pre-smoothing from x = 0
    t = b - L["Ad"] @ x                         # residual
    xc = amg_vcycle(H, L["R"] @ t, level + 1)   # coarse correction
    x = x + L["P"] @ xc
    x = x + w * (b - L["Ad"] @ x)               # post-smoothing
    return x


def pcg_columnwise(A, H, R, maxit=30, rel_tol=1e-2):
    """Preconditioned CG on A x_j = r_j (theta = 0), M^-1 = V-cycle of H.

    Same stopping rule as the unpreconditioned solver: the residual 2-norm
    falls to rel_tol of the initial one, maxit iterations, or p^T A p <= 0.
    Returns (x, iterations per column).
    """
    R = np.asarray(R, dtype=np.float64)
    n, k = R.shape
    X = np.zeros((n, k))
    its = np.zeros(k, dtype=np.int64)
    for j in range(k):
        x = np.zeros(n)
        r = R[:, j].copy()
        z = amg_vcycle(H, r)
        p = z.copy()
        rho = r @ z
        rr0 = r @ r
        rr = rr0
        it = 0
        while it < maxit and rr > rel_tol * rel_tol * rr0:
            q = spmm(A, p)
            pq = p @ q
            if pq <= 0.0:
                break
            alpha = rho / pq
            x = x + alpha * p
            r = r - alpha * q
            rr = r @ r
            z = amg_vcycle(H, r)
            rho_new = r @ z
            p = z + (rho_new / rho) * p
            rho = rho_new
            it += 1
        X[:, j] = x
        its[j] = it
    return X, its
