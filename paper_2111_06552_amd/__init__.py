"""MI355X (gfx950) GCG eigensolver: Python binding of libgcge.so.

Computes the nev smallest eigenpairs of A x = lambda B x (A symmetric, B
symmetric positive definite) with the GCG algorithm of Li, Wang and Xie,
"GCGE: A package for solving large scale eigenvalue problems by parallel block
damping inverse power method" (arXiv 2111.06552), Algorithm 1 with the
techniques of Section 3.  Every step runs in the HIP kernels of libgcge.so;
this module only marshals arguments (torch tensors provide device memory and
the stream).  There is no CPU fallback: without the built library every call
raises.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (B_CSR, B_DIAG, B_IDENTITY, GCGE_NOT_CONVERGED, GCGE_OK, PREC_FP64, PREC_MIXED,  # noqa: F401
                   GcgeError)

__all__ = [
    "DeviceCsr", "Solver", "solve", "GcgeEig", "eigvals", "spmm", "spmm_f32", "shifted_spmm", "residual", "gram",
    "gemm_update", "cg", "orth", "small_eigh", "p_hat", "pattern_grad", "GcgeError", "library_path", "Amg", "pcg",
]


def library_path() -> str:
    return _lib.LIB_PATH


def _L():
    return _lib.load()


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


def _rowmajor(t, name):
    """(ptr, ld) of a 2-D row-major view (stride(1) == 1)."""
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1) or t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        raise ValueError(f"{name} must be a 2-D row-major block")
    return ctypes.c_void_p(t.data_ptr()), max(t.stride(0), t.shape[1], 1)


class DeviceCsr:
    """CSR matrix on the device: int32 rowptr/colind and float64 values (torch tensors)."""

    def __init__(self, rowptr: torch.Tensor, colind: torch.Tensor, val: torch.Tensor, n: int | None = None):
        _check_dev(rowptr, torch.int32, "rowptr")
        _check_dev(colind, torch.int32, "colind")
        _check_dev(val, torch.float64, "val")
        self.rowptr, self.colind, self.val = rowptr.contiguous(), colind.contiguous(), val.contiguous()
        self.n = int(rowptr.numel() - 1) if n is None else int(n)
        self.nnz = int(colind.numel())

    @classmethod
    def from_host(cls, rowptr, colind, val, device="cuda"):
        return cls(torch.as_tensor(np.asarray(rowptr, dtype=np.int32), device=device),
                   torch.as_tensor(np.asarray(colind, dtype=np.int32), device=device),
                   torch.as_tensor(np.asarray(val, dtype=np.float64), device=device))

    @classmethod
    def from_csr(cls, A, device="cuda"):
        """From any object with rowptr, colind, val arrays (e.g. workloads.Csr)."""
        return cls.from_host(A.rowptr, A.colind, A.val, device)

    def c(self, val: torch.Tensor | None = None) -> _lib.Csr:
        v = self.val if val is None else val
        return _lib.Csr(self.n, self.nnz, self.rowptr.data_ptr(), self.colind.data_ptr(), v.data_ptr())


def _b_args(B):
    """(kind, pointer, keepalive) for B = None | diagonal tensor | DeviceCsr."""
    if B is None:
        return B_IDENTITY, None, None
    if isinstance(B, DeviceCsr):
        c = B.c()
        return B_CSR, ctypes.cast(ctypes.pointer(c), ctypes.c_void_p), c
    _check_dev(B, torch.float64, "B (diagonal)")
    return B_DIAG, ctypes.c_void_p(B.data_ptr()), None


_INT_OPTS = {"block_size", "size_x", "max_iter", "cg_max_iter", "precision", "moving", "shift", "seed", "check",
             "dense_eig", "orth", "orth_block", "orth_skip_final", "precond", "amg_levels", "amg_coarse",
             "profile", "cg_history"}
_DBL_OPTS = {"tol", "cg_rel_tol", "orth_tol", "drop_tol", "amg_strength"}


class Solver:
    """A solver handle for one pencil (A, B) on the current device.

    ``B`` is None (identity), a float64 CUDA vector (diagonal B) or a
    :class:`DeviceCsr`.  Options are those of ``gcge_set_option_*``;
    ``precision`` accepts "fp64" or "mixed".  A, B must stay alive while the
    solver exists (they are borrowed, as in the C ABI)."""

    def __init__(self, A: DeviceCsr, B=None, nev: int = 1, tol: float = 1e-8, **options):
        self.A, self.B = A, B
        self.nev, self.n = int(nev), A.n
        self._h = ctypes.c_void_p()
        kind, bp, self._bkeep = _b_args(B)
        self.b_kind = kind
        self._ac = A.c()
        _lib.check(_L().gcge_create(ctypes.byref(self._ac), kind, bp, self.nev, float(tol), ctypes.byref(self._h)))
        self.set_options(**options)
        self.last_stats = None
        self.last_evecs = None
        self._x0 = None
        # raised by every solve() and update_values(): a gradient belongs to the
        # solve it was taken from (GcgeEig checks it in backward)
        self.generation = 0

    def set_options(self, **options):
        for k, v in options.items():
            if k == "precision" and isinstance(v, str):
                v = {"fp64": PREC_FP64, "mixed": PREC_MIXED}[v]
            if isinstance(v, bool):
                v = int(v)
            if k in _INT_OPTS:
                _lib.check(_L().gcge_set_option_i(self._h, k.encode(), int(v)), self._h)
            elif k in _DBL_OPTS:
                _lib.check(_L().gcge_set_option_d(self._h, k.encode(), float(v)), self._h)
            else:
                raise KeyError(f"unknown option {k}")

    def set_initial_vectors(self, X0: torch.Tensor | None):
        if X0 is None:
            self._x0 = None
            _lib.check(_L().gcge_set_initial_vectors(self._h, None, 0, 0), self._h)
            return
        _check_dev(X0, torch.float64, "X0")
        p, ld = _rowmajor(X0, "X0")
        self._x0 = X0
        _lib.check(_L().gcge_set_initial_vectors(self._h, p, ld, X0.shape[1]), self._h)

    def solve(self, evecs: torch.Tensor | None = None, raise_not_converged: bool = True):
        """Returns (evals: CPU float64 [nev], evecs: CUDA float64 [n, nev], stats dict)."""
        L = _L()
        if evecs is None:
            evecs = torch.empty((self.n, self.nev), dtype=torch.float64, device=self.A.val.device)
        _check_dev(evecs, torch.float64, "evecs")
        p, ld = _rowmajor(evecs, "evecs")
        evals = np.zeros(self.nev, dtype=np.float64)
        st = _lib.Stats()
        _lib.check(L.gcge_set_stream(self._h, ctypes.c_void_p(_stream(evecs.device))), self._h)
        self.generation += 1
        rc = _lib.check(L.gcge_solve(self._h, evals.ctypes.data_as(ctypes.c_void_p), p, ld, ctypes.byref(st)),
                        self._h)
        self.last_stats = st.as_dict()
        self.last_stats["status"] = rc
        self.last_evecs = evecs
        if rc == GCGE_NOT_CONVERGED and raise_not_converged:
            raise GcgeError(rc, "not converged within max_iter")
        return torch.from_numpy(evals), evecs, self.last_stats

    def update_values(self, a_val: torch.Tensor | None, b_val: torch.Tensor | None = None):
        if a_val is not None:
            _check_dev(a_val, torch.float64, "a_val")
            a_val = a_val.contiguous()
        if b_val is not None:
            _check_dev(b_val, torch.float64, "b_val")
            b_val = b_val.contiguous()
        _lib.check(_L().gcge_set_stream(self._h, ctypes.c_void_p(_stream())), self._h)
        self.generation += 1
        _lib.check(_L().gcge_update_values(self._h, _p(a_val), _p(b_val)), self._h)
        self._keep = (a_val, b_val)

    def eig_grad(self, g):
        """Gradients of sum_i g_i lambda_i w.r.t. the stored nonzeros of A and of B."""
        g = np.ascontiguousarray(np.asarray(g.detach().cpu() if isinstance(g, torch.Tensor) else g,
                                            dtype=np.float64))
        dev = self.A.val.device
        gA = torch.empty(self.A.nnz, dtype=torch.float64, device=dev)
        gB = None
        if self.b_kind == B_CSR:
            gB = torch.empty(self.B.nnz, dtype=torch.float64, device=dev)
        elif self.b_kind == B_DIAG:
            gB = torch.empty(self.n, dtype=torch.float64, device=dev)
        _lib.check(_L().gcge_set_stream(self._h, ctypes.c_void_p(_stream(dev))), self._h)
        rc = _lib.check(_L().gcge_eig_grad(self._h, g.ctypes.data_as(ctypes.c_void_p), _p(gA), _p(gB)), self._h)
        if rc == GCGE_NOT_CONVERGED:
            raise GcgeError(rc, "the last solve did not converge: no gradient of unconverged pairs")
        return gA, gB

    def close(self):
        if self._h:
            _L().gcge_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def solve(A: DeviceCsr, B=None, nev: int = 1, tol: float = 1e-8, **options):
    """One-shot solve; returns (evals, evecs, stats)."""
    with Solver(A, B, nev, tol, **options) as s:
        return s.solve()


class GcgeEig(torch.autograd.Function):
    """Eigenvalues of (A, B) as a differentiable function of the stored values of
    A (and of B): backward applies d lambda_i / d a_jk = x_i[j] x_i[k] and
    d lambda_i / d b_jk = -lambda_i x_i[j] x_i[k] (B-normalized x_i, simple
    eigenvalues) in the sparsity-pattern kernel of libgcge.so."""

    @staticmethod
    def forward(ctx, a_val, b_val, solver: Solver):
        solver.update_values(a_val.detach(), None if b_val is None else b_val.detach())
        evals, evecs, _ = solver.solve()
        ctx.solver = solver
        ctx.generation = solver.generation
        ctx.has_b = b_val is not None
        return evals.to(a_val.device)

    @staticmethod
    def backward(ctx, g):
        # the kernel reads the solver's last eigenvectors: they must be this forward's
        if ctx.solver.generation != ctx.generation:
            raise RuntimeError("the solver ran another solve or update_values between this forward and its "
                               "backward; its eigenvectors no longer belong to this graph (use one solver "
                               "per differentiated solve, or call backward first)")
        gA, gB = ctx.solver.eig_grad(g)
        return gA, (gB if ctx.has_b else None), None


def eigvals(a_val: torch.Tensor, solver: Solver, b_val: torch.Tensor | None = None) -> torch.Tensor:
    """Differentiable eigenvalues lambda(a_val[, b_val]) for the pattern of ``solver``."""
    return GcgeEig.apply(a_val, b_val, solver)


# ----------------------------------------------------------------- step entries

def spmm(A: DeviceCsr, X: torch.Tensor, Y: torch.Tensor | None = None) -> torch.Tensor:
    _check_dev(X, torch.float64, "X")
    if Y is None:
        Y = torch.empty((A.n, X.shape[1]), dtype=torch.float64, device=X.device)
    px, ldx = _rowmajor(X, "X")
    py, ldy = _rowmajor(Y, "Y")
    c = A.c()
    _lib.check(_L().gcge_spmm(ctypes.byref(c), px, ldx, X.shape[1], py, ldy, ctypes.c_void_p(_stream(X.device))))
    return Y


def spmm_f32(A: DeviceCsr, val32: torch.Tensor, X: torch.Tensor, Y: torch.Tensor | None = None) -> torch.Tensor:
    _check_dev(val32, torch.float32, "val32")
    _check_dev(X, torch.float32, "X")
    if Y is None:
        Y = torch.empty((A.n, X.shape[1]), dtype=torch.float32, device=X.device)
    px, ldx = _rowmajor(X, "X")
    py, ldy = _rowmajor(Y, "Y")
    _lib.check(_L().gcge_spmm_f32(A.n, _p(A.rowptr), _p(A.colind), _p(val32), px, ldx, X.shape[1], py, ldy,
                                  ctypes.c_void_p(_stream(X.device))))
    return Y


def shifted_spmm(A: DeviceCsr, B, X: torch.Tensor, sigma) -> torch.Tensor:
    _check_dev(X, torch.float64, "X")
    k = X.shape[1]
    sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (k,)))
    Y = torch.empty((A.n, k), dtype=torch.float64, device=X.device)
    kind, bp, keep = _b_args(B)
    px, ldx = _rowmajor(X, "X")
    py, ldy = _rowmajor(Y, "Y")
    c = A.c()
    _lib.check(_L().gcge_shifted_spmm(ctypes.byref(c), kind, bp, sig.ctypes.data_as(ctypes.c_void_p), px, ldx, k,
                                      py, ldy, ctypes.c_void_p(_stream(X.device))))
    return Y


def residual(A: DeviceCsr, B, X: torch.Tensor, lam):
    """STEP 4: (R, ||r_j||, ||B x_j||)."""
    _check_dev(X, torch.float64, "X")
    k = X.shape[1]
    lam = np.ascontiguousarray(np.asarray(lam, dtype=np.float64).reshape(k))
    R = torch.empty((A.n, k), dtype=torch.float64, device=X.device)
    rn = np.zeros(k)
    bn = np.zeros(k)
    kind, bp, keep = _b_args(B)
    px, ldx = _rowmajor(X, "X")
    pr, ldr = _rowmajor(R, "R")
    c = A.c()
    _lib.check(_L().gcge_residual(ctypes.byref(c), kind, bp, lam.ctypes.data_as(ctypes.c_void_p), px, ldx, k, pr,
                                  ldr, rn.ctypes.data_as(ctypes.c_void_p), bn.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.c_void_p(_stream(X.device))))
    return R, rn, bn


def gram(X: torch.Tensor, Y: torch.Tensor, d: torch.Tensor | None = None) -> np.ndarray:
    """X^T diag(d) Y as a host float64 array."""
    _check_dev(X, torch.float64, "X")
    _check_dev(Y, torch.float64, "Y")
    if d is not None:
        _check_dev(d, torch.float64, "d")
    m, k = X.shape[1], Y.shape[1]
    C = np.zeros((m, k))
    px, ldx = _rowmajor(X, "X")
    py, ldy = _rowmajor(Y, "Y")
    _lib.check(_L().gcge_gram(X.shape[0], px, ldx, m, py, ldy, k, _p(d), C.ctypes.data_as(ctypes.c_void_p),
                              ctypes.c_void_p(_stream(X.device))))
    return C


def gram_noalloc(X: torch.Tensor, Y: torch.Tensor, d: torch.Tensor | None = None,
                 C: torch.Tensor | None = None) -> torch.Tensor:
    """X^T diag(d) Y into the device tensor C (m x k float64, contiguous), through the
    entry point that allocates nothing (partials in the library's fixed device array)."""
    _check_dev(X, torch.float64, "X")
    _check_dev(Y, torch.float64, "Y")
    if d is not None:
        _check_dev(d, torch.float64, "d")
    m, k = X.shape[1], Y.shape[1]
    if C is None:
        C = torch.empty((m, k), dtype=torch.float64, device=X.device)
    _check_dev(C, torch.float64, "C")
    if tuple(C.shape) != (m, k) or not C.is_contiguous():
        raise ValueError("C must be a contiguous m x k tensor")
    px, ldx = _rowmajor(X, "X")
    py, ldy = _rowmajor(Y, "Y")
    _lib.check(_L().gcge_gram_noalloc(X.shape[0], px, ldx, m, py, ldy, k, _p(d), _p(C),
                                      ctypes.c_void_p(_stream(X.device))))
    return C


def gemm_update(X: torch.Tensor, S, Y: torch.Tensor | None = None, alpha: float = 1.0, beta: float = 0.0):
    """Y = alpha X S + beta Y with S a host (m x k) array."""
    _check_dev(X, torch.float64, "X")
    S = np.ascontiguousarray(np.asarray(S, dtype=np.float64))
    m, k = S.shape
    if Y is None:
        Y = torch.zeros((X.shape[0], k), dtype=torch.float64, device=X.device)
    px, ldx = _rowmajor(X, "X")
    py, ldy = _rowmajor(Y, "Y")
    _lib.check(_L().gcge_gemm_update(X.shape[0], px, ldx, m, S.ctypes.data_as(ctypes.c_void_p), k, float(alpha),
                                     float(beta), py, ldy, ctypes.c_void_p(_stream(X.device))))
    return Y


def cg(A: DeviceCsr, B, theta: float, R: torch.Tensor, maxit: int = 30, rel_tol: float = 1e-2,
       precision: str = "fp64"):
    """STEP 6: (delta, iterations per column)."""
    _check_dev(R, torch.float64, "R")
    k = R.shape[1]
    D = torch.empty_like(R)
    its = np.zeros(k, dtype=np.int32)
    kind, bp, keep = _b_args(B)
    pr, ldr = _rowmajor(R, "R")
    pd, ldd = _rowmajor(D, "delta")
    c = A.c()
    prec = {"fp64": PREC_FP64, "mixed": PREC_MIXED}[precision]
    _lib.check(_L().gcge_cg(ctypes.byref(c), kind, bp, float(theta), pr, ldr, k, int(maxit), float(rel_tol), prec,
                            pd, ldd, its.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(_stream(R.device))))
    return D, its


class Amg:
    """Algebraic multigrid preconditioner of the STEP 6 systems (gcge_amg_*).

    Keeps a reference to A: its device arrays are the level-0 operator."""

    def __init__(self, A: DeviceCsr, max_levels: int = 10, coarse_max: int = 512, strength: float = 0.02):
        self._A = A
        self._c = A.c()
        h = ctypes.c_void_p()
        _lib.check(_L().gcge_amg_create(ctypes.byref(self._c), int(max_levels), int(coarse_max), float(strength),
                                        ctypes.c_void_p(_stream(A.rowptr.device)), ctypes.byref(h)))
        self._h = h

    def levels(self):
        """[(rows, stored entries)] per level; the last level is the dense coarsest one."""
        cap = 16
        rows = np.zeros(cap, dtype=np.int64)
        nnz = np.zeros(cap, dtype=np.int64)
        nl = ctypes.c_int(0)
        _lib.check(_L().gcge_amg_levels(self._h, ctypes.byref(nl), rows.ctypes.data_as(ctypes.c_void_p),
                                        nnz.ctypes.data_as(ctypes.c_void_p), cap))
        return [(int(rows[i]), int(nnz[i])) for i in range(nl.value)]

    def aggregates(self, level: int) -> np.ndarray:
        rows = self.levels()[level][0]
        agg = np.zeros(rows, dtype=np.int32)
        _lib.check(_L().gcge_amg_aggregates(self._h, int(level), agg.ctypes.data_as(ctypes.c_void_p)))
        return agg

    def apply(self, Bm: torch.Tensor, Y: torch.Tensor | None = None) -> torch.Tensor:
        """Y = V(B), one V-cycle on the columns of B (n x k, k <= 128)."""
        _check_dev(Bm, torch.float64, "B")
        if Y is None:
            Y = torch.empty_like(Bm)
        pb, ldb = _rowmajor(Bm, "B")
        py, ldy = _rowmajor(Y, "Y")
        _lib.check(_L().gcge_amg_apply(self._h, pb, ldb, Bm.shape[1], py, ldy, ctypes.c_void_p(_stream(Bm.device))))
        return Y

    def close(self):
        if self._h is not None and self._h.value:
            _L().gcge_amg_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def pcg(A: DeviceCsr, M: Amg, R: torch.Tensor, maxit: int = 30, rel_tol: float = 1e-2):
    """STEP 6 preconditioned by the V-cycle of M (theta = 0): (delta, iterations per column)."""
    _check_dev(R, torch.float64, "R")
    k = R.shape[1]
    D = torch.empty_like(R)
    its = np.zeros(k, dtype=np.int32)
    pr, ldr = _rowmajor(R, "R")
    pd, ldd = _rowmajor(D, "delta")
    c = A.c()
    _lib.check(_L().gcge_pcg(ctypes.byref(c), M._h, pr, ldr, k, int(maxit), float(rel_tol), pd, ldd,
                             its.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(_stream(R.device))))
    return D, its


def orth(W: torch.Tensor, Q: torch.Tensor | None = None, B=None, algorithm: int = 3, block: int = 0):
    """STEP 2: W B-orthogonalized against Q then by Algorithm 3 (or Algorithm 2
    with blocks of `block` columns); returns W[:, :kept]."""
    _check_dev(W, torch.float64, "W")
    kept = ctypes.c_int(0)
    kind, bp, keep = _b_args(B)
    pw, ldw = _rowmajor(W, "W")
    if Q is not None:
        _check_dev(Q, torch.float64, "Q")
        pq, ldq = _rowmajor(Q, "Q")
        mq = Q.shape[1]
    else:
        pq, ldq, mq = None, 0, 0
    if algorithm == 3:
        _lib.check(_L().gcge_orth(W.shape[0], kind, bp, pq, ldq, mq, pw, ldw, W.shape[1], ctypes.byref(kept),
                                  ctypes.c_void_p(_stream(W.device))))
    elif algorithm == 2:
        _lib.check(_L().gcge_orth_mbo(W.shape[0], kind, bp, pq, ldq, mq, pw, ldw, W.shape[1], int(block),
                                      ctypes.byref(kept), ctypes.c_void_p(_stream(W.device))))
    else:
        raise ValueError("algorithm must be 2 or 3")
    return W[:, :kept.value]


def small_eigh(M, nwant: int | None = None):
    """Host dense symmetric eigensolver of the library: (w ascending, Z[:, :nwant])."""
    a = np.array(M, dtype=np.float64, order="C", copy=True)
    n = a.shape[0]
    nwant = n if nwant is None else int(nwant)
    w = np.zeros(n)
    z = np.zeros((n, nwant))
    _lib.check(_L().gcge_small_eigh(n, a.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p),
                                    z.ctypes.data_as(ctypes.c_void_p) if nwant else None, nwant))
    return w, z


def dense_eig(M: torch.Tensor, nwant: int | None = None):
    """Device dense symmetric eigensolver: (w [nwant] ascending, X [n, nwant]), both on M's device."""
    _check_dev(M, torch.float64, "M")
    n = M.shape[0]
    if M.dim() != 2 or M.shape[1] != n:
        raise ValueError("M must be square")
    nwant = n if nwant is None else int(nwant)
    pm, ldm = _rowmajor(M, "M")
    w = torch.empty(nwant, dtype=torch.float64, device=M.device)
    X = torch.empty((n, nwant), dtype=torch.float64, device=M.device)
    px, ldx = _rowmajor(X, "X")
    _lib.check(_L().gcge_dense_eig(n, pm, ldm, nwant, _p(w), px, ldx, ctypes.c_void_p(_stream(M.device))))
    return w, X


def p_hat(xhat, shift: int, n_old: int, n_new: int, drop_tol: float = 1e-10):
    xh = np.ascontiguousarray(np.asarray(xhat, dtype=np.float64))
    dim, nx = xh.shape
    ph = np.zeros((dim, n_new))
    npc = ctypes.c_int(0)
    _lib.check(_L().gcge_p_hat(dim, nx, xh.ctypes.data_as(ctypes.c_void_p), shift, n_old, n_new, float(drop_tol),
                               ph.ctypes.data_as(ctypes.c_void_p), ctypes.byref(npc)))
    return ph[:, :npc.value]


def pattern_grad(A: DeviceCsr, X: torch.Tensor, wts) -> torch.Tensor:
    _check_dev(X, torch.float64, "X")
    w = np.ascontiguousarray(np.asarray(wts, dtype=np.float64))
    g = torch.empty(A.nnz, dtype=torch.float64, device=X.device)
    px, ldx = _rowmajor(X, "X")
    _lib.check(_L().gcge_pattern_grad(A.n, A.nnz, _p(A.rowptr), _p(A.colind), px, ldx, X.shape[1],
                                      w.ctypes.data_as(ctypes.c_void_p), _p(g), ctypes.c_void_p(_stream(X.device))))
    return g
