"""Pins of the block Lanczos reference eigensolver (oracle/lanczos.py) against
closed-form spectra with their multiplicities, the dense Jacobi oracle (itself
pinned) and invariants; its sparse kernels against dense products and
numpy.linalg.solve.  (No GPU.)"""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from oracle import lanczos as lz
from closed_forms import lap2d_eigs, lap3d_eigs, q1_eigs


def _invariants(A, bkind, B, lam, X, tol):
    BX = orc.apply_b(bkind, B, X)
    assert np.max(np.abs(X.T @ BX - np.eye(X.shape[1]))) < 1e-11
    rel = orc.relative_residuals(A, bkind, B, X, lam)
    assert rel.max() <= tol
    assert np.all(np.diff(lam) >= -1e-12 * np.abs(lam[1:]))


def test_csr_spmm_matches_dense_product():
    rng = np.random.default_rng(1)
    A = wl.varcoef3d_7pt(5)
    X = rng.standard_normal((A.n, 7))
    assert np.max(np.abs(lz.csr_spmm(A, X) - A.to_dense() @ X)) < 1e-12 * np.abs(A.val).max()
    assert np.max(np.abs(lz.csr_spmm(A, X[:, 0]) - A.to_dense() @ X[:, 0])) < 1e-12 * np.abs(A.val).max()


def test_csr_cg_solves_spd_systems():
    rng = np.random.default_rng(2)
    A = wl.laplace3d_7pt(6)
    Bm = rng.standard_normal((A.n, 5))
    Bm[:, 3] = 0.0                               # a zero right-hand side stays zero
    X, its = lz.csr_cg(A, Bm, 1e-14, 5000)
    ref = np.linalg.solve(A.to_dense(), Bm)
    assert np.max(np.abs(X - ref)) < 1e-11 * np.abs(ref).max()
    assert its[3] == 0 and np.all(X[:, 3] == 0.0)
    assert np.all(its[[0, 1, 2, 4]] > 0)


def test_csr_cg_detects_an_indefinite_matrix():
    A = wl.laplace2d_5pt(6)
    A = A.with_values(A.val - 100.0 * (A.row_of_entry() == A.colind))   # shifted past lambda_1 = 19.4
    with pytest.raises(np.linalg.LinAlgError):
        lz.csr_cg(A, np.ones((A.n, 1)), 1e-12, 1000)


def test_lanczos_2d_laplacian_closed_form():
    A = wl.laplace2d_5pt(30)
    lam, X, info = lz.lanczos_eigs(A, "identity", None, 16)
    ref = lap2d_eigs(30)[:16]                    # pairs (i, j), (j, i): multiplicity 2
    assert np.max(np.abs(lam - ref) / ref) < 1e-12
    _invariants(A, "identity", None, lam, X, 1e-12)
    assert info["max_rel_residual"] <= info["max_gate"]


def test_lanczos_3d_laplacian_closed_form_with_multiplicities():
    # lambda_2..4 triple, a sixfold cluster among the first 30: a single-vector
    # Krylov space cannot hold the copies, the block of 8 must
    A = wl.laplace3d_7pt(10)
    nev = 30
    lam, X, _ = lz.lanczos_eigs(A, "identity", None, nev)
    ref = lap3d_eigs(10)[:nev]
    assert np.max(np.abs(lam - ref) / ref) < 1e-12
    _invariants(A, "identity", None, lam, X, 1e-12)
    # every copy of a multiple eigenvalue is a distinct direction
    ev = np.sort(lap3d_eigs(10))
    for v in np.unique(np.round(ref, 8)):
        mult = int(np.sum(np.abs(ev - v) < 1e-8 * v))
        got = int(np.sum(np.abs(lam - v) < 1e-8 * v))
        if np.sum(np.abs(ref - v) < 1e-8 * v) == mult:   # cluster not cut by nev
            assert got == mult


def test_lanczos_diagonal_b_matches_dense_oracle():
    A = wl.laplace3d_7pt(9)
    d = wl.diag_uniform(A.n)
    nev = 24
    lam, X, _ = lz.lanczos_eigs(A, "diag", d, nev, seed=3)
    ref, Xr = orc.pencil_eigs(A, "diag", d, nev)
    assert np.max(np.abs(lam - ref) / ref) < 1e-11
    _invariants(A, "diag", d, lam, X, 1e-12)
    # random B splits the clusters: each eigenvector matches up to sign
    c = np.abs(np.sum(X * (d[:, None] * Xr), axis=0))
    assert np.min(c) > 1 - 1e-9


def test_lanczos_csr_b_q1_closed_form():
    A, B = wl.q1_fem(7, constant=True)
    nev = 20
    lam, X, _ = lz.lanczos_eigs(A, "csr", B, nev)
    ref = q1_eigs(7)[:nev]
    assert np.max(np.abs(lam - ref) / ref) < 1e-12
    _invariants(A, "csr", B, lam, X, 1e-12)


def test_lanczos_variable_coefficients_match_dense_oracle():
    A = wl.varcoef3d_7pt(7)
    nev = 25
    lam, X, _ = lz.lanczos_eigs(A, "identity", None, nev, seed=7)
    ref, Xr = orc.pencil_eigs(A, "identity", None, nev)
    assert np.max(np.abs(lam - ref) / ref) < 1e-11
    _invariants(A, "identity", None, lam, X, 1e-12)
    assert np.min(np.abs(np.sum(X * Xr, axis=0))) > 1 - 1e-9


def test_lanczos_rejects_bad_nev():
    A = wl.laplace2d_5pt(4)
    with pytest.raises(ValueError):
        lz.lanczos_eigs(A, "identity", None, 0)
    with pytest.raises(ValueError):
        lz.lanczos_eigs(A, "identity", None, A.n + 1)
