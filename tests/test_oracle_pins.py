"""Pins of the CPU oracle against facts fixed by the paper and by mathematics:
closed-form spectra, the one-step formula of Remark rem:shift, the paper's
reduction counts, invariants and brute force on tiny inputs.  None of these
checks re-derives a value with the oracle's own formula.  (No GPU.)"""
import numpy as np
import pytest

import oracle as orc
import workloads as wl

RNG = np.random.default_rng(12345)


# ---------------------------------------------------------------- closed forms

def lap2d_eigs(m):
    """(4/h^2)(sin^2(i pi h/2) + sin^2(j pi h/2)), h = 1/(m+1)."""
    h = 1.0 / (m + 1)
    s = np.sin(np.arange(1, m + 1) * np.pi * h / 2) ** 2
    return np.sort((4.0 / h ** 2 * (s[:, None] + s[None, :])).ravel())


def lap3d_eigs(n):
    h = 1.0 / (n + 1)
    s = np.sin(np.arange(1, n + 1) * np.pi * h / 2) ** 2
    return np.sort((4.0 / h ** 2 * (s[:, None, None] + s[None, :, None] + s[None, None, :])).ravel())


def q1_eigs(n):
    """(6/h^2) sum_d (1 - cos(i_d pi h)) / (2 + cos(i_d pi h)), h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    c = np.cos(np.arange(1, n + 1) * np.pi * h)
    t = 6.0 / h ** 2 * (1 - c) / (2 + c)
    return np.sort((t[:, None, None] + t[None, :, None] + t[None, None, :]).ravel())


def test_closed_form_values_quoted_for_the_64x64_grid():
    # The first eigenvalues of the 64x64 grid, checked against the closed form
    # as written above (values computed independently of the oracle).
    ev = lap2d_eigs(64)
    assert abs(ev[0] - 19.73536653368066) < 1e-9
    assert abs(ev[1] - 49.31536990270943) < 1e-9 and abs(ev[2] - ev[1]) < 1e-9
    assert abs(ev[10] - 177.3418492772364) < 1e-9


# ---------------------------------------------------------------- jacobi_eigh

def test_jacobi_1d_laplacian_closed_form():
    n = 50
    T = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    w, V = orc.jacobi_eigh(T)
    exact = 4 * np.sin(np.arange(1, n + 1) * np.pi / (2 * (n + 1))) ** 2
    assert np.max(np.abs(w - exact)) < 1e-13


def test_jacobi_2d_laplacian_closed_form():
    A = wl.laplace2d_5pt(10)
    w, V = orc.jacobi_eigh(A.to_dense())
    ex = lap2d_eigs(10)
    assert np.max(np.abs(w - ex) / ex) < 1e-13


def test_jacobi_exact_small_cases():
    w, V = orc.jacobi_eigh(np.diag([3.0, -1.0, 2.0]))
    assert np.array_equal(w, [-1.0, 2.0, 3.0])
    w, V = orc.jacobi_eigh(np.array([[2.0, 1.0], [1.0, 2.0]]))
    assert np.allclose(w, [1.0, 3.0], atol=1e-15)
    assert abs(abs(V[0, 0]) - np.sqrt(0.5)) < 1e-15
    w, V = orc.jacobi_eigh(np.array([[5.0]]))
    assert w[0] == 5.0 and V[0, 0] == 1.0


@pytest.mark.parametrize("n", [7, 64, 200])
def test_jacobi_invariants(n):
    M = RNG.standard_normal((n, n))
    M = M + M.T
    w, V = orc.jacobi_eigh(M)
    assert np.max(np.abs(V.T @ V - np.eye(n))) < 1e-13
    assert np.max(np.abs(M @ V - V * w)) < 1e-12 * np.abs(M).max() * n ** 0.5
    assert np.all(np.diff(w) >= 0)


def test_jacobi_repeated_eigenvalues():
    Q, _ = np.linalg.qr(RNG.standard_normal((6, 6)))
    d = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 3.0])
    w, V = orc.jacobi_eigh(Q @ np.diag(d) @ Q.T)
    assert np.max(np.abs(w - d)) < 1e-14


def test_jacobi_brute_force_against_lapack():
    # test-only cross-check against a LAPACK-backed routine (never used inside the oracle)
    M = RNG.standard_normal((120, 120))
    M = M + M.T
    w, _ = orc.jacobi_eigh(M)
    assert np.max(np.abs(w - np.linalg.eigvalsh(M))) < 1e-12 * np.abs(w).max()


# ---------------------------------------------------------------- cholesky

def test_cholesky_recovers_constructed_factor():
    n = 30
    L0 = np.tril(RNG.standard_normal((n, n)))
    L0[np.arange(n), np.arange(n)] = np.abs(L0[np.arange(n), np.arange(n)]) + 1.0
    L = orc.cholesky(L0 @ L0.T)
    assert np.max(np.abs(L - L0)) < 1e-12
    with pytest.raises(np.linalg.LinAlgError):
        orc.cholesky(np.diag([1.0, -1.0]))
    X = RNG.standard_normal((n, 3))
    assert np.allclose(L0 @ orc.solve_lower(L0, X), X, atol=1e-12)
    assert np.allclose(L0.T @ orc.solve_lower_t(L0, X), X, atol=1e-12)


# ---------------------------------------------------------------- pencil_eigs

def test_pencil_q1_fem_closed_form():
    n = 5
    A, B = wl.q1_fem(n, constant=True)
    lam, X = orc.pencil_eigs(A, "csr", B, 40)
    ex = q1_eigs(n)[:40]
    assert np.max(np.abs(lam - ex) / ex) < 1e-12
    assert np.max(np.abs(X.T @ orc.apply_b("csr", B, X) - np.eye(40))) < 1e-12


def test_pencil_lap3d_closed_form_and_diag_sandwich():
    n = 6
    A = wl.laplace3d_7pt(n)
    lam, X = orc.pencil_eigs(A, "identity", None, 30)
    ex = lap3d_eigs(n)[:30]
    assert np.max(np.abs(lam - ex) / ex) < 1e-12
    d = wl.diag_uniform(A.n)
    lamd, Xd = orc.pencil_eigs(A, "diag", d, 30)
    # Courant-Fischer: D in [0.5, 1.5] gives lambda_k(A)/1.5 <= lambda_k(A, D) <= lambda_k(A)/0.5
    assert np.all(lamd >= ex / 1.5 - 1e-9) and np.all(lamd <= ex / 0.5 + 1e-9)
    rel = orc.relative_residuals(A, "diag", d, Xd, lamd)
    assert rel.max() < 1e-12
    assert np.max(np.abs(Xd.T @ (d[:, None] * Xd) - np.eye(30))) < 1e-12


def test_pencil_config1_closed_form_small_grid():
    A = wl.laplace2d_5pt(16)
    lam, X = orc.pencil_eigs(A, "identity", None, 10)
    assert np.max(np.abs(lam - lap2d_eigs(16)[:10]) / lam) < 1e-12


def test_pencil_q1_random_kappa_sandwich():
    n = 4
    A, B = wl.q1_fem(n)
    A1, _ = wl.q1_fem(n, constant=True)
    lam, X = orc.pencil_eigs(A, "csr", B, 20)
    ex = q1_eigs(n)[:20]
    assert np.all(lam >= 0.1 * ex - 1e-9) and np.all(lam <= 10 * ex + 1e-9)
    assert orc.relative_residuals(A, "csr", B, X, lam).max() < 1e-11


def test_pencil_varcoef_sandwich():
    n = 5
    A = wl.varcoef3d_7pt(n)
    lam, _ = orc.pencil_eigs(A, "identity", None, 20)
    ex = lap3d_eigs(n)[:20]
    assert np.all(lam >= 0.5 * ex - 1e-9) and np.all(lam <= 2.0 * ex + 1e-9)


# ---------------------------------------------------------------- spmm / gram / residual

def _random_csr(n, density, empty_rows=()):
    D = np.where(RNG.random((n, n)) < density, RNG.standard_normal((n, n)), 0.0)
    for r in empty_rows:
        D[r, :] = 0.0
    rows, cols = np.nonzero(D)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return wl.Csr(n, rowptr, cols.astype(np.int32), D[rows, cols]), D


def test_spmm_against_dense():
    A, D = _random_csr(40, 0.2, empty_rows=(0, 17, 39))
    X = RNG.standard_normal((40, 5))
    assert np.max(np.abs(orc.spmm(A, X) - D @ X)) < 1e-13
    assert np.max(np.abs(orc.spmm_rows(A, X, [3, 17, 39]) - (D @ X)[[3, 17, 39]])) < 1e-13


def test_spmm_laplacian_on_closed_form_eigenvectors():
    m = 12
    A = wl.laplace2d_5pt(m)
    h = 1.0 / (m + 1)
    x = np.arange(1, m + 1) * h
    i, j = 2, 5
    v = (np.sin(i * np.pi * x)[None, :] * np.sin(j * np.pi * x)[:, None]).ravel()  # x fastest
    lam = 4 / h ** 2 * (np.sin(i * np.pi * h / 2) ** 2 + np.sin(j * np.pi * h / 2) ** 2)
    assert np.max(np.abs(orc.spmm(A, v) - lam * v)) < 1e-9 * lam


def test_gram_and_residual():
    X = RNG.standard_normal((30, 4))
    Y = RNG.standard_normal((30, 3))
    d = RNG.random(30) + 0.5
    assert np.allclose(orc.gram(X, Y, d), X.T @ np.diag(d) @ Y, atol=1e-13)
    A = wl.laplace2d_5pt(6)
    lam = lap2d_eigs(6)[:3]
    _, V = orc.jacobi_eigh(A.to_dense())
    R, rn, bn = orc.residual(A, "identity", None, V[:, :3], lam)
    assert rn.max() < 1e-11 and np.allclose(bn, 1.0)


def test_converged_prefix():
    assert orc.converged_prefix([1e-9, 1e-10, 1e-3, 1e-12], 1e-8) == 2
    assert orc.converged_prefix([1e-3, 1e-10], 1e-8) == 0


# ---------------------------------------------------------------- CG (STEP 6)

def test_cg_remark_shift_one_step_closed_form():
    # Remark rem:shift: standard problem, lambda_1 found, x0 = a2 v2 + a3 v3,
    # one CG step on (A - theta I) w = (lambda~ - theta) x0 from x0.
    n = 8
    lam = np.array([1.0, 2.0, 3.5, 4.0, 6.0, 7.0, 9.0, 11.0])
    Q, _ = np.linalg.qr(RNG.standard_normal((n, n)))
    A = Q @ np.diag(lam) @ Q.T
    rows, cols = np.nonzero(np.ones((n, n)))
    Acsr = wl.Csr(n, np.arange(0, n * n + 1, n, dtype=np.int32), cols.astype(np.int32), A[rows, cols])
    a2, a3, theta = 0.8, 0.6, 1.0
    v2, v3 = Q[:, 1], Q[:, 2]
    x0 = a2 * v2 + a3 * v3
    lt = x0 @ A @ x0 / (x0 @ x0)
    x1, its = orc.cg_columnwise(Acsr, "identity", None, theta, ((lt - theta) * x0)[:, None],
                                maxit=1, rel_tol=0.0, x0=x0[:, None])
    l2, l3 = lam[1], lam[2]
    coef = (a2 ** 2 + a3 ** 2) / (a3 ** 2 * (l2 - theta) + a2 ** 2 * (l3 - theta))
    exact = coef * ((l3 - theta) * a2 * v2 + (l2 - theta) * a3 * v3)
    assert its[0] == 1
    assert np.max(np.abs(x1[:, 0] - exact)) < 1e-13


def test_cg_terminates_in_n_steps_on_spd():
    n = 12
    M = RNG.standard_normal((n, n))
    S = M @ M.T + n * np.eye(n)
    rows, cols = np.nonzero(np.ones((n, n)))
    Scsr = wl.Csr(n, np.arange(0, n * n + 1, n, dtype=np.int32), cols.astype(np.int32), S[rows, cols])
    b = RNG.standard_normal((n, 2))
    x, its = orc.cg_columnwise(Scsr, "identity", None, 0.0, b, maxit=n, rel_tol=0.0)
    ref = np.linalg.solve(S, b)  # test-only brute force
    assert np.max(np.abs(x - ref)) < 1e-9 * np.abs(ref).max()


def test_cg_correction_form_equals_initial_guess_form():
    # (A - theta B) W = B X (Lam - theta) from W0 = X  versus  (A - theta B) delta = -R from 0,
    # R = A X - B X Lam: the iterates differ exactly by X.
    A = wl.laplace3d_7pt(5)
    d = wl.diag_uniform(A.n)
    X = RNG.standard_normal((A.n, 3))
    lam = np.array([40.0, 70.0, 90.0])
    theta = 25.0
    rhs = (d[:, None] * X) * (lam - theta)[None, :]
    W, its1 = orc.cg_columnwise(A, "diag", d, theta, rhs, maxit=7, rel_tol=0.0, x0=X)
    R, _, _ = orc.residual(A, "diag", d, X, lam)
    delta, its2 = orc.cg_columnwise(A, "diag", d, theta, -R, maxit=7, rel_tol=0.0)
    assert np.array_equal(its1, its2)
    assert np.max(np.abs((W - X) - delta)) < 1e-12 * np.abs(delta).max()


def test_cg_stops_on_relative_tolerance_and_breakdown():
    A = wl.laplace2d_5pt(8)
    b = RNG.standard_normal((A.n, 1))
    x, its = orc.cg_columnwise(A, "identity", None, 0.0, b, maxit=200, rel_tol=1e-2)
    r = b[:, 0] - orc.spmm(A, x[:, 0])
    assert np.linalg.norm(r) <= 1e-2 * np.linalg.norm(b) and its[0] < 200
    # theta above every eigenvalue: p^T (A - theta I) p < 0 at once -> zero iterations
    x, its = orc.cg_columnwise(A, "identity", None, 1e6, b, maxit=30, rel_tol=1e-2)
    assert its[0] == 0 and np.all(x == 0)


# ---------------------------------------------------------------- orthogonalization

def _b_orthonormal(n, k, d):
    Q, _ = np.linalg.qr(RNG.standard_normal((n, k)))  # test-only construction
    return Q / np.sqrt(d)[:, None]


def test_deflate_invariants():
    n = 200
    d = RNG.random(n) + 0.5
    Q = _b_orthonormal(n, 10, d)
    W = RNG.standard_normal((n, 6))
    W[:, 4] = 3.0 * Q[:, 2] - Q[:, 7]        # inside span(Q): dropped
    Wo, passes = orc.deflate(W, Q, "diag", d)
    assert Wo.shape[1] == 5
    assert np.max(np.abs(Q.T @ (d[:, None] * Wo))) < 1e-13
    assert np.max(np.abs(np.sum(Wo * d[:, None] * Wo, axis=0) - 1.0)) < 1e-13
    # each output column is the B-projection of its input column off span(Q), rescaled
    Wk = np.delete(W, 4, axis=1)
    proj = Wk - Q @ (Q.T @ (d[:, None] * Wk))
    cos = np.sum(proj * d[:, None] * Wo, axis=0) / np.sqrt(np.sum(proj * d[:, None] * proj, axis=0))
    assert np.max(np.abs(cos - 1.0)) < 1e-12
    assert 1 <= passes <= 3


@pytest.mark.parametrize("m", [5, 16, 40])
def test_recursive_orth_invariants(m):
    n = 300
    d = RNG.random(n) + 0.5
    W = RNG.standard_normal((n, m))
    Wo, k = orc.recursive_orth_svd(W, "diag", d)
    assert k == m
    assert np.max(np.abs(Wo.T @ (d[:, None] * Wo) - np.eye(m))) < 1e-13
    # span preservation: W = Wo (Wo^T B W)
    assert np.max(np.abs(Wo @ (Wo.T @ (d[:, None] * W)) - W)) < 1e-12 * np.abs(W).max()


@pytest.mark.parametrize("m", [16, 40, 50])
def test_orth_skip_final_option(m):
    """The skip-final option (not the paper's listing): the output meets the
    stopping test itself (B-orthonormal to 1e-13 up to rounding), spans the same
    space, keeps the same columns, and applies fewer updates than Algorithm 3 as
    printed; the deflation keeps W B-orthogonal to Q at the same level."""
    n = 300
    d = RNG.random(n) + 0.5
    W = RNG.standard_normal((n, m))
    W[:, 3] = W[:, 1] - W[:, 0]               # dependent: dropped either way
    c_ref, c_skip = {}, {}
    Wr, kr = orc.recursive_orth_svd(W, "diag", d, counters=c_ref)
    Ws, ks = orc.recursive_orth_svd(W, "diag", d, counters=c_skip, skip_final=True)
    assert ks == kr == m - 1
    assert np.max(np.abs(Ws.T @ (d[:, None] * Ws) - np.eye(ks))) < 2e-13
    # same span: the B-projector onto each output reproduces the other
    assert np.max(np.abs(Wr @ (Wr.T @ (d[:, None] * Ws)) - Ws)) < 1e-12
    assert c_skip["update"] < c_ref["update"]
    assert c_skip["gram"] == c_ref["gram"]
    Q = _b_orthonormal(n, 12, d)
    Wd = RNG.standard_normal((n, 8))
    Dr, pr = orc.deflate(Wd, Q, "diag", d)
    Ds, ps = orc.deflate(Wd, Q, "diag", d, skip_final=True)
    assert ps <= pr and Ds.shape == Dr.shape
    assert np.max(np.abs(Q.T @ (d[:, None] * Ds))) <= 1e-13
    assert np.max(np.abs(Ds - Dr)) < 1e-12


def test_recursive_orth_drops_dependent_columns():
    n = 100
    W = RNG.standard_normal((n, 20))
    W[:, 5] = W[:, 2]                       # duplicate
    W[:, 11] = 0.0                          # zero column
    W[:, 17] = W[:, 0] - 2 * W[:, 9]        # combination across leaves
    Wo, k = orc.recursive_orth_svd(W, "identity", None, c=4)
    assert k == 17
    assert np.max(np.abs(Wo.T @ Wo - np.eye(k))) < 1e-13
    assert np.max(np.abs(Wo @ (Wo.T @ W) - W)) < 1e-11 * np.abs(W).max()


@pytest.mark.parametrize("m", [64, 128, 256])
def test_recursive_orth_reduction_count(m):
    # Section 3.1: with c = 16 and three SVD passes per leaf, Algorithm 3 needs
    # 2^0 + ... + 2^(eta-5) + 3 * 2^(eta-4) = m/4 - 1 global reductions.
    n = 400
    W = RNG.standard_normal((n, m))
    cnt = {}
    orc.recursive_orth_svd(W, "identity", None, c=16, leaf_passes=3, int_passes=1, counters=cnt)
    assert cnt["gram"] == m // 4 - 1


def test_modified_block_orth_invariants_and_count():
    n, m = 300, 32
    d = RNG.random(n) + 0.5
    X0 = _b_orthonormal(n, 8, d)
    X = RNG.standard_normal((n, m))
    Xo, k = orc.modified_block_orth(X, X0, "diag", d, max_pass=3)
    assert k == m
    assert np.max(np.abs(Xo.T @ (d[:, None] * Xo) - np.eye(m))) < 1e-13
    assert np.max(np.abs(X0.T @ (d[:, None] * Xo))) < 1e-13
    # Section 3.1 count m + m/b - 1 (one reduction per column of a block and one
    # deflation pass per later-block update; no X0)
    cnt = {}
    b = 8
    orc.modified_block_orth(X, None, "identity", None, b=b, max_pass=1, counters=cnt)
    assert cnt["gram"] == m + m // b - 1


# ---------------------------------------------------------------- STEP 3 / STEP 5

def test_p_hat_orthonormal_and_complete_basis_gives_empty():
    dim, nx = 30, 20
    Q, _ = np.linalg.qr(RNG.standard_normal((dim, dim)))
    xhat = Q[:, :nx]
    ph = orc.p_hat(xhat, 2, 5, 5)
    assert ph.shape[1] == 5
    XP = np.hstack([xhat, ph])
    assert np.max(np.abs(XP.T @ XP - np.eye(nx + 5))) < 1e-14
    assert orc.p_hat(Q, 0, 5, 5).shape[1] == 0


def _same_columns_up_to_sign(P, Ref):
    assert P.shape == Ref.shape
    for j in range(Ref.shape[1]):
        s = 1.0 if P[:, j] @ Ref[:, j] >= 0 else -1.0
        assert np.max(np.abs(s * P[:, j] - Ref[:, j])) < 1e-14, (j, P[:, j], Ref[:, j])


def test_p_hat_hand_derived_single_column():
    """Eq. CP_tilde by hand: xhat = [a, b] with a = (1,0,1,1,0)/sqrt3 and
    b = (0,1,0,0,1)/sqrt2, next active column 0 (shift 0), current active block
    one row (row 0 zeroed): ptilde = (0,0,1,1,0)/sqrt3; removing a (a.ptilde =
    2/3) leaves (-2,0,1,1,0)/(3 sqrt3), b-free, i.e. phat = (-2,0,1,1,0)/sqrt6.
    Zeroing the wrong row (row 2) would give (1,0,-2,1,0)/sqrt6, and the wrong
    column window (shift 1: ptilde = b, already in span(xhat)) no column."""
    a = np.array([1.0, 0.0, 1.0, 1.0, 0.0]) / np.sqrt(3.0)
    b = np.array([0.0, 1.0, 0.0, 0.0, 1.0]) / np.sqrt(2.0)
    xhat = np.stack([a, b], axis=1)
    ph = orc.p_hat(xhat, 0, 1, 1)
    _same_columns_up_to_sign(ph, np.array([[-2.0, 0.0, 1.0, 1.0, 0.0]]).T / np.sqrt(6.0))
    assert orc.p_hat(xhat, 1, 1, 1).shape[1] == 0


def test_p_hat_hand_derived_two_columns():
    """Two active columns and two zeroed rows: xhat = [a, b, c] with a, b as
    above padded by a zero and c = e_6.  ptilde_1 = a with rows 0-1 zeroed
    -> (-2,0,1,1,0,0)/sqrt6 as above; ptilde_2 = b with rows 0-1 zeroed =
    e_5/sqrt2, minus b/2 -> (0,-1,0,0,1,0)/sqrt2 (orthogonal to the first)."""
    a = np.array([1.0, 0.0, 1.0, 1.0, 0.0, 0.0]) / np.sqrt(3.0)
    b = np.array([0.0, 1.0, 0.0, 0.0, 1.0, 0.0]) / np.sqrt(2.0)
    c = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 1.0])
    ph = orc.p_hat(np.stack([a, b, c], axis=1), 0, 2, 2)
    ref = np.stack([np.array([-2.0, 0.0, 1.0, 1.0, 0.0, 0.0]) / np.sqrt(6.0),
                    np.array([0.0, -1.0, 0.0, 0.0, 1.0, 0.0]) / np.sqrt(2.0)], axis=1)
    _same_columns_up_to_sign(ph, ref)


def test_structured_abar_equals_explicit_projection():
    # One exact GCG step on a small pencil: V_old = [X, P, W] B-orthonormal,
    # RR -> (lam, xhat), X_new = V_old xhat, P_new = V_old phat, W_new a fresh
    # block B-orthogonalized against [X_new, P_new]; then the structured Abar of
    # Section 3.2 must equal V_u^T A V_u computed explicitly.
    A = wl.laplace3d_7pt(5)
    n = A.n
    d = wl.diag_uniform(n)
    nx, bs = 8, 3
    V0, _ = orc.recursive_orth_svd(RNG.standard_normal((n, nx + 2 * bs)), "diag", d)
    Ab_old = V0.T @ orc.spmm(A, V0)
    Ab_old = 0.5 * (Ab_old + Ab_old.T)
    lam, xhat = orc.rayleigh_ritz(Ab_old, nx)
    ph = orc.p_hat(xhat, 1, bs, bs)
    Xn = V0 @ xhat
    Pn = V0 @ ph
    Wn = RNG.standard_normal((n, bs))
    Q = np.hstack([Xn, Pn])
    Wn, _ = orc.deflate(Wn, Q, "diag", d)
    Wn, kw = orc.recursive_orth_svd(Wn, "diag", d)
    Vu = np.hstack([Xn, Pn, Wn])
    G = Vu.T @ orc.spmm(A, Wn)
    Ab = orc.assemble_abar(lam, ph.T @ Ab_old @ ph, G, nx, ph.shape[1], kw)
    Ex = Vu.T @ orc.spmm(A, Vu)
    assert np.max(np.abs(Ab - Ex)) < 1e-10 * np.abs(Ex).max()


# ---------------------------------------------------------------- gradients

def test_eig_grad_against_central_differences():
    n = 4
    A = wl.varcoef3d_7pt(n)          # 64 x 64, B = I
    nev = 6
    lam, X = orc.pencil_eigs(A, "identity", None, nev)
    g = np.array([0.3, -1.2, 0.7, 1.1, -0.4, 0.9])
    gA = orc.eig_grad(A, X, lam, g)
    rows = A.row_of_entry()
    for e in [0, 5, 77, 150, 300]:
        r, c = int(rows[e]), int(A.colind[e])
        # symmetric perturbation of the pair (r, c), (c, r)
        e2 = int(np.nonzero((rows == c) & (A.colind == r))[0][0])
        step = 1e-6 * abs(A.val[e])
        vp = A.val.copy()
        vm = A.val.copy()
        vp[e] += step
        vm[e] -= step
        if e2 != e:
            vp[e2] += step
            vm[e2] -= step
        lp, _ = orc.pencil_eigs(A.with_values(vp), "identity", None, nev)
        lm, _ = orc.pencil_eigs(A.with_values(vm), "identity", None, nev)
        fd = (g @ lp - g @ lm) / (2 * step)
        an = gA[e] + (gA[e2] if e2 != e else 0.0)
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (e, fd, an)


def test_eig_grad_b_csr_and_diag():
    n = 3
    A, B = wl.q1_fem(n)
    nev = 4
    lam, X = orc.pencil_eigs(A, "csr", B, nev)
    g = np.array([1.0, -0.5, 0.25, 2.0])
    gB = orc.eig_grad(B, X, lam, g, kind="B")
    rows = B.row_of_entry()
    e = int(np.nonzero(rows == B.colind)[0][4])   # a diagonal entry
    step = 1e-6 * B.val[e]
    vp = B.val.copy(); vp[e] += step
    vm = B.val.copy(); vm[e] -= step
    lp, _ = orc.pencil_eigs(A, "csr", B.with_values(vp), nev)
    lm, _ = orc.pencil_eigs(A, "csr", B.with_values(vm), nev)
    fd = (g @ lp - g @ lm) / (2 * step)
    assert abs(fd - gB[e]) < 1e-6 * max(1.0, abs(gB[e]))
    # diagonal B
    A2 = wl.laplace3d_7pt(3)
    d = wl.diag_uniform(A2.n)
    lam2, X2 = orc.pencil_eigs(A2, "diag", d, 3)
    g2 = np.array([1.0, 0.5, -1.0])
    gd = orc.eig_grad_diag(X2, lam2, g2)
    j = 7
    step = 1e-6 * d[j]
    dp = d.copy(); dp[j] += step
    dm = d.copy(); dm[j] -= step
    lp, _ = orc.pencil_eigs(A2, "diag", dp, 3)
    lm, _ = orc.pencil_eigs(A2, "diag", dm, 3)
    assert abs((g2 @ lp - g2 @ lm) / (2 * step) - gd[j]) < 1e-6 * max(1.0, abs(gd[j]))


def test_modified_block_orth_drops_columns_dependent_on_earlier_blocks():
    """Algorithm 2 keeps one column per independent direction: a column equal
    to a combination of columns in earlier blocks is reduced to rounding by
    those blocks' deflations and must be dropped, like a duplicate inside a
    block; the output spans the input."""
    rng = np.random.default_rng(11)
    X = rng.standard_normal((200, 24))
    X[:, 5] = X[:, 2]                          # duplicate inside the first block
    X[:, 17] = X[:, 1] - 2.0 * X[:, 9]         # dependent on the first two blocks
    Xo, k = orc.modified_block_orth(X, None, "identity", None, b=6, drop_tol=1e-4)
    assert k == 22
    assert np.max(np.abs(Xo.T @ Xo - np.eye(k))) < 1e-13
    proj = Xo @ (Xo.T @ X)
    assert np.max(np.abs(proj - X)) < 1e-12 * np.max(np.abs(X))
