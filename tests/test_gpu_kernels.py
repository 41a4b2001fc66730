"""Parity of each HIP step of one GCG iteration with the CPU oracle, through
the C ABI (sizes span several tiles and a ragged tail; edge cases included)."""
import numpy as np
import pytest

import oracle as orc
import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_06552_amd as gg
    gg._lib.load()
    return gg


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


RNG = np.random.default_rng(2024)


def random_csr(n, per_row, empty_rows=(), seed=0):
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(n):
        if i in empty_rows:
            continue
        c = np.unique(rng.integers(0, n, per_row))
        rows += [i] * len(c)
        cols += c.tolist()
        vals += rng.standard_normal(len(c)).tolist()
    rows = np.array(rows)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    return wl.Csr(n, np.cumsum(rowptr).astype(np.int32), np.array(cols, dtype=np.int32), np.array(vals))


def abs_csr(A):
    return A.with_values(np.abs(A.val))


@pytest.mark.parametrize("k", [1, 7, 16, 17, 50, 64, 65, 100, 128, 130])
def test_spmm_fp64(g, k):
    A = random_csr(1037, 7, empty_rows=(0, 5, 1036))
    X = RNG.standard_normal((A.n, k))
    ld = k + 3
    Xd = torch.zeros((A.n, ld), dtype=torch.float64, device="cuda")
    Xd[:, :k] = dev(X)
    Y = g.spmm(g.DeviceCsr.from_csr(A), Xd[:, :k])
    ref = orc.spmm(A, X)
    bound = orc.spmm(abs_csr(A), np.abs(X))
    assert np.all(np.abs(host(Y) - ref) <= 1e-13 * bound + 1e-300)


def test_spmm_stencils_and_fp32(g):
    for A in (wl.laplace2d_5pt(33), wl.laplace3d_7pt(11), wl.q1_fem(7)[0]):
        X = RNG.standard_normal((A.n, 10))
        Ad = g.DeviceCsr.from_csr(A)
        Y = host(g.spmm(Ad, dev(X)))
        ref = orc.spmm(A, X)
        assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(orc.spmm(abs_csr(A), np.abs(X)))
        X32 = X.astype(np.float32)
        Y32 = host(g.spmm_f32(Ad, dev(A.val, torch.float32), dev(X32, torch.float32)))
        ref32 = orc.spmm(A.with_values(A.val.astype(np.float32).astype(np.float64)), X32.astype(np.float64))
        scale = orc.spmm(abs_csr(A), np.abs(X32.astype(np.float64)))
        assert np.max(np.abs(Y32 - ref32) / scale) < 1e-6


@pytest.mark.parametrize("bkind", ["identity", "diag", "csr_same", "csr_other"])
def test_shifted_spmm_and_residual(g, bkind):
    A = wl.laplace3d_7pt(9)
    n = A.n
    if bkind == "identity":
        B, Bd = None, None
        ok, ob = "identity", None
    elif bkind == "diag":
        d = wl.diag_uniform(n)
        B, Bd, ok, ob = d, dev(d), "diag", d
    elif bkind == "csr_same":
        B = A.with_values(np.abs(A.val) / 1000 + 0.01)
        Bd, ok, ob = g.DeviceCsr.from_csr(B), "csr", B
    else:
        B = random_csr(n, 3, seed=9)
        Bd, ok, ob = g.DeviceCsr.from_csr(B), "csr", B
    k = 19
    X = RNG.standard_normal((n, k))
    sig = RNG.uniform(10, 200, k)
    Ad = g.DeviceCsr.from_csr(A)
    Y = host(g.shifted_spmm(Ad, Bd, dev(X), sig))
    ref = orc.shifted_spmm(A, ok, ob, X, sig)
    assert np.max(np.abs(Y - ref)) < 1e-12 * np.max(np.abs(ref))
    R, rn, bn = g.residual(Ad, Bd, dev(X), sig)
    Rr, rnr, bnr = orc.residual(A, ok, ob, X, sig)
    assert np.max(np.abs(host(R) - Rr)) < 1e-12 * np.max(np.abs(Rr))
    assert np.max(np.abs(rn - rnr) / rnr) < 1e-13 and np.max(np.abs(bn - bnr) / bnr) < 1e-13


@pytest.mark.parametrize("n,m,k", [(1, 1, 1), (15, 3, 2), (1000, 16, 16), (4099, 17, 5), (20000, 50, 50),
                                   (12345, 65, 64), (9999, 130, 33), (7000, 350, 50), (3000, 400, 100)])
def test_gram(g, n, m, k):
    X = RNG.standard_normal((n, m))
    Y = RNG.standard_normal((n, k))
    d = RNG.uniform(0.5, 1.5, n)
    for dd in (None, d):
        C = g.gram(dev(X), dev(Y), None if dd is None else dev(dd))
        ref = orc.gram(X, Y, dd)
        bound = orc.gram(np.abs(X), np.abs(Y), dd)
        assert np.all(np.abs(C - ref) <= 1e-13 * bound + 1e-300)
    C1 = g.gram(dev(X), dev(Y))
    C2 = g.gram(dev(X), dev(Y))
    assert np.array_equal(C1, C2)   # fixed summation order


@pytest.mark.parametrize("n,m", [(1, 1), (1000, 16), (4099, 13), (3001, 32), (777, 7), (20000, 20)])
def test_gram_self(g, n, m):
    """X^T D X with Y the very same device buffer (the Algorithm 3 leaf Gram,
    where the kernel does not load Y separately)."""
    X = RNG.standard_normal((n, m))
    d = RNG.uniform(0.5, 1.5, n)
    Xd = dev(X)
    for dd in (None, d):
        C = g.gram(Xd, Xd, None if dd is None else dev(dd))
        ref = orc.gram(X, X, dd)
        bound = orc.gram(np.abs(X), np.abs(X), dd)
        assert np.all(np.abs(C - ref) <= 1e-13 * bound + 1e-300)


@pytest.mark.parametrize("n,m,k", [(1, 1, 1), (63, 5, 3), (1000, 16, 16), (5001, 25, 32), (2049, 32, 7),
                                   (100, 3, 32), (4099, 50, 50), (5000, 450, 350), (777, 100, 130),
                                   (1, 16, 9), (130, 12, 16), (65537, 13, 12), (64, 9, 1)])
def test_gemm_update(g, n, m, k):
    X = RNG.standard_normal((n, m))
    S = RNG.standard_normal((m, k))
    Y0 = RNG.standard_normal((n, k))
    Y = g.gemm_update(dev(X), S, dev(Y0), alpha=-1.5, beta=0.5)
    ref = -1.5 * (X @ S) + 0.5 * Y0
    bound = 1.5 * (np.abs(X) @ np.abs(S)) + 0.5 * np.abs(Y0)
    assert np.all(np.abs(host(Y) - ref) <= 1e-13 * bound)


@pytest.mark.parametrize("s0,k,kout", [(0, 16, 12), (3, 25, 25), (7, 9, 16), (1, 60, 50), (2, 13, 13)])
def test_gemm_in_place_row_transform(g, s0, k, kout):
    """Y aliases X (the in-place updates of Algorithm 3), columns starting at
    an odd offset of a wider block."""
    n = 3001
    W = RNG.standard_normal((n, 64))
    S = RNG.standard_normal((k, kout))
    Wd = dev(W)
    X = W[:, s0:s0 + k].copy()
    g.gemm_update(Wd[:, s0:s0 + k], S, Wd[:, s0:s0 + kout])
    out = host(Wd)
    assert np.max(np.abs(out[:, s0:s0 + kout] - X @ S)) <= 1e-13 * np.max(np.abs(X) @ np.abs(S))
    assert np.array_equal(out[:, :s0], W[:, :s0]) and np.array_equal(out[:, s0 + kout:], W[:, s0 + kout:])


@pytest.mark.parametrize("k,kout", [(16, 16), (13, 9), (6, 8), (25, 30)])
def test_gemm_in_place_with_beta(g, k, kout):
    """Y = alpha X S + beta Y with Y the same columns as X (each row is read
    before it is written), for the 8-, 16- and 32-lane row kernels."""
    n = 4099
    W = RNG.standard_normal((n, 40))
    S = RNG.standard_normal((k, kout))
    Wd = dev(W)
    g.gemm_update(Wd[:, 2:2 + k], S, Wd[:, 2:2 + kout], alpha=0.75, beta=-0.5)
    out = host(Wd)
    ref = 0.75 * (W[:, 2:2 + k] @ S) - 0.5 * W[:, 2:2 + kout]
    bound = 0.75 * (np.abs(W[:, 2:2 + k]) @ np.abs(S)) + 0.5 * np.abs(W[:, 2:2 + kout])
    assert np.all(np.abs(out[:, 2:2 + kout] - ref) <= 1e-13 * bound)
    assert np.array_equal(out[:, :2], W[:, :2]) and np.array_equal(out[:, 2 + kout:], W[:, 2 + kout:])


def test_gemm_overlap_other_than_a_row_transform_is_rejected(g):
    """Y overlapping X must be a row transform (row i of Y inside row i of X's
    stride): Y = X shifted by one row, or by columns past the stride, is an
    invalid argument and nothing is launched."""
    from paper_2111_06552_amd import _lib
    W = RNG.standard_normal((500, 24))
    Wd = dev(W)
    S = RNG.standard_normal((8, 8))
    with pytest.raises(_lib.GcgeError) as ei:
        g.gemm_update(Wd[:-1, 0:8], S, Wd[1:, 0:8])        # Y = X + ldx
    assert ei.value.code == _lib.GCGE_ERR_INVALID_ARG
    Yv = torch.as_strided(Wd, (499, 8), (24, 1), storage_offset=20)   # row i of Y runs into row i + 1 of X
    with pytest.raises(_lib.GcgeError):
        g.gemm_update(Wd[:499, 0:8], S, Yv)
    assert np.array_equal(host(Wd), W)
    g.gemm_update(Wd[:, 0:8], S, Wd[:, 10:18])              # disjoint columns of the same rows: allowed
    assert np.max(np.abs(host(Wd)[:, 10:18] - W[:, 0:8] @ S)) <= 1e-13 * np.max(np.abs(W[:, 0:8]) @ np.abs(S))


@pytest.mark.parametrize("maxit", [1, 2, 5, 30])
def test_cg_fp64_matches_oracle(g, maxit):
    A = wl.laplace3d_7pt(10)
    d = wl.diag_uniform(A.n)
    R = RNG.standard_normal((A.n, 12))
    theta = 25.0
    D, its = g.cg(g.DeviceCsr.from_csr(A), dev(d), theta, dev(R), maxit=maxit, rel_tol=1e-2)
    ref, its_r = orc.cg_columnwise(A, "diag", d, theta, R, maxit=maxit, rel_tol=1e-2)
    assert np.array_equal(its, its_r)
    assert np.max(np.abs(host(D) - ref)) < 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("k", [1, 7, 26, 33, 40, 50, 64, 100])
def test_cg_fp64_block_widths(g, k):
    """Every stored-width layout of the CG vectors (flat kernels with 1 to 13
    slots per thread, and the row-group kernels beyond), ragged row counts."""
    A = wl.laplace3d_7pt(11)
    d = wl.diag_uniform(A.n)
    R = RNG.standard_normal((A.n, k))
    D, its = g.cg(g.DeviceCsr.from_csr(A), dev(d), 30.0, dev(R), maxit=6, rel_tol=1e-3)
    ref, its_r = orc.cg_columnwise(A, "diag", d, 30.0, R, maxit=6, rel_tol=1e-3)
    assert np.array_equal(its, its_r)
    assert np.max(np.abs(host(D) - ref)) < 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cg_plane_blocked_spmm_order(g, precision):
    """A 48^3 grid couples rows 2304 apart: the operator's SpMM visits row
    blocks plane by plane within blocks of positions; the products (and so the
    CG iterates) must equal natural order's."""
    A = wl.laplace3d_7pt(48)
    d = wl.diag_uniform(A.n)
    R = RNG.standard_normal((A.n, 8))
    D, its = g.cg(g.DeviceCsr.from_csr(A), dev(d), 40.0, dev(R), maxit=3, rel_tol=0.0, precision=precision)
    ref, _ = orc.cg_columnwise(A, "diag", d, 40.0, R, maxit=3, rel_tol=0.0)
    tol = 1e-12 if precision == "fp64" else 1e-4
    assert np.max(np.abs(host(D) - ref)) < tol * np.max(np.abs(ref))


def test_cg_fp64_plane_blocked_order_full_width(g):
    """The FP64 CG product at the benchmark's block width (50 columns, 32
    lanes per row) over the plane-blocked row order of a 48^3 grid."""
    A = wl.laplace3d_7pt(48)
    d = wl.diag_uniform(A.n)
    R = RNG.standard_normal((A.n, 50))
    D, its = g.cg(g.DeviceCsr.from_csr(A), dev(d), 40.0, dev(R), maxit=3, rel_tol=0.0)
    ref, _ = orc.cg_columnwise(A, "diag", d, 40.0, R, maxit=3, rel_tol=0.0)
    assert np.max(np.abs(host(D) - ref)) < 1e-12 * np.max(np.abs(ref))


def arrow_matrix(m):
    """A 2D five-point Laplacian (m x m) plus rows 0 and n // 2 coupled to
    every row with weight -1e-3 (and the diagonal raised to keep it SPD by
    diagonal dominance): the row blocks holding those two rows carry more
    nonzeros than the SpMM's LDS pattern stage (1 024), so they read the
    pattern from global memory."""
    L = wl.laplace2d_5pt(m)
    n = L.n
    D = L.to_dense()
    for h in (0, n // 2):
        D[h, :] -= 1e-3
        D[:, h] -= 1e-3
        D[h, h] += 2e-3
    D += np.diag(np.abs(D).sum(axis=1) - np.abs(np.diag(D)) - np.diag(D) + 4.0 * (np.abs(np.diag(D)) > 0))
    rows, cols = np.nonzero(D)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    return wl.Csr(n, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), D[rows, cols].astype(np.float64))


@pytest.mark.parametrize("k", [8, 50])
def test_cg_fp64_long_rows(g, k):
    A = arrow_matrix(40)
    assert np.max(np.diff(A.rowptr)) == A.n
    R = RNG.standard_normal((A.n, k))
    D, its = g.cg(g.DeviceCsr.from_csr(A), None, 0.0, dev(R), maxit=5, rel_tol=0.0)
    ref, _ = orc.cg_columnwise(A, "identity", None, 0.0, R, maxit=5, rel_tol=0.0)
    assert np.max(np.abs(host(D) - ref)) < 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("k", [13, 50, 100])
def test_cg_mixed_block_widths(g, k):
    A = wl.laplace3d_7pt(11)
    R = RNG.standard_normal((A.n, k))
    D, its = g.cg(g.DeviceCsr.from_csr(A), None, 0.0, dev(R), maxit=6, rel_tol=0.0, precision="mixed")
    ref, _ = orc.cg_columnwise(A, "identity", None, 0.0, R, maxit=6, rel_tol=0.0)
    assert np.max(np.abs(host(D) - ref)) < 1e-4 * np.max(np.abs(ref))
    assert np.all(its == 6)


def test_cg_mixed_precision_close_to_oracle(g):
    A = wl.laplace3d_7pt(10)
    R = RNG.standard_normal((A.n, 10))
    D, its = g.cg(g.DeviceCsr.from_csr(A), None, 0.0, dev(R), maxit=8, rel_tol=0.0, precision="mixed")
    ref, _ = orc.cg_columnwise(A, "identity", None, 0.0, R, maxit=8, rel_tol=0.0)
    assert np.max(np.abs(host(D) - ref)) < 1e-4 * np.max(np.abs(ref))
    assert np.all(its == 8)


def test_cg_breakdown_freezes_columns(g):
    A = wl.laplace2d_5pt(10)
    R = RNG.standard_normal((A.n, 3))
    D, its = g.cg(g.DeviceCsr.from_csr(A), None, 1e7, dev(R), maxit=30)
    assert np.all(its == 0) and np.all(host(D) == 0)


@pytest.mark.parametrize("bkind", ["identity", "diag", "csr"])
def test_orth_invariants_and_kept_count(g, bkind):
    A, Bq = wl.q1_fem(9)
    n = A.n
    if bkind == "identity":
        Bd, ok, ob = None, "identity", None
    elif bkind == "diag":
        d = wl.diag_uniform(n)
        Bd, ok, ob = dev(d), "diag", d
    else:
        Bd, ok, ob = g.DeviceCsr.from_csr(Bq), "csr", Bq
    Q0 = RNG.standard_normal((n, 30))
    Q, kq = orc.recursive_orth_svd(Q0, ok, ob)
    W0 = RNG.standard_normal((n, 41))
    W0[:, 7] = W0[:, 3]                        # duplicate column
    W0[:, 20] = Q[:, 5] * 2.0                  # inside span(Q)
    W0[:, 33] = W0[:, 1] - 0.5 * W0[:, 30]     # dependent across leaves
    Wd = dev(W0)
    Wo = host(g.orth(Wd, dev(Q), Bd))
    kept = Wo.shape[1]
    ref, kref = orc.deflate(W0, Q, ok, ob)
    ref, kref = orc.recursive_orth_svd(ref, ok, ob)
    assert kept == kref == 38
    BW = orc.apply_b(ok, ob, Wo)
    assert np.max(np.abs(Wo.T @ BW - np.eye(kept))) < 1e-13
    assert np.max(np.abs(Q.T @ BW)) < 1e-13
    # span([Q, Wo]) contains W0
    V = np.hstack([Q, Wo])
    proj = V @ (V.T @ orc.apply_b(ok, ob, W0))
    assert np.max(np.abs(proj - W0)) < 1e-11 * np.max(np.abs(W0))


@pytest.mark.parametrize("bkind", ["identity", "diag", "csr"])
@pytest.mark.parametrize("block", [0, 5])
def test_orth_algorithm2_invariants_and_kept_count(g, bkind, block):
    """Modified block orthogonalization (Algorithm 2) against the oracle's: the
    same deflation against Q, then blocks of b columns (default min(m/4, 200))."""
    A, Bq = wl.q1_fem(9)
    n = A.n
    if bkind == "identity":
        Bd, ok, ob = None, "identity", None
    elif bkind == "diag":
        d = wl.diag_uniform(n)
        Bd, ok, ob = dev(d), "diag", d
    else:
        Bd, ok, ob = g.DeviceCsr.from_csr(Bq), "csr", Bq
    Q0 = RNG.standard_normal((n, 30))
    Q, kq = orc.recursive_orth_svd(Q0, ok, ob)
    W0 = RNG.standard_normal((n, 41))
    W0[:, 7] = W0[:, 3]                        # duplicate inside a block
    W0[:, 20] = Q[:, 5] * 2.0                  # inside span(Q)
    W0[:, 33] = W0[:, 1] - 0.5 * W0[:, 30]     # dependent across blocks
    Wo = host(g.orth(dev(W0), dev(Q), Bd, algorithm=2, block=block))
    kept = Wo.shape[1]
    ref, _ = orc.deflate(W0, Q, ok, ob)
    b = block if block > 0 else max(1, min(ref.shape[1] // 4, 200))
    ref, kref = orc.modified_block_orth(ref, None, ok, ob, b=b, drop_tol=1e-4)
    assert kept == kref == 38
    BW = orc.apply_b(ok, ob, Wo)
    assert np.max(np.abs(Wo.T @ BW - np.eye(kept))) < 1e-13
    assert np.max(np.abs(Q.T @ BW)) < 1e-13
    # the kept columns are those of the oracle up to rounding (Gram-Schmidt fixes them)
    assert np.max(np.abs(Wo - ref)) < 1e-9
    V = np.hstack([Q, Wo])
    proj = V @ (V.T @ orc.apply_b(ok, ob, W0))
    assert np.max(np.abs(proj - W0)) < 1e-11 * np.max(np.abs(W0))


def test_pattern_grad_matches_formula(g):
    A = wl.varcoef3d_7pt(8)
    X = RNG.standard_normal((A.n, 37))
    w = RNG.standard_normal(37)
    gd = host(g.pattern_grad(g.DeviceCsr.from_csr(A), dev(X), w))
    ref = orc.eig_grad(A, X, np.ones(37), w)
    bound = orc.eig_grad(A, np.abs(X), np.ones(37), np.abs(w))
    assert np.all(np.abs(gd - ref) <= 1e-13 * bound)


# ------------------------------------------------------- device dense eigensolver

def _check_dense_eig(g, A, nwant, ref=None):
    """Eigenvalues against the oracle's Jacobi, residuals, orthonormality and
    per-cluster subspaces of the device eigensolver's output."""
    n = A.shape[0]
    w, X = g.dense_eig(dev(A), nwant)
    w, X = host(w), host(X)
    wo, Vo = orc.jacobi_eigh(A) if ref is None else ref
    nrm = max(np.max(np.abs(wo)), 1e-300)
    assert np.all(np.diff(w) >= 0)
    assert np.max(np.abs(w - wo[:nwant])) <= 5e-13 * nrm
    assert np.max(np.abs(X.T @ X - np.eye(nwant))) <= 1e-13
    R = A @ X - X * w[None, :]
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-12 * nrm
    # X^T A X diagonal up to rounding (the structured Rayleigh-Ritz matrix relies on it)
    H = X.T @ A @ X
    assert np.max(np.abs(H - np.diag(np.diag(H)))) <= 1e-12 * nrm
    # subspaces of clusters not cut by nwant
    i = 0
    while i < nwant:
        j = i + 1
        while j < n and wo[j] - wo[j - 1] <= 1e-8 * nrm:
            j += 1
        if j <= nwant:
            s = np.linalg.svd(X[:, i:j].T @ Vo[:, i:j], compute_uv=False)   # test-only
            assert s.min() > 1 - 1e-9, (i, j, s)
        i = j
    return w, X


@pytest.mark.parametrize("n,nwant", [(1, 1), (2, 2), (3, 2), (4, 4), (5, 3), (17, 17), (64, 40), (65, 65), (200, 150),
                                     (300, 200), (310, 250), (384, 384), (385, 100), (450, 350), (513, 300), (640, 64),
                                     (700, 350), (768, 500)])
def test_dense_eig_random_symmetric(g, n, nwant):
    M = RNG.standard_normal((n, n))
    A = (M + M.T) * 10.0
    _check_dense_eig(g, A, nwant)


def test_dense_eig_exact_multiplicities(g):
    """Q diag(lam) Q^T with eigenvalues of multiplicity up to 6, and a diagonal
    matrix with repeated entries (already tridiagonal, every reflector empty)."""
    n = 120
    lam = np.repeat(np.arange(1.0, 21.0) ** 2, 6)
    Q, _ = np.linalg.qr(RNG.standard_normal((n, n)))   # test-only input construction
    A = (Q * lam[None, :]) @ Q.T
    A = 0.5 * (A + A.T)
    _check_dense_eig(g, A, 90, ref=(lam, Q))
    D = np.diag(np.repeat([3.0, 1.0, 2.0, 1.0], 8))
    wo = np.sort(np.diag(D))
    Vo = np.eye(32)[:, np.argsort(np.diag(D), kind="stable")]
    _check_dense_eig(g, D, 32, ref=(wo, Vo))


def test_dense_eig_rayleigh_ritz_structure(g):
    """The structured Abar of STEP 3: diagonal Ritz block, zero X-P block,
    dense P and W blocks, graded couplings."""
    nx, bs = 300, 50
    lam = np.sort(30.0 + 600.0 * RNG.random(nx))
    n = nx + 2 * bs
    A = np.zeros((n, n))
    A[:nx, :nx] = np.diag(lam)
    a0 = RNG.standard_normal((bs, bs))
    A[nx:nx + bs, nx:nx + bs] = 300.0 * np.eye(bs) + 20.0 * (a0 + a0.T)
    a3 = RNG.standard_normal((bs, bs))
    A[nx + bs:, nx + bs:] = 3000.0 * np.eye(bs) + 200.0 * (a3 + a3.T)
    a1 = RNG.standard_normal((nx, bs)) * np.logspace(-8, 1, nx)[:, None]
    A[:nx, nx + bs:] = a1
    A[nx + bs:, :nx] = a1.T
    a2 = 5.0 * RNG.standard_normal((bs, bs))
    A[nx:nx + bs, nx + bs:] = a2
    A[nx + bs:, nx:nx + bs] = a2.T
    _check_dense_eig(g, A, nx)
    _check_dense_eig(g, A, n)


def test_dense_eig_graded_and_deterministic(g):
    n = 96
    Q, _ = np.linalg.qr(RNG.standard_normal((n, n)))   # test-only input construction
    lam = np.sort(np.concatenate([-np.logspace(-8, 4, n // 2), np.logspace(-8, 4, n - n // 2)]))
    A = (Q * lam[None, :]) @ Q.T
    A = 0.5 * (A + A.T)
    w1, X1 = g.dense_eig(dev(A), n)
    w2, X2 = g.dense_eig(dev(A), n)
    assert torch.equal(w1, w2) and torch.equal(X1, X2)
    _check_dense_eig(g, A, n, ref=(lam, Q))


def test_dense_eig_rejects_bad_sizes(g):
    with pytest.raises(Exception):
        g.dense_eig(dev(np.eye(4)), 5)
    with pytest.raises(Exception):
        g.dense_eig(dev(np.eye(769)), 10)
