"""End-to-end GCG solves on the GPU against the oracle (reduced grids, element
by element) and against closed forms / invariants (full grids)."""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from closed_forms import lap2d_eigs, lap3d_eigs, q1_eigs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_06552_amd as gg
    gg._lib.load()
    return gg


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def to_dev(g, bkind, B):
    if bkind == "identity":
        return None
    if bkind == "diag":
        return torch.as_tensor(B, dtype=torch.float64, device="cuda")
    return g.DeviceCsr.from_csr(B)


def gpu_solve(g, A, bkind, B, nev, tol=1e-8, **opts):
    Ad = g.DeviceCsr.from_csr(A)
    Bd = to_dev(g, bkind, B)
    with g.Solver(Ad, Bd, nev, tol, **opts) as s:
        lam, X, st = s.solve()
    return lam.numpy(), host(X), st


def check_pairs(A, bkind, B, lam, X, tol, orth=1e-12):
    rel = orc.relative_residuals(A, bkind, B, X, lam)
    assert rel.max() <= tol, rel.max()
    G = X.T @ orc.apply_b(bkind, B, X)
    assert np.max(np.abs(G - np.eye(len(lam)))) < orth
    assert np.all(np.diff(lam) >= -1e-12 * np.abs(lam).max())


def compare_vectors(bkind, B, lam_o, X_o, X, nev, gap=1e-8):
    """Per cluster of the oracle spectrum (relative gap < gap): the GPU vectors
    span the same subspace (singular values of X^T B X_o near 1)."""
    i = 0
    while i < nev:
        j = i + 1
        while j < len(lam_o) and abs(lam_o[j] - lam_o[i]) <= gap * abs(lam_o[i]):
            j += 1
        if j <= nev:
            M = X[:, i:j].T @ orc.apply_b(bkind, B, X_o[:, i:j])
            s = np.linalg.svd(M, compute_uv=False)   # test-only
            assert s.min() > 1 - 1e-8, (i, j, s)
        i = j


def test_config1_full_grid_closed_form(g):
    A = wl.laplace2d_5pt(64)
    lam, X, st = gpu_solve(g, A, "identity", None, 10, block_size=10)
    ex = lap2d_eigs(64)[:10]
    assert np.max(np.abs(lam - ex) / ex) < 1e-10
    check_pairs(A, "identity", None, lam, X, 1e-8)
    assert st["status"] == 0 and st["max_rel_residual"] <= 1e-8


CASES = [
    ("lap2d_24", lambda: (wl.laplace2d_5pt(24), "identity", None), 10, dict(block_size=10)),
    ("lap3d_10_diagB", lambda: (wl.laplace3d_7pt(10), "diag", wl.diag_uniform(1000)), 20, dict(block_size=5)),
    ("lap3d_10_diagB_mixed", lambda: (wl.laplace3d_7pt(10), "diag", wl.diag_uniform(1000)), 20,
     dict(block_size=5, precision="mixed")),
    ("q1fem_9_moving", lambda: (*wl.q1_fem(9)[:1], "csr", wl.q1_fem(9)[1]), 40, dict(block_size=8, moving=1)),
    ("q1fem_9", lambda: (*wl.q1_fem(9)[:1], "csr", wl.q1_fem(9)[1]), 24, dict(block_size=6)),
    ("varcoef_10", lambda: (wl.varcoef3d_7pt(10), "identity", None), 10, dict(block_size=3)),
]


@pytest.mark.parametrize("name,make,nev,opts", CASES, ids=[c[0] for c in CASES])
def test_reduced_grid_parity_with_oracle(g, name, make, nev, opts):
    A, bkind, B = make()
    lam_o, X_o = orc.pencil_eigs(A, bkind, B, nev + 8)
    lam, X, st = gpu_solve(g, A, bkind, B, nev, **opts)
    assert np.max(np.abs(lam - lam_o[:nev]) / np.abs(lam_o[:nev])) < 1e-10, (lam - lam_o[:nev])
    check_pairs(A, bkind, B, lam, X, 1e-8)
    compare_vectors(bkind, B, lam_o, X_o, X, nev)
    if opts.get("moving"):
        assert st["moves"] >= 1


@pytest.mark.parametrize("name,make,nev,opts", [
    ("lap3d_10_diagB_alg2", lambda: (wl.laplace3d_7pt(10), "diag", wl.diag_uniform(1000)), 20,
     dict(block_size=5, orth=2)),
    ("q1fem_9_moving_alg2", lambda: (wl.q1_fem(9)[0], "csr", wl.q1_fem(9)[1]), 60,
     dict(block_size=10, moving=1, orth=2, orth_block=4)),
])
def test_reduced_grid_parity_algorithm2(g, name, make, nev, opts):
    """The solver with the modified block orthogonalization (Algorithm 2) in STEP 2."""
    A, bkind, B = make()
    lam, X, st = gpu_solve(g, A, bkind, B, nev, **opts)
    lam_o, X_o = orc.pencil_eigs(A, bkind, B, nev + 6)
    assert np.max(np.abs(lam - lam_o[:nev]) / np.abs(lam_o[:nev])) < 1e-10
    check_pairs(A, bkind, B, lam, X, 1e-8)
    compare_vectors(bkind, B, lam_o, X_o, X, nev)


@pytest.mark.parametrize("name,make,nev,opts", [
    ("lap3d_10_diagB_skipfinal", lambda: (wl.laplace3d_7pt(10), "diag", wl.diag_uniform(1000)), 20,
     dict(block_size=5, orth_skip_final=1)),
    ("q1fem_9_moving_skipfinal", lambda: (wl.q1_fem(9)[0], "csr", wl.q1_fem(9)[1]), 40,
     dict(block_size=8, moving=1, orth_skip_final=1)),
])
def test_reduced_grid_parity_orth_skip_final(g, name, make, nev, opts):
    """The solver with the option that ends Algorithm 3's pass loops before the
    last (sub-tolerance) update: same eigenpairs as the oracle."""
    A, bkind, B = make()
    lam, X, st = gpu_solve(g, A, bkind, B, nev, **opts)
    lam_o, X_o = orc.pencil_eigs(A, bkind, B, nev + 8)
    assert np.max(np.abs(lam - lam_o[:nev]) / np.abs(lam_o[:nev])) < 1e-10
    check_pairs(A, bkind, B, lam, X, 1e-8)
    compare_vectors(bkind, B, lam_o, X_o, X, nev)
    assert st["orth_error"] < 1e-11


def test_deterministic(g):
    A = wl.laplace3d_7pt(12)
    d = wl.diag_uniform(A.n)
    r1 = gpu_solve(g, A, "diag", d, 16, block_size=4)
    r2 = gpu_solve(g, A, "diag", d, 16, block_size=4)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])


@pytest.mark.parametrize("prec,precond", [("fp64", 0), ("mixed", 0), ("fp64", 1), ("mixed", 1)])
def test_cg_history_gives_the_same_solve_to_the_bit(g, prec, precond):
    """The inner CG with a search-direction history forms x = sum_i alpha_i p_i
    when the ring of H slots fills and at the end, in the order of the steps;
    the solve is the same to the bit as with x updated in every step
    (cg_history = 0), for every ring size, with and without the multigrid
    preconditioner and in both precisions."""
    A = wl.laplace3d_7pt(14)
    d = wl.diag_uniform(A.n)
    opts = dict(block_size=8, precision=prec, precond=precond)
    ref = gpu_solve(g, A, "diag", d, 24, **opts, cg_history=0)
    assert ref[2]["status"] == 0
    for H in (2, 3, 7, 32):
        r = gpu_solve(g, A, "diag", d, 24, **opts, cg_history=H)
        # (cg_iterations counts the steps the host enqueued before its
        # non-blocking poll saw convergence, a timing matter; the steps past
        # convergence do nothing on the device)
        assert r[2]["iterations"] == ref[2]["iterations"], H
        assert np.array_equal(r[0], ref[0]) and np.array_equal(r[1], ref[1]), H
    # a fixed CG length (no early stop) with a ring that fills several times
    fixed = dict(block_size=8, precision=prec, precond=precond, cg_max_iter=9)
    ref = gpu_solve(g, A, "diag", d, 24, **fixed, cg_history=0, cg_rel_tol=0.0)
    r = gpu_solve(g, A, "diag", d, 24, **fixed, cg_history=4, cg_rel_tol=0.0)
    assert np.array_equal(r[0], ref[0]) and np.array_equal(r[1], ref[1])


def test_cg_history_option_range(g):
    Ad = g.DeviceCsr.from_csr(wl.laplace3d_7pt(6))
    with g.Solver(Ad, None, 4, 1e-8) as s:
        for bad in (1, 33, -1):
            with pytest.raises(Exception):
                s.set_options(cg_history=bad)
        s.set_options(cg_history=0)
        s.set_options(cg_history=2)


def test_edge_cases(g):
    # nev == n: the initial block spans the whole space
    A = wl.laplace2d_5pt(4)
    lam, X, st = gpu_solve(g, A, "identity", None, 16, block_size=4)
    assert np.max(np.abs(lam - lap2d_eigs(4)) / lap2d_eigs(4)) < 1e-10
    # nev = 1
    A = wl.laplace3d_7pt(7)
    lam, X, st = gpu_solve(g, A, "identity", None, 1)
    assert abs(lam[0] - lap3d_eigs(7)[0]) / lam[0] < 1e-10
    # max_iter reached: status NOT_CONVERGED, best approximations returned
    Ad = g.DeviceCsr.from_csr(wl.laplace3d_7pt(12))
    with g.Solver(Ad, None, 10, 1e-12, max_iter=1, block_size=2) as s:
        lam, X, st = s.solve(raise_not_converged=False)
    assert st["status"] == 1 and np.all(np.isfinite(lam.numpy()))


def test_warm_start_reduces_iterations(g):
    A = wl.laplace3d_7pt(12)
    d = wl.diag_uniform(A.n)
    Ad = g.DeviceCsr.from_csr(A)
    with g.Solver(Ad, torch.as_tensor(d, device="cuda"), 12, 1e-9, block_size=4) as s:
        lam, X, st = s.solve()
        it0 = st["iterations"]
        s.set_initial_vectors(X.clone())
        lam2, X2, st2 = s.solve()
    assert st2["iterations"] < it0
    assert np.max(np.abs(lam2.numpy() - lam.numpy()) / lam.numpy()) < 1e-10


def test_indefinite_b_is_rejected(g):
    """B must be positive definite (Section 2): a diagonal B with a
    non-positive entry, a CSR B with a non-positive or missing diagonal entry,
    and such a B passed to update_values return GCGE_ERR_NOT_SPD."""
    from paper_2111_06552_amd import _lib
    A = wl.laplace3d_7pt(6)
    Ad = g.DeviceCsr.from_csr(A)
    d = wl.diag_uniform(A.n)
    for bad in (-0.25, 0.0, float("nan")):
        dd = d.copy()
        dd[37] = bad
        with pytest.raises(_lib.GcgeError) as ei:
            g.Solver(Ad, torch.as_tensor(dd, device="cuda"), 4, 1e-8)
        assert ei.value.code == _lib.GCGE_ERR_NOT_SPD and "row 37" in str(ei.value)
    # CSR B: the mass matrix of the Q1 operator with one diagonal entry negated
    Aq, Bq = wl.q1_fem(4)
    rows = Bq.row_of_entry()
    e = int(np.nonzero((rows == 9) & (Bq.colind == 9))[0][0])
    v = Bq.val.copy()
    v[e] = -v[e]
    with pytest.raises(_lib.GcgeError) as ei:
        g.Solver(g.DeviceCsr.from_csr(Aq), g.DeviceCsr.from_csr(Bq.with_values(v)), 4, 1e-8)
    assert ei.value.code == _lib.GCGE_ERR_NOT_SPD and "row 9" in str(ei.value)
    # CSR B without a stored diagonal in row 0 (an off-diagonal-only row)
    keep = ~((rows == 0) & (Bq.colind == 0))
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=Bq.n))]).astype(np.int32)
    Bm = wl.Csr(Bq.n, rp, Bq.colind[keep].astype(np.int32), Bq.val[keep])
    with pytest.raises(_lib.GcgeError) as ei:
        g.Solver(g.DeviceCsr.from_csr(Aq), g.DeviceCsr.from_csr(Bm), 4, 1e-8)
    assert ei.value.code == _lib.GCGE_ERR_NOT_SPD and "row 0" in str(ei.value)
    # a valid solver whose diagonal B is replaced by an indefinite one
    with g.Solver(Ad, torch.as_tensor(d, device="cuda"), 4, 1e-8) as s:
        dd = torch.as_tensor(d, device="cuda").clone()
        dd[5] = -1.0
        with pytest.raises(_lib.GcgeError) as ei:
            s.update_values(None, dd)
        assert ei.value.code == _lib.GCGE_ERR_NOT_SPD


def test_gradient_needs_its_own_solve(g):
    """backward reads the solver's last eigenvectors: after a second forward on
    the same solver, the first graph's backward raises instead of returning the
    second solve's gradient; the second graph's backward works."""
    A = wl.laplace3d_7pt(6)
    Ad = g.DeviceCsr.from_csr(A)
    with g.Solver(Ad, None, 3, 1e-10, block_size=3) as s:
        a1 = torch.as_tensor(A.val, device="cuda").clone().requires_grad_(True)
        l1 = g.eigvals(a1, s)
        a2 = (torch.as_tensor(A.val, device="cuda") * 1.5).requires_grad_(True)
        l2 = g.eigvals(a2, s)
        with pytest.raises(RuntimeError, match="another solve"):
            l1.sum().backward()
        l2.sum().backward()
        assert a2.grad is not None and torch.isfinite(a2.grad).all()


def test_gradient_after_an_unconverged_solve_is_refused(g):
    from paper_2111_06552_amd import _lib
    A = wl.laplace3d_7pt(10)
    Ad = g.DeviceCsr.from_csr(A)
    with g.Solver(Ad, None, 8, 1e-12, max_iter=1, block_size=2) as s:
        lam, X, st = s.solve(raise_not_converged=False)
        assert st["status"] == _lib.GCGE_NOT_CONVERGED
        with pytest.raises(_lib.GcgeError) as ei:
            s.eig_grad(np.ones(8))
        assert ei.value.code == _lib.GCGE_NOT_CONVERGED
