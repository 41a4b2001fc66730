"""Full-size GPU solves of the benchmark workloads, in the launch configuration
that bench.py times (FP64 and FP32-inner-CG paths, default options).

The dense oracle does not reach these sizes, so each solve is checked against
what holds at any size: exact spectra where the operator has one (constant
coefficients), Courant-Fischer bounds where the coefficients are random,
residuals and B-orthonormality recomputed on the host by the oracle's CSR
products for sampled (or all) columns, agreement of the mixed-precision and
FP64 paths, and, for the gradients, central finite differences of warm-started
solves and the oracle's gradient formula evaluated on the returned vectors."""
import numpy as np
import pytest

import oracle as orc
import workloads as wl
from closed_forms import lap3d_eigs, q1_eigs

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


def sampled_columns(nev, count, seed):
    """``count`` distinct column indices in [0, nev), always including the first and last."""
    u = wl.uniform(seed, np.arange(4 * count, dtype=np.uint64))
    idx = [0, nev - 1]
    for i in (u * nev).astype(int):
        if len(idx) == count:
            break
        if i not in idx:
            idx.append(int(i))
    return np.array(sorted(idx))


def check_sampled(A, bkind, B, lam, X, cols, tol):
    """Residuals of the sampled pairs and B-orthonormality of the sampled
    columns, recomputed by the oracle on the host."""
    Xs = X[:, cols]
    rel = orc.relative_residuals(A, bkind, B, Xs, lam[cols])
    assert rel.max() <= tol * (1 + 1e-6), (rel.max(), cols[np.argmax(rel)])
    G = Xs.T @ orc.apply_b(bkind, B, Xs)
    assert np.max(np.abs(G - np.eye(len(cols)))) < 1e-12


# ------------------------------------------------------------ 128^3, diagonal B

@pytest.fixture(scope="module")
def config2(g):
    A, bkind, B, p = wl.build_workload("lap3d_7pt_128_diagB")
    Ad = g.DeviceCsr.from_csr(A)
    Bd = torch.as_tensor(B, dtype=torch.float64, device="cuda")
    out = {}
    for prec in ("fp64", "mixed"):
        with g.Solver(Ad, Bd, p["nev"], p["tol"], block_size=p["block_size"], precision=prec) as s:
            lam, X, st = s.solve()
            out[prec] = (lam.numpy().copy(), host(X), st)
        print(f"[config2] {prec}: {st['iterations']} iterations, max residual {st['max_rel_residual']:.2e}",
              flush=True)
    return A, B, p, out


def test_config2_fp64_full(config2):
    A, B, p, out = config2
    lam, X, st = out["fp64"]
    nev, tol = p["nev"], p["tol"]
    assert st["status"] == 0 and st["nconv"] == nev
    assert np.all(np.diff(lam) > 0)
    # Courant-Fischer: 0.5 <= D <= 1.5 gives lambda_k(A)/1.5 <= lambda_k(A, D) <= lambda_k(A)/0.5
    ex = lap3d_eigs(128, nev)
    assert np.all(lam >= ex / 1.5 * (1 - 1e-12)) and np.all(lam <= ex / 0.5 * (1 + 1e-12))
    # B-orthonormality of all 200 vectors and residuals of sampled pairs on the host
    G = X.T @ (B[:, None] * X)
    assert np.max(np.abs(G - np.eye(nev))) < 1e-12
    check_sampled(A, "diag", B, lam, X, sampled_columns(nev, 24, 71), tol)


def test_config4_mixed_matches_fp64_full(config2):
    A, B, p, out = config2
    lam64 = out["fp64"][0]
    lam, X, st = out["mixed"]
    assert st["status"] == 0 and st["nconv"] == p["nev"]
    # mixed-precision eigenvalues agree with the FP64 path to 1e-10 relative
    assert np.max(np.abs(lam - lam64) / np.abs(lam64)) < 1e-10
    check_sampled(A, "diag", B, lam, X, sampled_columns(p["nev"], 24, 72), p["tol"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_config2_multigrid_inner_solve_full(g, config2, prec):
    # STEP 6 as PCG at theta = 0 with the multigrid V-cycle (Section 2's
    # suggestion): the same 200 eigenpairs as the FP64 shifted-CG solve.
    A, B, p, out = config2
    lam64 = out["fp64"][0]
    Ad = g.DeviceCsr.from_csr(A)
    Bd = torch.as_tensor(B, dtype=torch.float64, device="cuda")
    with g.Solver(Ad, Bd, p["nev"], p["tol"], block_size=p["block_size"], precision=prec, precond=1) as s:
        lam, X, st = s.solve()
        lam, X = lam.numpy().copy(), host(X)
    print(f"[config2 multigrid] {prec}: {st['iterations']} iterations, {st['cg_iterations']} PCG iterations, "
          f"max residual {st['max_rel_residual']:.2e}", flush=True)
    assert st["status"] == 0 and st["nconv"] == p["nev"]
    assert np.max(np.abs(lam - lam64) / np.abs(lam64)) < 1e-10
    check_sampled(A, "diag", B, lam, X, sampled_columns(p["nev"], 12, 73), p["tol"])


def test_config2_other_initial_block_same_spectrum_full(g, config2):
    """A second FP64 solve from an unrelated random initial block (another
    SplitMix64 seed) converges to the same 200 eigenvalues: a pair missed
    inside a cluster would have to be missed from both starting subspaces."""
    A, B, p, out = config2
    lam64 = out["fp64"][0]
    Ad = g.DeviceCsr.from_csr(A)
    Bd = torch.as_tensor(B, dtype=torch.float64, device="cuda")
    with g.Solver(Ad, Bd, p["nev"], p["tol"], block_size=p["block_size"], seed=7) as s:
        lam, X, st = s.solve()
        lam, X = lam.numpy().copy(), host(X)
    print(f"[config2 seed 7] {st['iterations']} iterations, max residual {st['max_rel_residual']:.2e}", flush=True)
    assert st["status"] == 0 and st["nconv"] == p["nev"]
    assert np.max(np.abs(lam - lam64) / np.abs(lam64)) < 1e-10
    # the leading m vectors of this solve lie in the span of the other's 200:
    # the cosines of the principal angles (singular values of X_7[:, :m]^T D
    # X_1) are 1 up to the residual over the gap that separates lambda_m from
    # the rest of the spectrum (at least lambda_200 - lambda_m; a factor 10
    # covers the norm constants for 0.5 <= D <= 1.5)
    X1 = out["fp64"][1]
    m = p["nev"] - 10
    gap = lam64[-1] - lam64[m - 1]
    sin_bound = 10 * np.sqrt(m) * p["tol"] * lam64[m - 1] / gap
    sv = np.linalg.svd(X[:, :m].T @ (B[:, None] * X1), compute_uv=False)
    assert sv.max() < 1 + 1e-10, sv.max()
    assert sv.min() >= np.sqrt(1 - min(1.0, sin_bound ** 2)) - 1e-12, (sv.min(), sin_bound)


def test_config2_identity_B_closed_form_full(g):
    """128^3 Laplacian with B = I: the 200 smallest eigenvalues are known exactly
    (the 6-fold cluster 197-202 is cut by nev; eigenvalues are still unique)."""
    A = wl.laplace3d_7pt(128)
    Ad = g.DeviceCsr.from_csr(A)
    with g.Solver(Ad, None, 200, 1e-8, block_size=50) as s:
        lam, X, st = s.solve()
    lam = lam.numpy()
    ex = lap3d_eigs(128, 200)
    assert np.max(np.abs(lam - ex) / ex) < 1e-10
    Xh = host(X)
    check_sampled(A, "identity", None, lam, Xh, sampled_columns(200, 16, 73), 1e-8)


# ------------------------------------------------- Q1 FEM 96^3, moving mechanism

def test_config3_moving_full(g):
    A, bkind, B, p = wl.build_workload("q1fem_96_moving")
    Ad = g.DeviceCsr.from_csr(A)
    Bd = g.DeviceCsr.from_csr(B)
    nev, tol = p["nev"], p["tol"]
    with g.Solver(Ad, Bd, nev, tol, block_size=p["block_size"], moving=1) as s:
        lam, X, st = s.solve()
    print(f"[config3] {st['iterations']} iterations, {st['moves']} moves, max residual "
          f"{st['max_rel_residual']:.2e}", flush=True)
    lam = lam.numpy()
    assert st["status"] == 0 and st["nconv"] == nev and st["moves"] >= 1
    assert np.all(np.diff(lam) > 0)
    # 0.1 <= kappa <= 10 per cell: 0.1 lambda_k(K_1, M) <= lambda_k <= 10 lambda_k(K_1, M)
    ex = q1_eigs(96, nev)
    assert np.all(lam >= 0.1 * ex * (1 - 1e-12)) and np.all(lam <= 10 * ex * (1 + 1e-12))
    Xh = host(X)
    del X
    # columns from every stretch of the locked set (before and after each move)
    check_sampled(A, "csr", B, lam, Xh, sampled_columns(nev, 48, 74), tol)


# ------------------------------------- 64^3 variable coefficients, gradients

def transposed_entry(A, e):
    """Index of the stored entry (c, r) for entry e = (r, c) of a symmetric pattern."""
    r = int(np.searchsorted(A.rowptr, e, side="right") - 1)
    c = int(A.colind[e])
    lo, hi = A.rowptr[c], A.rowptr[c + 1]
    t = lo + int(np.searchsorted(A.colind[lo:hi], r))
    assert A.colind[t] == r
    return r, c, t


def test_config5_gradient_full(g):
    A, bkind, B, p = wl.build_workload("varcoef3d_7pt_64_grad")
    nev, bs = p["nev"], p["block_size"]
    w = wl.loss_weights(nev)
    a_val = torch.as_tensor(A.val, dtype=torch.float64, device="cuda")
    Ad = g.DeviceCsr.from_csr(A)
    tight = 1e-11
    with g.Solver(Ad, None, nev + 1, 1e-8, block_size=bs) as s:
        lam51 = s.solve()[0].numpy()
    # simple eigenvalues: every gap among lambda_1 .. lambda_51 at least 1e-6 lambda_50
    assert np.min(np.diff(lam51)) >= 1e-6 * lam51[nev - 1]
    # 0.5 <= c_e <= 2 on every edge: Courant-Fischer between the unit-conductance spectra
    ex = lap3d_eigs(64, nev + 1)
    assert np.all(lam51 >= 0.5 * ex * (1 - 1e-12)) and np.all(lam51 <= 2.0 * ex * (1 + 1e-12))
    with g.Solver(Ad, None, nev, tight, block_size=bs) as s:
        a = a_val.clone().requires_grad_(True)
        lam = g.eigvals(a, s)
        loss = (torch.as_tensor(w, device=lam.device) * lam).sum()
        loss.backward()
        gA = host(a.grad)
        X = s.last_evecs.clone()
        lam0 = lam.detach().cpu().numpy()
        # the backward kernel against the gradient formula on the returned vectors
        ref = orc.eig_grad(A, host(X), lam0, w)
        assert np.max(np.abs(gA - ref)) <= 1e-12 * np.max(np.abs(ref))
        # central differences on 20 sampled stored nonzeros (symmetric pairs
        # perturbed together), relative step 1e-6, warm-started solves
        errs = []
        for e in wl.fd_sample(A):
            r, c, t = transposed_entry(A, int(e))
            h = 1e-6 * abs(A.val[e])
            vals = []
            for sgn in (1.0, -1.0):
                v = a_val.clone()
                v[e] += sgn * h
                if t != e:
                    v[t] += sgn * h
                s.update_values(v)
                s.set_initial_vectors(X)
                lam_p = s.solve()[0].numpy()
                vals.append(float(np.dot(w, lam_p)))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = gA[e] + (gA[t] if t != e else 0.0)
            errs.append((abs(fd - an), abs(an)))
            print(f"[config5] entry {int(e)} ({r}, {c}): gradient {an:.6e}, FD {fd:.6e}, "
                  f"|FD - gradient| {abs(fd - an):.2e}", flush=True)
            assert abs(fd - an) <= 1e-6, (int(e), r, c, fd, an)
            # relative to the entry as well: the differences' noise floor is
            # 1e-8 .. 5e-8 (largest measured 1.2e-8 and 5e-8 on two boxes, over
            # entries of 8e-8 .. 2e-4), so a gradient wrong by 1 % fails for
            # every entry above 1e-5
            assert abs(fd - an) <= 1e-3 * abs(an) + 1e-7, (int(e), r, c, fd, an)
        s.update_values(a_val)
    worst = max(errs)
    print(f"[config5] max |FD - gradient| = {worst[0]:.2e}; gradients {min(a for _, a in errs):.2e} .. "
          f"{max(a for _, a in errs):.2e}", flush=True)


def test_gradient_reduced_grid_vs_oracle(g):
    """On a 10^3 grid the oracle's own eigenvectors give the reference gradient."""
    A = wl.varcoef3d_7pt(10)
    nev = 8
    w = wl.loss_weights(nev)
    lam_o, X_o = orc.pencil_eigs(A, "identity", None, nev + 1)
    assert np.min(np.diff(lam_o)) > 1e-6 * lam_o[-1]
    ref = orc.eig_grad(A, X_o[:, :nev], lam_o[:nev], w)
    Ad = g.DeviceCsr.from_csr(A)
    with g.Solver(Ad, None, nev, 1e-11, block_size=4) as s:
        a = torch.as_tensor(A.val, dtype=torch.float64, device="cuda").requires_grad_(True)
        lam = g.eigvals(a, s)
        (torch.as_tensor(w, device=lam.device) * lam).sum().backward()
    assert np.max(np.abs(lam.detach().cpu().numpy() - lam_o[:nev]) / lam_o[:nev]) < 1e-10
    assert np.max(np.abs(host(a.grad) - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_gradient_diag_B_reduced_grid(g):
    """d lambda_i / d d_j = -lambda_i x_i[j]^2 for a diagonal B, against the
    oracle's eigenvectors and a central difference."""
    A = wl.laplace3d_7pt(8)
    d = wl.diag_uniform(A.n)
    nev = 6
    w = wl.loss_weights(nev)
    lam_o, X_o = orc.pencil_eigs(A, "diag", d, nev + 1)
    assert np.min(np.diff(lam_o)) > 1e-6 * lam_o[-1]
    ref = orc.eig_grad_diag(X_o[:, :nev], lam_o[:nev], w)
    Ad = g.DeviceCsr.from_csr(A)
    dd = torch.as_tensor(d, dtype=torch.float64, device="cuda")
    with g.Solver(Ad, dd, nev, 1e-11, block_size=3) as s:
        lam, X, st = s.solve()
        gA, gB = s.eig_grad(w)
        assert np.max(np.abs(host(gB) - ref)) <= 1e-8 * np.max(np.abs(ref))
        j = 100
        h = 1e-6 * d[j]
        vals = []
        for sgn in (1.0, -1.0):
            d2 = dd.clone()
            d2[j] += sgn * h
            s.update_values(None, d2)
            s.set_initial_vectors(X.clone())
            vals.append(float(np.dot(w, s.solve()[0].numpy())))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - float(host(gB)[j])) <= 1e-6 * max(1.0, abs(fd))


def test_gradient_csr_B_reduced_grid(g):
    """Gradients with respect to the stored nonzeros of A and of a CSR B (Q1
    stiffness and consistent mass on a 7^3 grid with random cell coefficients):
    the backward kernels against the gradient formula on the oracle's
    eigenvectors, and the autograd path against central differences of
    warm-started solves on entries of both matrices."""
    A, Bm = wl.q1_fem(7)
    nev = 6
    w = wl.loss_weights(nev)
    lam_o, X_o = orc.pencil_eigs(A, "csr", Bm, nev + 1)
    assert np.min(np.diff(lam_o)) > 1e-6 * lam_o[-1]
    refA = orc.eig_grad(A, X_o[:, :nev], lam_o[:nev], w)
    refB = orc.eig_grad(Bm, X_o[:, :nev], lam_o[:nev], w, kind="B")
    Ad = g.DeviceCsr.from_csr(A)
    Bd = g.DeviceCsr.from_csr(Bm)
    a_val = torch.as_tensor(A.val, dtype=torch.float64, device="cuda")
    b_val = torch.as_tensor(Bm.val, dtype=torch.float64, device="cuda")
    with g.Solver(Ad, Bd, nev, 1e-11, block_size=3) as s:
        a = a_val.clone().requires_grad_(True)
        b = b_val.clone().requires_grad_(True)
        lam = g.eigvals(a, s, b)
        (torch.as_tensor(w, device=lam.device) * lam).sum().backward()
        gA, gB = host(a.grad), host(b.grad)
        assert np.max(np.abs(lam.detach().cpu().numpy() - lam_o[:nev]) / lam_o[:nev]) < 1e-10
        assert np.max(np.abs(gA - refA)) <= 1e-8 * np.max(np.abs(refA))
        assert np.max(np.abs(gB - refB)) <= 1e-8 * np.max(np.abs(refB))
        X = s.last_evecs.clone()
        for M, vals, grad, which in ((A, a_val, gA, "A"), (Bm, b_val, gB, "B")):
            for e in wl.fd_sample(M, count=4, seed=57):
                r, c, t = transposed_entry(M, int(e))
                # step relative to the matrix's largest entry (entries range over
                # orders of magnitude, some are stored zeros).  A central
                # difference errs by O(h^2) (truncation) plus O(delta f / h),
                # where delta f ~ 1e-14 |f| is the rounding noise between two
                # warm-started solves.  For A (entries ~1.8, gradients ~0.1) a
                # relative step of 1e-4 shows a truncation error of 1.3e-5
                # relative, so 1e-5 leaves ~1.3e-7; at 1e-6 the noise term
                # (delta f ~ 4e-12 over 2h = 3.6e-6) reaches the 1e-5 relative
                # tolerance.  For the mass matrix (entries ~6e-4, gradients
                # ~100) 1e-6 puts the noise term at the tolerance, 1e-5 at about
                # a third of it.
                h = 1e-5 * np.max(np.abs(M.val))
                f = []
                for sgn in (1.0, -1.0):
                    v = vals.clone()
                    v[e] += sgn * h
                    if t != e:
                        v[t] += sgn * h
                    if which == "A":
                        s.update_values(v, b_val)
                    else:
                        s.update_values(a_val, v)
                    s.set_initial_vectors(X)
                    f.append(float(np.dot(w, s.solve()[0].numpy())))
                fd = (f[0] - f[1]) / (2 * h)
                an = grad[e] + (grad[t] if t != e else 0.0)
                assert abs(fd - an) <= 1e-5 * abs(an) + 1e-9, (which, int(e), fd, an)
        s.update_values(a_val, b_val)
