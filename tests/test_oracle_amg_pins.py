"""Pins of the AMG/PCG oracle (the preconditioned inner solve of Section 2)
against hand-derived cases, library routines and invariants.  (No GPU.)"""
import numpy as np
import pytest

import oracle.amg as amg
import workloads as wl
from oracle.core import cg_columnwise


def lap1d(n):
    """tridiag(-1, 2, -1), n x n."""
    rp, ci, va = [0], [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                ci.append(j)
                va.append(v)
        rp.append(len(ci))
    return wl.Csr(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))


def test_aggregates_of_the_1d_laplacian_by_hand():
    # eps = 0.08: every off-diagonal entry is strong (1 >= 0.08 * sqrt(2 * 2)).
    # Phase 1 in row order: row 0 -> {0, 1}; row 2 is blocked by 1; row 3 ->
    # {2, 3, 4}; row 5 is blocked by 4; row 6 -> {5, 6, 7}; row 8 is blocked.
    # Phase 2: row 8 joins the aggregate of its only neighbour 7.
    agg, nagg = amg.aggregate(lap1d(9), 0.08)
    assert nagg == 3
    assert agg.tolist() == [0, 0, 1, 1, 1, 2, 2, 2, 2]


def _graph(n, edges, diag):
    D = diag * np.eye(n)
    for (i, j), a in edges.items():
        D[i, j] = D[j, i] = -a
    return amg._from_dense(D)


@pytest.mark.parametrize("w12,w23,expect", [
    (0.3, 0.7, [0, 0, 1, 1, 1, 1]),                # stronger link to row 3 (aggregate 1)
    (0.7, 0.3, [0, 0, 0, 1, 1, 1]),                # stronger link to row 1 (aggregate 0)
    (0.5, 0.5, [0, 0, 0, 1, 1, 1]),                # tie: first neighbour in column order
    (0.5, 0.5 * (1 + 1e-12), [0, 0, 0, 1, 1, 1]),  # within the relative tie margin
    (0.5, 0.5 * (1 + 1e-6), [0, 0, 1, 1, 1, 1]),   # beyond it
])
def test_phase_two_joins_the_strongest_phase_one_neighbour(w12, w23, expect):
    # Edges 0-1, 1-2, 1-3, 2-3, 3-4, 4-5, diagonal 2.5 (threshold 0.08 * 2.5 =
    # 0.2, every edge strong).  Phase 1: row 0 seeds {0, 1}; row 2 (neighbour
    # 1 taken) and row 3 (neighbour 1 taken) are blocked; row 4 seeds {3, 4, 5}.
    # Phase 2: row 2 joins the aggregate of its stronger link.
    A = _graph(6, {(0, 1): 1.0, (1, 2): w12, (1, 3): 1.0, (2, 3): w23, (3, 4): 1.0, (4, 5): 1.0}, 2.5)
    agg, nagg = amg.aggregate(A, 0.08)
    assert nagg == 2 and agg.tolist() == expect


def test_weak_links_leave_a_singleton():
    # Diagonal 4 and eps = 0.2: the threshold is 0.8, so the 0.5 links of row 2
    # are weak; row 2 has no strong neighbour and seeds a singleton in phase 1.
    A = _graph(5, {(0, 1): 1.0, (1, 2): 0.5, (2, 3): 0.5, (3, 4): 1.0}, 4.0)
    agg, nagg = amg.aggregate(A, 0.2)
    assert agg.tolist() == [0, 0, 1, 2, 2] and nagg == 3


def test_tentative_prolongator_is_orthonormal():
    A = wl.laplace2d_5pt(9)
    agg, nagg = amg.aggregate(A, 0.08)
    Pt = amg.tentative_p(agg, nagg).to_dense()
    np.testing.assert_allclose(Pt.T @ Pt, np.eye(nagg), atol=1e-15)
    # every row has exactly one entry, the aggregates partition the rows
    assert np.all((Pt != 0).sum(axis=1) == 1)
    assert sorted(set(agg.tolist())) == list(range(nagg))


def test_smoothed_prolongator_column_by_hand():
    # 1D, aggregates {0,1},{2,3,4},{5..8}; rho = max((2+2)/2, (2+1)/2) = 2, so
    # omega = 2/3 and P = Pt - (1/3) A Pt.  Column 0: Pt e_0 = t (e0 + e1),
    # t = 1/sqrt(2); A Pt e_0 = t (e0 + e1 - e2); P e_0 = t (2/3, 2/3, 1/3, 0...).
    H = amg.amg_setup(lap1d(9), coarse_max=2)
    assert H[0]["rho"] == 2.0
    P = H[0]["P"]
    t = 1 / np.sqrt(2)
    np.testing.assert_allclose(P[:, 0], t * np.array([2 / 3, 2 / 3, 1 / 3, 0, 0, 0, 0, 0, 0]), atol=1e-15)


def test_one_level_vcycle_is_the_exact_inverse():
    A = wl.laplace2d_5pt(6)
    H = amg.amg_setup(A, coarse_max=100)
    assert len(H) == 1
    b = np.random.default_rng(1).standard_normal((36, 3))
    np.testing.assert_allclose(amg.amg_vcycle(H, b), np.linalg.solve(A.to_dense(), b), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("make", [lambda: wl.laplace2d_5pt(16), lambda: wl.laplace3d_7pt(7),
                                  lambda: wl.varcoef3d_7pt(7)])
def test_vcycle_is_spd_and_contracts(make):
    A = make()
    n = A.n
    H = amg.amg_setup(A, coarse_max=20)
    assert len(H) >= 2
    V = amg.amg_vcycle(H, np.eye(n))
    np.testing.assert_allclose(V, V.T, atol=1e-12 * np.abs(V).max())
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0
    # error propagation I - V A: spectral radius well below one (a plain
    # Jacobi sweep alone would be 1 - O(h^2))
    E = np.eye(n) - V @ A.to_dense()
    rho = np.abs(np.linalg.eigvals(E)).max()
    assert rho < 0.7, rho


def test_pcg_with_exact_preconditioner_takes_one_step():
    A = wl.laplace2d_5pt(6)
    H = amg.amg_setup(A, coarse_max=100)
    R = np.random.default_rng(2).standard_normal((36, 4))
    X, its = amg.pcg_columnwise(A, H, R, maxit=30, rel_tol=1e-12)
    assert its.tolist() == [1, 1, 1, 1]
    np.testing.assert_allclose(X, np.linalg.solve(A.to_dense(), R), rtol=1e-11, atol=1e-13)


def test_pcg_solves_and_beats_plain_cg():
    A = wl.laplace2d_5pt(24)
    H = amg.amg_setup(A, coarse_max=30)
    R = np.random.default_rng(3).standard_normal((A.n, 2))
    X, its = amg.pcg_columnwise(A, H, R, maxit=200, rel_tol=1e-10)
    np.testing.assert_allclose(X, np.linalg.solve(A.to_dense(), R), rtol=1e-7, atol=1e-9 * np.abs(X).max())
    _, its_cg = cg_columnwise(A, "identity", None, 0.0, R, maxit=500, rel_tol=1e-10)
    assert its.max() * 3 < its_cg.min(), (its, its_cg)


def test_coarsening_stops_on_poor_aggregation_and_dense_levels():
    # No off-diagonal entries: every row is a singleton aggregate, so
    # aggregation would keep all rows and the first level is the coarsest.
    n = 50
    D = amg._from_dense(np.diag(np.arange(1.0, n + 1)))
    H = amg.amg_setup(D, coarse_max=4)
    assert len(H) == 1
    # A level storing more than 400 entries per row is not coarsened.
    rng = np.random.default_rng(4)
    G = rng.standard_normal((450, 450))
    M = amg._from_dense(G @ G.T / 450 + np.eye(450))
    assert M.nnz > 400 * M.n
    assert len(amg.amg_setup(M, coarse_max=4)) == 1
    b = rng.standard_normal((450, 2))
    np.testing.assert_allclose(amg.amg_vcycle(amg.amg_setup(M, coarse_max=4), b),
                               np.linalg.solve(M.to_dense(), b), rtol=1e-10)
