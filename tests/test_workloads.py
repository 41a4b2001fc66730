"""Checks of the seeded input generators (no GPU)."""
import numpy as np
import pytest

import workloads as wl


def test_splitmix64_published_vector():
    # SplitMix64 seeded with 0: the first three outputs of the published generator.
    got = wl.splitmix64(0, np.arange(3, dtype=np.uint64))
    assert [int(x) for x in got] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_range_and_order_independence():
    u = wl.uniform(7, np.arange(10000, dtype=np.uint64))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.02
    idx = np.array([9999, 3, 500], dtype=np.uint64)
    assert np.array_equal(wl.uniform(7, idx), u[[9999, 3, 500]])


def test_normal_moments():
    z = wl.normal(55, np.arange(20000, dtype=np.uint64))
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1.0) < 0.03


def test_initial_block_keying():
    X = wl.initial_block(1, 50, 8)
    assert X.shape == (50, 8) and X.min() >= -1.0 and X.max() < 1.0
    X2 = wl.initial_block(1, 50, 3, col0=5)
    assert np.array_equal(X[:, 5:8], X2)


def _check_csr(A):
    rp = A.rowptr.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == A.nnz and np.all(np.diff(rp) >= 0)
    for i in range(A.n):
        c = A.colind[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0)
    D = A.to_dense()
    assert np.allclose(D, D.T, rtol=0, atol=1e-12 * np.abs(D).max())


@pytest.mark.parametrize("m", [1, 3, 8])
def test_lap2d_structure(m):
    A = wl.laplace2d_5pt(m)
    assert A.n == m * m and A.nnz == 5 * m * m - 4 * m
    _check_csr(A)


def test_workload_sizes_match_stated_nnz():
    # The stated sizes of the five workloads (formulae checked at full size where cheap).
    A = wl.laplace2d_5pt(64)
    assert (A.n, A.nnz) == (4096, 20224)
    n = 128
    assert 7 * n ** 3 - 6 * n ** 2 == 14581760
    n = 96
    assert (3 * n - 2) ** 3 == 23393656
    n = 64
    assert 7 * n ** 3 - 6 * n ** 2 == 1810432


@pytest.mark.parametrize("n", [2, 5])
def test_lap3d_structure(n):
    A = wl.laplace3d_7pt(n)
    assert A.n == n ** 3 and A.nnz == 7 * n ** 3 - 6 * n ** 2
    _check_csr(A)


@pytest.mark.parametrize("n", [3, 6])
def test_varcoef_structure_and_constant_case(n):
    A = wl.varcoef3d_7pt(n)
    assert A.nnz == 7 * n ** 3 - 6 * n ** 2
    _check_csr(A)
    h2 = (n + 1) ** 2
    off = A.val[A.colind != A.row_of_entry()] / -h2
    assert off.min() >= 0.5 and off.max() <= 2.0
    # row sums: interior rows sum to 0 (sum over edges c_e (e_i - e_j)), boundary rows positive
    D = A.to_dense()
    assert np.all(D.sum(axis=1) >= -1e-9)
    L = wl.varcoef3d_7pt(n, constant=True)
    L0 = wl.laplace3d_7pt(n)
    assert np.array_equal(L.rowptr, L0.rowptr) and np.array_equal(L.colind, L0.colind)
    assert np.allclose(L.val, L0.val, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n", [2, 4])
def test_q1_structure(n):
    A, B = wl.q1_fem(n)
    assert A.nnz == (3 * n - 2) ** 3 and np.array_equal(A.colind, B.colind)
    _check_csr(A)
    _check_csr(B)
    # B entries are positive; the mass of each interior node row sums to h^3 (8 cells x h^3/8)
    h = 1.0 / (n + 1)
    assert B.val.min() > 0


def test_q1_element_row_sums():
    # constant kappa: every interior row of A sums to 0 for nodes whose whole 27-neighbourhood is interior
    n = 5
    A, B = wl.q1_fem(n, constant=True)
    D = A.to_dense()
    # node (2,2,2) 0-based is fully interior
    i = 2 + n * (2 + n * 2)
    assert abs(D[i].sum()) < 1e-12 * abs(D[i, i])
    h = 1.0 / (n + 1)
    assert abs(B.to_dense()[i].sum() - h ** 3) < 1e-15


def test_kappa_range():
    u = wl.uniform(wl.SEED_KAPPA, np.arange(1000, dtype=np.uint64))
    k = 10.0 ** (-1 + 2 * u)
    assert k.min() >= 0.1 and k.max() <= 10.0


def test_diag_b_range():
    d = wl.diag_uniform(5000)
    assert d.min() >= 0.5 and d.max() < 1.5


def test_fd_sample_distinct():
    A = wl.varcoef3d_7pt(4)
    s = wl.fd_sample(A, 20)
    assert len(set(s.tolist())) == 20 and s.min() >= 0 and s.max() < A.nnz
