"""The C-ABI library loads, exports every symbol include/gcge.h declares, and
its host-only logic (dense Rayleigh-Ritz eigensolver, STEP 5 coefficients,
argument checking) agrees with the oracle.  No GPU is touched."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as orc
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gcge.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2111_06552_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2111_06552_amd import build
        build.build()
    return _lib.load()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gcge_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_list():
    from paper_2111_06552_amd import _lib
    assert declared_symbols() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(os.path.join(ROOT, "paper_2111_06552_amd", "libgcge.so"))
    for name in declared_symbols():
        assert hasattr(raw, name), name


@pytest.mark.parametrize("n", [0, 1, 2, 5, 64, 200])
def test_host_small_eigh_matches_oracle(lib, n):
    import paper_2111_06552_amd as g
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n))
    M = M + M.T
    if n == 0:
        w, Z = g.small_eigh(np.zeros((0, 0)), 0)
        assert w.shape == (0,)
        return
    w, Z = g.small_eigh(M, n)
    w2, _ = orc.jacobi_eigh(M)
    assert np.max(np.abs(w - w2)) < 1e-13 * max(1.0, np.abs(w2).max()) * max(1, n) ** 0.5
    assert np.max(np.abs(M @ Z - Z * w)) < 1e-12 * max(1.0, np.abs(w2).max())
    assert np.max(np.abs(Z.T @ Z - np.eye(n))) < 1e-13


def test_host_small_eigh_clustered_spectrum(lib):
    import paper_2111_06552_amd as g
    A = wl.laplace2d_5pt(12).to_dense()      # multiplicity-2 eigenvalues
    w, Z = g.small_eigh(A, 30)
    w2, _ = orc.jacobi_eigh(A)
    assert np.max(np.abs(w - w2) / w2) < 1e-13
    assert np.max(np.abs(Z.T @ Z - np.eye(30))) < 1e-13
    assert np.max(np.abs(A @ Z - Z * w[:30])) < 1e-11 * w2.max()


def test_host_p_hat_matches_oracle(lib):
    import paper_2111_06552_amd as g
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    for nx, shift, n_old, n_new in [(25, 0, 5, 5), (25, 3, 5, 5), (30, 2, 6, 4), (40, 0, 5, 5)]:
        xh = Q[:, :nx]
        a = g.p_hat(xh, shift, n_old, n_new)
        b = orc.p_hat(xh, shift, n_old, n_new)
        assert a.shape == b.shape
        if a.size:
            assert np.max(np.abs(a - b)) < 1e-13


def test_invalid_arguments_return_codes_without_gpu(lib):
    from paper_2111_06552_amd import _lib
    h = ctypes.c_void_p()
    rc = lib.gcge_create(None, 0, None, 1, 1e-8, ctypes.byref(h))
    assert rc == _lib.GCGE_ERR_INVALID_ARG
    assert lib.gcge_last_error(None)
    assert lib.gcge_set_option_i(None, b"max_iter", 5) == _lib.GCGE_ERR_INVALID_ARG
    assert lib.gcge_small_eigh(-1, None, None, None, 0) == _lib.GCGE_ERR_INVALID_ARG
    assert lib.gcge_spmm(None, None, 0, 0, None, 0, None) == _lib.GCGE_ERR_INVALID_ARG
    lib.gcge_destroy(None)
    amg = ctypes.c_void_p()
    assert lib.gcge_amg_create(None, 10, 512, 0.02, None, ctypes.byref(amg)) == _lib.GCGE_ERR_INVALID_ARG
    assert not amg.value
    assert lib.gcge_amg_apply(None, None, 0, 1, None, 0, None) == _lib.GCGE_ERR_INVALID_ARG
    nl = ctypes.c_int(0)
    assert lib.gcge_amg_levels(None, ctypes.byref(nl), None, None, 0) == _lib.GCGE_ERR_INVALID_ARG
    assert lib.gcge_pcg(None, None, None, 0, 1, 30, 1e-2, None, 0, None, None) == _lib.GCGE_ERR_INVALID_ARG
    lib.gcge_amg_destroy(None)


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2111_06552_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dp, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f


def test_host_p_hat_hand_derived(lib):
    """The library's STEP 5 coefficients on the hand-derived case of eq.
    CP_tilde (see tests/test_oracle_pins.py): phat = (-2,0,1,1,0)/sqrt6."""
    import paper_2111_06552_amd as g
    a = np.array([1.0, 0.0, 1.0, 1.0, 0.0]) / np.sqrt(3.0)
    b = np.array([0.0, 1.0, 0.0, 0.0, 1.0]) / np.sqrt(2.0)
    ph = g.p_hat(np.stack([a, b], axis=1), 0, 1, 1)
    ref = np.array([-2.0, 0.0, 1.0, 1.0, 0.0]) / np.sqrt(6.0)
    assert ph.shape == (5, 1)
    assert np.max(np.abs(np.sign(ph[:, 0] @ ref) * ph[:, 0] - ref)) < 1e-14
    assert g.p_hat(np.stack([a, b], axis=1), 1, 1, 1).shape[1] == 0
