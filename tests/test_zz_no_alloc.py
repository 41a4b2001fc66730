"""The entry point that allocates nothing (gcge_gram_noalloc: partial tiles in
the library's fixed device array, result in a caller-owned device buffer)
against gcge_gram, through the C ABI: two calls in a row on one device (the
second smaller, so the array holds the first call's partials when it starts),
each checked element by element against gcge_gram and the oracle's Gram."""
import numpy as np
import pytest

import oracle as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_06552_amd as gg
    gg._lib.load()
    return gg


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _check(g, X, Y, d):
    Xd, Yd = dev(X), dev(Y)
    dd = None if d is None else dev(d)
    print(f"gram_noalloc n={X.shape[0]} m={X.shape[1]} k={Y.shape[1]} d={'yes' if d is not None else 'no'}",
          flush=True)
    C = g.gram_noalloc(Xd, Yd, dd)
    torch.cuda.synchronize()
    C = C.cpu().numpy()
    ref_lib = g.gram(Xd, Yd, dd)
    ref = orc.gram(X, Y, d)
    bound = orc.gram(np.abs(X), np.abs(Y), d)
    assert np.all(np.abs(C - ref) <= 1e-13 * bound + 1e-300)
    assert np.all(np.abs(C - ref_lib) <= 1e-13 * bound + 1e-300)
    return C


@pytest.mark.parametrize("shapes", [
    [(200_000, 64, 50), (20_000, 50, 50)],     # 64 x 64 MFMA tiles, then fewer rows
    [(300_000, 400, 50), (7_001, 13, 5)],      # several row tiles, then the 16 x 16 kernel
    [(50_000, 32, 32), (4_099, 17, 5)],        # the 32 x 32 kernel, then a ragged tail
])
def test_noalloc_gram_matches_gcge_gram_on_two_calls(g, shapes):
    rng = np.random.default_rng(11)
    for (n, m, k) in shapes:
        X = rng.standard_normal((n, m))
        Y = rng.standard_normal((n, k))
        d = rng.uniform(0.5, 1.5, n)
        _check(g, X, Y, None)
        _check(g, X, Y, d)


def test_noalloc_gram_repeated_calls_are_reproducible(g):
    rng = np.random.default_rng(12)
    X = dev(rng.standard_normal((100_000, 50)))
    Y = dev(rng.standard_normal((100_000, 50)))
    a = g.gram_noalloc(X, Y).cpu().numpy()
    b = g.gram_noalloc(X, Y).cpu().numpy()
    assert np.array_equal(a, b)


def test_noalloc_gram_edge_cases(g):
    from paper_2111_06552_amd import _lib
    # zero rows: C = 0, written by a kernel
    X = torch.zeros((0, 5), dtype=torch.float64, device="cuda")
    Y = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    C = torch.full((5, 3), 7.0, dtype=torch.float64, device="cuda")
    g.gram_noalloc(X, Y, None, C)
    assert torch.count_nonzero(C).item() == 0
    # beyond the maximum: the row tiles of X exceed what the kernels take
    Xb = torch.zeros((64, 3073), dtype=torch.float64, device="cuda")
    Yb = torch.zeros((64, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.GcgeError) as ei:
        g.gram_noalloc(Xb, Yb)
    assert ei.value.code == _lib.GCGE_ERR_INVALID_ARG
    # one chunk of partial tiles larger than the scratch array: 48 x 24 tiles of 32 KiB = 36 MiB
    Xc = torch.zeros((64, 3072), dtype=torch.float64, device="cuda")
    Yc = torch.zeros((64, 1536), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.GcgeError) as ei:
        g.gram_noalloc(Xc, Yc)
    assert ei.value.code == _lib.GCGE_ERR_INVALID_ARG
    assert "scratch" in str(ei.value)
