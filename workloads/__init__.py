"""Seeded synthetic inputs for the GCG eigensolver: sparse operators, random
draws and the five benchmark workloads.

This module holds input generation only. It contains none of the eigensolver's
arithmetic, so both the CPU oracle (``oracle/``) and the GPU product path
(``paper_2111_06552_amd``) may import it without sharing method code.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw number ``i`` of the stream seeded with ``s`` is
``mix64(s + (i + 1) * GAMMA)``.  Every entity (a matrix row, a mesh cell, an
edge, an entry of a block of vectors) is keyed by its own index, so the values
do not depend on the order in which they are generated.  A uniform double in
[0, 1) keeps the top 53 bits: ``(z >> 11) * 2**-53``.

Operators are returned as :class:`Csr` with int32 row pointers and column
indices (columns sorted and unique within each row) and float64 values.

The paper measures on SuiteSparse electronic-structure matrices and on finite
element Laplace matrices (Section 4, Table of test matrices); neither is
available here, so the stencil and trilinear finite element operators below
stand in for them: symmetric positive definite, 5 to 27 nonzeros per row and a
clustered low spectrum.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Seeds of the five workloads (one stream per random quantity).
SEED_DIAG_B = 2        # diagonal B of the 128^3 seven-point workload
SEED_KAPPA = 3         # per-cell coefficients of the trilinear FEM workload
SEED_EDGE = 5          # per-edge conductances of the differentiation workload
SEED_LOSS = 55         # loss weights w_i ~ N(0, 1)
SEED_FD_SAMPLE = 56    # which stored nonzeros the finite-difference check perturbs
SEED_SOLVER = 1        # initial block X0 of the solver


def mix64(z):
    """SplitMix64 output function applied to uint64 array ``z``."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, idx):
    """Draw number ``idx`` (array) of the SplitMix64 stream seeded with ``seed``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx + np.uint64(1)) * GAMMA
    return mix64(z)


def uniform(seed: int, idx):
    """Uniform doubles in [0, 1) keyed by (seed, idx)."""
    z = splitmix64(seed, idx)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, idx):
    """Standard normal doubles keyed by (seed, idx), by the Box-Muller transform
    of draws 2*idx and 2*idx+1."""
    idx = np.asarray(idx, dtype=np.uint64)
    u1 = uniform(seed, np.uint64(2) * idx)
    u2 = uniform(seed, np.uint64(2) * idx + np.uint64(1))
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)


def initial_block(seed: int, n: int, k: int, col0: int = 0) -> np.ndarray:
    """Random starting block (n x k, row-major) with entries uniform in [-1, 1).

    Entry (row, col) is draw ``col * n + row`` of the stream ``seed``; columns
    ``col0 .. col0+k-1`` are returned.
    """
    rows = np.arange(n, dtype=np.uint64)[:, None]
    cols = np.arange(col0, col0 + k, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        idx = cols * np.uint64(n) + rows
    return 2.0 * uniform(seed, idx) - 1.0


@dataclass
class Csr:
    """Square sparse matrix in compressed sparse row form."""
    n: int
    rowptr: np.ndarray   # int32[n+1]
    colind: np.ndarray   # int32[nnz]
    val: np.ndarray      # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.colind.shape[0])

    def row_of_entry(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.rowptr))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        d[self.row_of_entry(), self.colind] = self.val
        return d

    def with_values(self, val: np.ndarray) -> "Csr":
        return Csr(self.n, self.rowptr, self.colind, np.ascontiguousarray(val, dtype=np.float64))


def _stencil_csr(shape, offsets, values) -> Csr:
    """Assemble a CSR matrix from a structured-grid stencil.

    ``shape`` is the node grid (x fastest in the row numbering), ``offsets`` a
    list of integer offset tuples (dx, dy, dz...) and ``values[k]`` an array of
    the grid's shape holding the coefficient that couples node p with node
    p + offsets[k].  Couplings that leave the grid are dropped (Dirichlet
    nodes).  Columns come out sorted because offsets are visited in order of
    their linear index offset.
    """
    dims = len(shape)
    n = int(np.prod(shape))
    strides = [int(np.prod(shape[:d])) for d in range(dims)]
    lin = [sum(o[d] * strides[d] for d in range(dims)) for o in offsets]
    order = np.argsort(lin, kind="stable")
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    # node coordinate arrays flattened in x-fastest order
    coords = [g.transpose(tuple(range(dims))[::-1]).reshape(-1) for g in grids]
    masks, vals, cols = [], [], []
    row_idx = np.arange(n, dtype=np.int64)
    for k in order:
        o = offsets[k]
        m = np.ones(n, dtype=bool)
        for d in range(dims):
            c = coords[d] + o[d]
            m &= (c >= 0) & (c < shape[d])
        v = np.asarray(values[k]).transpose(tuple(range(dims))[::-1]).reshape(-1)
        masks.append(m)
        vals.append(v)
        cols.append(row_idx + lin[k])
    mask = np.stack(masks, axis=1)                  # n x noff
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colmat = np.stack(cols, axis=1)
    valmat = np.stack(vals, axis=1)
    colind = colmat[mask].astype(np.int32)          # row-major boolean indexing keeps row order
    val = valmat[mask].astype(np.float64)
    return Csr(n, rowptr.astype(np.int32), colind, val)


def laplace2d_5pt(m: int) -> Csr:
    """Five-point finite-difference Laplacian on an m x m interior grid of the
    unit square, Dirichlet boundary, h = 1/(m+1): (1/h^2) * [4, -1 x 4]."""
    h2 = float(m + 1) ** 2
    shape = (m, m)
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    vals = [np.full(shape, 4.0 * h2)] + [np.full(shape, -h2)] * 4
    return _stencil_csr(shape, offs, vals)


def laplace3d_7pt(n: int) -> Csr:
    """Seven-point finite-difference Laplacian on an n^3 interior grid of the
    unit cube, Dirichlet boundary, h = 1/(n+1): (1/h^2) * [6, -1 x 6]."""
    h2 = float(n + 1) ** 2
    shape = (n, n, n)
    offs = [(0, 0, 0)] + [tuple(s if d == a else 0 for d in range(3)) for a in range(3) for s in (-1, 1)]
    vals = [np.full(shape, 6.0 * h2)] + [np.full(shape, -h2)] * 6
    return _stencil_csr(shape, offs, vals)


def diag_uniform(n: int, seed: int = SEED_DIAG_B) -> np.ndarray:
    """Diagonal of B with i.i.d. entries 0.5 + U[0,1) keyed by row."""
    return 0.5 + uniform(seed, np.arange(n, dtype=np.uint64))


def varcoef3d_7pt(n: int, seed: int = SEED_EDGE, constant: bool = False) -> Csr:
    """Seven-point operator with per-edge conductances on an n^3 interior grid,
    h = 1/(n+1): A = (1/h^2) * sum_e c_e (e_i - e_j)(e_i - e_j)^T over all grid
    edges, including the 6 n^2 edges that join a boundary node to a Dirichlet
    node (those add c_e / h^2 to the diagonal only).

    c_e = 0.5 + 1.5 U keyed by edge id; edge (axis a, lower-node coordinate
    p with p_a in [0, n], other coordinates in [1, n]) has id
    a * (n+1) * n^2 + linear index of p in the (n+1) x n x n grid ordered with
    axis a fastest.  ``constant=True`` sets c_e = 1 (the plain Laplacian).
    """
    h2 = float(n + 1) ** 2
    # cond[a] has shape (n+1, n, n) in (axis a, other1, other2) order, x fastest storage
    cond = []
    ne = (n + 1) * n * n
    for a in range(3):
        if constant:
            c = np.ones(ne)
        else:
            c = 0.5 + 1.5 * uniform(seed, np.arange(a * ne, (a + 1) * ne, dtype=np.uint64))
        cond.append(c)
    # Express per-node couplings: for node p (coords x,y,z in 0..n-1 meaning grid 1..n),
    # edge along axis a between p - e_a and p has lower coordinate p_a (0-based: p_a),
    # edge between p and p + e_a has lower coordinate p_a + 1.
    def edge_field(a, shift):
        # returns array shape (n, n, n) indexed [x, y, z] with the conductance of the
        # axis-a edge whose lower node has coordinate (node coord along a) + shift (1-based
        # lower coordinate = 0-based node coord + shift)
        c = cond[a]
        # storage: index = pa + (n+1) * (q1 + n * q2) where (q1, q2) are the other axes in
        # increasing axis order
        others = [d for d in range(3) if d != a]
        idx = np.indices((n, n, n))  # [3, x, y, z]
        pa = idx[a] + shift
        lin = pa + (n + 1) * (idx[others[0]] + n * idx[others[1]])
        return c[lin]
    diag = np.zeros((n, n, n))
    offs = [(0, 0, 0)]
    vals = [None]
    for a in range(3):
        lower = edge_field(a, 0)   # edge between node-1 and node (lower coord = node coord 0-based)
        upper = edge_field(a, 1)   # edge between node and node+1
        diag += lower + upper
        e = tuple(1 if d == a else 0 for d in range(3))
        em = tuple(-1 if d == a else 0 for d in range(3))
        offs.append(em)
        vals.append(-lower * h2)
        offs.append(e)
        vals.append(-upper * h2)
    vals[0] = diag * h2
    return _stencil_csr((n, n, n), offs, vals)


def q1_fem(n: int, seed: int = SEED_KAPPA, constant: bool = False):
    """Trilinear (Q1) finite elements on (n+1)^3 cubic cells of the unit cube,
    h = 1/(n+1), homogeneous Dirichlet boundary (n^3 interior nodes).

    Stiffness K_e = kappa_e * h * Khat and consistent mass M_e = h^3 * Mhat, where
    for two vertices of a cell at Hamming distance d (0..3):
    Khat = (1/12) * {4, 0, -1, -1} and Mhat = (1/216) * {8, 4, 2, 1}.
    kappa_e = 10^(-1 + 2U) keyed by the cell index (cells indexed by their lowest
    corner c in [0, n]^3, x fastest).  ``constant=True`` sets kappa = 1.

    Returns (A, B) with the same 27-point pattern (face-neighbour entries of A
    are stored, with value 0).
    """
    h = 1.0 / (n + 1)
    ncell = (n + 1) ** 3
    if constant:
        kap = np.ones(ncell)
    else:
        kap = 10.0 ** (-1.0 + 2.0 * uniform(seed, np.arange(ncell, dtype=np.uint64)))
    kap = kap.reshape(n + 1, n + 1, n + 1).transpose(2, 1, 0)  # [cx, cy, cz]
    khat = {0: 4.0 / 12.0, 1: 0.0, 2: -1.0 / 12.0, 3: -1.0 / 12.0}
    mhat = {0: 8.0 / 216.0, 1: 4.0 / 216.0, 2: 2.0 / 216.0, 3: 1.0 / 216.0}
    offs, avals, bvals = [], [], []
    for oz in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                o = (ox, oy, oz)
                d = sum(1 for t in o if t != 0)
                # sum of kappa over cells containing node p (1-based coords 1..n) and p+o:
                # along an axis with o_a = 0 the cell corner is p_a - 1 or p_a, otherwise min(p_a, p_a + o_a) - 0
                ksum = np.zeros((n, n, n))
                ncount = 0
                choices = []
                for a in range(3):
                    if o[a] == 0:
                        choices.append((-1, 0))
                    else:
                        choices.append((min(0, o[a]),))
                for sx in choices[0]:
                    for sy in choices[1]:
                        for sz in choices[2]:
                            # node p has 1-based coordinate i+1 for 0-based i; cell corner = p + s (1-based p) - ... corner index in [0, n]
                            # corner 0-based index along axis = (i + 1) + s - 0 - 1 + 1 => i + 1 + s
                            ksum += kap[1 + sx:1 + sx + n, 1 + sy:1 + sy + n, 1 + sz:1 + sz + n]
                            ncount += 1
                offs.append(o)
                avals.append(h * khat[d] * ksum)
                bvals.append(np.full((n, n, n), h ** 3 * mhat[d] * ncount))
    A = _stencil_csr((n, n, n), offs, avals)
    Bm = _stencil_csr((n, n, n), offs, bvals)
    return A, Bm


def fd_sample(A: Csr, count: int = 20, seed: int = SEED_FD_SAMPLE) -> np.ndarray:
    """Indices of ``count`` distinct stored nonzeros of A chosen by draws of the
    stream ``seed`` (draw i picks entry floor(U_i * nnz); repeats are skipped)."""
    picked, seen, i = [], set(), 0
    while len(picked) < count:
        e = int(np.floor(uniform(seed, np.uint64(i)) * A.nnz))
        i += 1
        if e not in seen:
            seen.add(e)
            picked.append(e)
    return np.array(picked, dtype=np.int64)


def loss_weights(nev: int, seed: int = SEED_LOSS) -> np.ndarray:
    """Loss weights w_i ~ N(0, 1), i = 0..nev-1."""
    return normal(seed, np.arange(nev, dtype=np.uint64))


# ---------------------------------------------------------------------------
# The five benchmark workloads.  ``scale`` shrinks the grid for quick runs.
# ---------------------------------------------------------------------------

WORKLOADS = {
    "lap2d_5pt_64": dict(desc="2D 5-point Laplacian 64x64, B=I, nev=10, bs=10, tol 1e-8, FP64",
                         grid=64, nev=10, block_size=10, tol=1e-8, precision="fp64", moving=False),
    "lap3d_7pt_128_diagB": dict(desc="3D 7-point Laplacian 128^3, random diagonal B, nev=200, bs=50, tol 1e-8, FP64",
                                grid=128, nev=200, block_size=50, tol=1e-8, precision="fp64", moving=False),
    "q1fem_96_moving": dict(desc="Q1 FEM 96^3 interior nodes, log-uniform kappa, consistent mass B, nev=1000, "
                                 "bs=100, moving mechanism, tol 1e-8, FP64",
                            grid=96, nev=1000, block_size=100, tol=1e-8, precision="fp64", moving=True),
    "lap3d_7pt_128_diagB_mixed": dict(desc="as lap3d_7pt_128_diagB with FP32 inner CG and FP32 CG SpMM",
                                      grid=128, nev=200, block_size=50, tol=1e-8, precision="mixed", moving=False),
    "varcoef3d_7pt_64_grad": dict(desc="3D 7-point variable-coefficient 64^3, B=I, nev=50, bs=10, eigenvalue "
                                       "gradients of sum w_i lambda_i", grid=64, nev=50, block_size=10, tol=1e-8,
                                  precision="fp64", moving=False),
}


def build_workload(name: str, grid: int | None = None):
    """Return (A, b_kind, B, params) for a named workload, optionally on a
    smaller grid.  b_kind is 'identity', 'diag' (B is a float64 vector) or
    'csr' (B is a Csr with the same pattern as A)."""
    p = dict(WORKLOADS[name])
    g = p["grid"] if grid is None else grid
    p["grid"] = g
    if name == "lap2d_5pt_64":
        return laplace2d_5pt(g), "identity", None, p
    if name.startswith("lap3d_7pt_128_diagB"):
        A = laplace3d_7pt(g)
        return A, "diag", diag_uniform(A.n), p
    if name == "q1fem_96_moving":
        A, B = q1_fem(g)
        return A, "csr", B, p
    if name == "varcoef3d_7pt_64_grad":
        return varcoef3d_7pt(g), "identity", None, p
    raise KeyError(name)
