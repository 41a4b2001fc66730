"""Write the block Lanczos oracle's results for the workload generators on
grids where the GPU tests need reference eigenvalues (and, for the
differentiation workload, reference gradients) but the oracle takes minutes.

The problem is the definition of Section 2: the nev smallest eigenpairs of
A x = lambda B x.  Every value here comes from ``oracle/`` (block Lanczos with
full reorthogonalization on A^{-1} B, explicit relative residuals at most
1e-12 or the rounding floor of a stored vector) applied to inputs from
``workloads``; nothing comes from the GPU
library.  Usage (from the repository root, several minutes on 8 cores):

    python tests/golden/make_lanczos_golden.py [name ...]

Names: lap3d_diagB_32, lap3d_diagB_48, varcoef_64.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as orc  # noqa: E402
import workloads as wl  # noqa: E402
from oracle.lanczos import lanczos_eigs  # noqa: E402

# which stored nonzeros the gradient comparison samples (besides the 20 of the
# finite-difference check): draws of its own SplitMix64 stream
SEED_GRAD_SAMPLE = 57
GRAD_SAMPLE = 2000


def _header(f, lines):
    for ln in lines:
        f.write("# " + ln + "\n")


def lap3d_diagB(grid):
    A = wl.laplace3d_7pt(grid)
    d = wl.diag_uniform(A.n)
    nev = 200
    lam, X, info = lanczos_eigs(A, "diag", d, nev, verbose=True)
    rel = orc.relative_residuals(A, "diag", d, X, lam)
    path = os.path.join(HERE, f"lanczos_lap3d_7pt_diagB_{grid}.txt")
    with open(path, "w") as f:
        _header(f, [
            f"nev = {nev} smallest eigenvalues of A x = lambda D x (Section 2, the eigenvalue problem)",
            f"A: 3D seven-point Laplacian on a {grid}^3 interior grid, h = 1/{grid + 1} "
            f"(workloads.laplace3d_7pt({grid})), n = {A.n}, nnz = {A.nnz}",
            f"D: diagonal 0.5 + U[0,1) keyed by row, seed {wl.SEED_DIAG_B} (workloads.diag_uniform)",
            "oracle: oracle.lanczos.lanczos_eigs (block 8, seed 1; explicit relative residuals at most 1e-12 or the "
            "rounding floor of a stored vector, whichever is larger)",
            f"Lanczos steps {info['steps']}, Krylov dimension {info['dim']}, CG iterations "
            f"{info['cg_iterations']}, max relative residual {rel.max():.3e} (largest gate "
            f"{info['max_gate']:.3e}), {info['seconds']:.0f} s",
            "written by tests/golden/make_lanczos_golden.py",
            "one eigenvalue per line, ascending",
        ])
        for v in lam:
            f.write(f"{v:.17e}\n")
    print(f"wrote {path}: {info}", flush=True)


def varcoef(grid):
    A = wl.varcoef3d_7pt(grid)
    nev = 50
    lam, X, info = lanczos_eigs(A, "identity", None, nev, verbose=True)
    rel = orc.relative_residuals(A, "identity", None, X, lam)
    w = wl.loss_weights(nev)
    gA = orc.eig_grad(A, X, lam, w)
    fd = wl.fd_sample(A)
    extra = wl.fd_sample(A, count=GRAD_SAMPLE, seed=SEED_GRAD_SAMPLE)
    idx = np.concatenate([fd, extra[~np.isin(extra, fd)]])
    gap = np.min(np.diff(lam)) / lam[-1]
    path = os.path.join(HERE, f"lanczos_varcoef3d_7pt_{grid}.txt")
    with open(path, "w") as f:
        _header(f, [
            f"nev = {nev} smallest eigenvalues of A x = lambda x (Section 2) and the gradient of "
            "L = sum_i w_i lambda_i with respect to sampled stored nonzeros of A",
            f"A: 3D seven-point operator with per-edge conductances 0.5 + 1.5 U (seed {wl.SEED_EDGE}) on a "
            f"{grid}^3 interior grid (workloads.varcoef3d_7pt({grid})), n = {A.n}, nnz = {A.nnz}",
            f"w_i ~ N(0,1), seed {wl.SEED_LOSS} (workloads.loss_weights); gradient dL/da_e = "
            "sum_i w_i x_i[row_e] x_i[col_e] (oracle.eig_grad) on the oracle's eigenvectors",
            f"sampled entries: the 20 of workloads.fd_sample (seed {wl.SEED_FD_SAMPLE}), then up to "
            f"{GRAD_SAMPLE} of fd_sample(count={GRAD_SAMPLE}, seed={SEED_GRAD_SAMPLE})",
            "oracle: oracle.lanczos.lanczos_eigs (block 8, seed 1; explicit relative residuals at most 1e-12 or the "
            "rounding floor of a stored vector, whichever is larger)",
            f"Lanczos steps {info['steps']}, Krylov dimension {info['dim']}, CG iterations "
            f"{info['cg_iterations']}, max relative residual {rel.max():.3e} (largest gate "
            f"{info['max_gate']:.3e}), smallest relative gap {gap:.3e}, {info['seconds']:.0f} s",
            "written by tests/golden/make_lanczos_golden.py",
            f"first {nev} data lines: eigenvalues ascending; then 'entry gradient' lines",
        ])
        for v in lam:
            f.write(f"{v:.17e}\n")
        for e in idx:
            f.write(f"{int(e)} {gA[e]:.17e}\n")
    print(f"wrote {path}: {info}", flush=True)


JOBS = {
    "lap3d_diagB_32": lambda: lap3d_diagB(32),
    "lap3d_diagB_48": lambda: lap3d_diagB(48),
    "varcoef_64": lambda: varcoef(64),
}


def main(argv):
    names = argv or list(JOBS)
    for nm in names:
        t0 = time.time()
        JOBS[nm]()
        print(f"{nm}: {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
