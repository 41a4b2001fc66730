#!/usr/bin/env python
"""Benchmark of the GCG eigensolver on one MI355X.

A step is one complete solve (gcge_solve: all steps of Algorithm 1 until the
nev smallest eigenpairs reach the relative residual tolerance) on the 128^3
seven-point Laplacian with a random diagonal B (nev = 200, blockSize = 50,
tol 1e-8).  The headline value is the FP64 time to solution; the same solve
with the FP32 inner CG is reported beside it.  Inputs are generated and
uploaded before the timed region.

Prints one JSON line.  Fields beyond the required ones:
  mixed         the FP32-inner-CG solve: time, speedup and eigenvalue agreement
  solve         iteration counts, residual and B-orthonormality of the FP64 solve
  roofline      the dominant kernel's achieved rate from HIP-event timings of
                every launch of one instrumented solve run after the timed
                ones (the timed solves carry no instrumentation); HBM rates are
                also given as a fraction of a copy measured on the same GPU
  cpu_baseline  the CPU oracle (block Lanczos) solving the same generator on a
                reduced grid on the host cores, with the GPU solve of that very
                input timed beside it
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to nev eigenpairs @ resid 1e-8, FP64 vs mixed; SpMM/CG HBM GB/s"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def row_kernel(base, s, k, tail=""):
    """Name of the row-group SpMM instance launched for k columns of s-byte
    scalars (16-byte accesses: V = 16 / s scalars per lane, G lanes per row)."""
    v = 16 // s
    lanes = (k + v - 1) // v
    g = next(x for x in (4, 8, 16, 32, 64) if lanes <= x)
    return f"{base}<{'double' if s == 8 else 'float'}, {g}, {v}{tail}>"


def flat_kernel(base, s, tail=""):
    """Name of a flat CG update kernel instance for s-byte scalars."""
    return f"{base}<{'double' if s == 8 else 'float'}, {16 // s}{tail}>"


def class_roofline(name, p, n, nnz, s=8, bs=None, lazy=False):
    """Achieved rate of one kernel class from its HIP-event timings.

    Algorithmic bytes per launch with k columns (s bytes per scalar):
      CG SpMM        nnz (4 + s) + 4 (n + 1) + 2 n k s   (CSR once, p gathered once, q written once)
      CG r update    3 n k s                              (q, r read; r written)
      CG x, p update 5 n k s                              (x, p, r read; x, p written)
        with the search-direction history (lazy): p update 3 n k s (p, r read; new p written)
      CG iterate     n s c                                (c = the launch's column count: the
                     from the history                     terms and x, times k)
    For the CG classes only the launches over a full block (k = bs columns, one
    kernel instance) are used.  Flops per launch of the GEMMs and Grams with
    m x k coefficient blocks: 2 n m k."""
    if p["launches"] == 0 or p["ms"] <= 0:
        return None
    avg_ms = p["ms"] / p["launches"]
    k = p["columns"] / p["launches"]
    launches = p["launches"]
    if bs is not None and p.get("full_launches"):
        avg_ms = p["full_ms"] / p["full_launches"]
        k = bs
        launches = p["full_launches"]
    kr = round(k)
    hbm = {"cg_spmm": lambda: (nnz * (4 + s) + 4 * (n + 1) + 2 * n * k * s,
                               row_kernel("k_spmms", s, kr, ", 0, 2") + " (CG: q = (A - theta B) p with p.q)"),
           "cg_update_r": lambda: (3 * n * k * s, flat_kernel("k_cg_update_r_pk", s, ", 4") + " (CG: r -= alpha q, r.r)"),
           "cg_update_xp": lambda: ((3 * n * k * s, flat_kernel("k_cg_update_p_flat", s)
                                     + " (CG: p_new = r + beta p, search-direction history)") if lazy else
                                    (5 * n * k * s, flat_kernel("k_cg_update_xp_flat", s)
                                     + " (CG: x += alpha p, p = r + beta p)")),
           "cg_fold": lambda: (n * s * p["columns"] / p["launches"],
                               flat_kernel("k_cg_fold", s) + " (CG: x = sum_i alpha_i p_i from the history)")}
    if name in hbm:
        per_launch, kern = hbm[name]()
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        return {"kernel": kern, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes_per_launch": per_launch,
                "avg_launch_ms": avg_ms, "launches": launches,
                "avg_launch_ms_all_widths": p["ms"] / p["launches"], "launches_all_widths": p["launches"]}
    if name == "amg_vcycle":   # several kernels per application: time only
        return {"kernel": "multigrid V-cycle (all levels, one application)", "bound": None,
                "avg_launch_ms": p["ms"] / p["launches"], "launches": p["launches"],
                "columns_per_launch": p["columns"] / p["launches"]}
    kern = {"rotation_gemm": "k_gemm (Ritz rotation V_u xhat)", "p_gemm": "k_gemm (P block V_u phat)",
            "gram": "k_gram_lds + k_tile_reduce (Gram products)"}[name]
    per_launch = 2.0 * n * k
    achieved = per_launch / (avg_ms * 1e-3) / 1e12
    return {"kernel": kern, "bound": "mfma", "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "traffic": None,
            "algorithmic_flops_per_launch": per_launch, "avg_launch_ms": avg_ms, "launches": p["launches"]}


def cg_iteration_roofline(kr, lazy=False):
    """One full-block CG iteration (its three kernels) as one HBM-bound step:
    the sum of their algorithmic bytes over the sum of their average
    full-block launch times.  With the search-direction history the third
    kernel is the p update alone; the iterate, formed once per CG solve, is
    the class cg_fold."""
    parts = [kr.get(c) for c in ("cg_spmm", "cg_update_r", "cg_update_xp")]
    if any(p is None for p in parts):
        return None
    b = sum(p["algorithmic_bytes_per_launch"] for p in parts)
    ms = sum(p["avg_launch_ms"] for p in parts)
    achieved = b / (ms * 1e-3) / 1e9
    return {"kernels": "SpMM + r update + " + ("p update" if lazy else "x/p update"), "bound": "hbm",
            "algorithmic_bytes": b, "ms": ms, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS}


def dominant_roofline(prof, n, nnz, s=8, bs=None, lazy=False):
    """Roofline entry of the kernel class with the largest summed device time."""
    name = max(prof, key=lambda c: prof[c]["ms"])
    return class_roofline(name, prof[name], n, nnz, s, bs, lazy), name


def uses_history(prof):
    """True when the CG formed its iterates from the search-direction history."""
    return prof.get("cg_fold", {}).get("launches", 0) > 0


def sum_prof(stats):
    """Per-class HIP-event totals over several solves."""
    out = {}
    for c in stats[0]["prof"]:
        if c.startswith("unused"):
            continue
        out[c] = {f: sum(x["prof"][c][f] for x in stats) for f in stats[0]["prof"][c]}
    return out


def spmm_extrapolation(A, spmm_columns, budget_s):
    """Oracle SpMM on the full operator, timed on a sample of columns and
    scaled to the number of columns the GPU solve pushed through sparse
    products (the solve's dominant work; Gram, orthogonalization and the dense
    eigensolves are not included, so this underestimates the CPU time)."""
    import numpy as np

    import oracle as orc
    rng = np.random.default_rng(0)
    k = 8
    X = rng.standard_normal((A.n, k))
    t0 = time.perf_counter()
    reps = 0
    while True:
        orc.spmm(A, X)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= 20:
            break
    per_col = el / (reps * k)
    return {"value": per_col * spmm_columns, "unit": "s", "cores": 1,
            "sample": f"oracle.spmm (numpy, one thread) of the full operator on {k} columns x {reps} repetitions "
                      f"({el:.1f} s), scaled to the {spmm_columns} SpMM columns of the FP64 GPU solve; "
                      f"excludes the orthogonalization and Rayleigh-Ritz work"}


def host_threads():
    """Threads the oracle's OpenMP code runs with."""
    v = os.environ.get("OMP_NUM_THREADS")
    try:
        return int(v) if v else (os.cpu_count() or 1)
    except ValueError:
        return os.cpu_count() or 1


def cpu_baseline(g, workload, grid, dev):
    """The oracle solving the benchmark's generator on a reduced grid (the
    block Lanczos reference eigensolver on the host cores, all nev pairs to an
    explicit relative residual of 1e-12 or its rounding floor), and the GPU
    solver on that same input in the benchmark's configuration."""
    import numpy as np
    import torch

    import workloads as wl
    from oracle.lanczos import lanczos_eigs
    A, bkind, B, p = wl.build_workload(workload, grid)
    nev, bs, tol = p["nev"], p["block_size"], p["tol"]
    t0 = time.perf_counter()
    lam_o, _, info = lanczos_eigs(A, bkind, B, nev)
    cpu_s = time.perf_counter() - t0
    Ad = g.DeviceCsr.from_csr(A, dev)
    Bd = None
    if bkind == "diag":
        Bd = torch.as_tensor(B, dtype=torch.float64, device=dev)
    elif bkind == "csr":
        Bd = g.DeviceCsr.from_csr(B, dev)
    with g.Solver(Ad, Bd, nev, tol, block_size=bs, moving=int(p["moving"])) as s:
        s.solve()                      # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        lam, _, st = s.solve()
        torch.cuda.synchronize()
        gpu_s = time.perf_counter() - t
    err = float(np.max(np.abs(lam.numpy() - lam_o) / np.abs(lam_o)))
    return {"value": cpu_s, "unit": "s", "cores": host_threads(), "kind": "oracle",
            "sample": f"oracle.lanczos.lanczos_eigs (block Lanczos, OpenMP CSR products and CG) solving the "
                      f"{workload} generator on a {grid}^3 grid (n = {A.n}), all {nev} pairs; "
                      f"{info['steps']} Lanczos steps, {info['cg_iterations']} CG iterations",
            "gpu_same_input_s": gpu_s, "gpu_speedup": cpu_s / gpu_s, "gpu_iterations": st["iterations"],
            "max_eig_rel_diff_gpu_vs_oracle": err}


def copy_peak_gbs(dev, nbytes=1 << 30, reps=10):
    """HBM rate of a plain device copy (bytes read + bytes written per second)."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        dst.copy_(src)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def add_measured_peak(entry, copy_gbs):
    if entry is not None and entry.get("bound") == "hbm" and copy_gbs:
        entry["peak_measured_copy"] = copy_gbs
        entry["frac_of_measured_copy"] = entry["achieved"] / copy_gbs
    return entry


KERNEL_SOURCE = os.path.join(ROOT, "paper_2111_06552_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "kernel_traffic.json")


def short_name(kernel_name):
    """'void gcge::k_x<double, 32, 2>(long, ...)' -> 'k_x<double, 32, 2>'."""
    n = kernel_name.replace("(anonymous namespace)::", "").split("(")[0]
    for pre in ("void ", "gcge::"):
        n = n.replace(pre, "")
    return n.strip()


def kernel_source_hash():
    """SHA-256 of the kernel source with comments and blank lines removed, so
    that counters stay attached to the code they were taken on, not to its
    comments."""
    import hashlib
    import re
    with open(KERNEL_SOURCE) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
    code = "\n".join(ln for ln in lines if ln.strip())
    return hashlib.sha256(code.encode()).hexdigest()


def summarize_trace(d, top=30):
    """Markdown table of a rocprofv3 --stats kernel summary (directory d)."""
    import csv
    import glob
    f = sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True))[-1]
    rows = list(csv.DictReader(open(f)))
    lines = ["| kernel | calls | total ms | average us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {r['Percentage']} |")
    return "\n".join(lines)


def pmc_means(d, counter):
    """Median counter value per dispatch and kernel of a rocprofv3 --pmc run
    (directory d); the median is the value of the most common launch shape
    (for the CG kernels: launches over a full block)."""
    import csv
    import glob
    f = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))[-1]
    acc = {}
    for r in csv.DictReader(open(f)):
        if r["Counter_Name"] != counter:
            continue
        acc.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    out = {}
    for k, v in acc.items():
        v.sort()
        out[k] = v[len(v) // 2]
    return out


def summarize_gaps(d, min_gap_us=20.0, top=8):
    """Markdown summary of the idle time between kernels in a rocprofv3
    --kernel-trace run (directory d): busy fraction of the traced span and the
    gaps longer than min_gap_us, grouped by the kernel pair around them."""
    import csv
    import glob
    f = sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True))[-1]
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"]))
                for r in csv.DictReader(open(f)))
    t0, t1 = iv[0][0], max(b for _, b, _ in iv)
    end, busy, prev = iv[0][1], iv[0][1] - iv[0][0], iv[0][2]
    gap_ns, gap_n = {}, {}
    for a, b, nm in iv[1:]:
        if a - end > min_gap_us * 1e3:
            key = f"`{prev}` → `{nm}`"
            gap_ns[key] = gap_ns.get(key, 0) + (a - end)
            gap_n[key] = gap_n.get(key, 0) + 1
        busy += max(0, b - max(a, end))
        end = max(end, b)
        prev = nm
    lines = [f"traced span {(t1 - t0) / 1e6:.1f} ms, kernels busy {busy / 1e6:.1f} ms "
             f"({100.0 * busy / (t1 - t0):.1f} %), {len(iv)} dispatches; "
             f"gaps over {min_gap_us:g} us: {sum(gap_ns.values()) / 1e6:.1f} ms in {sum(gap_n.values())}", "",
             "| before → after | gaps | total ms | average us |", "|---|---:|---:|---:|"]
    for k in sorted(gap_ns, key=lambda k: -gap_ns[k])[:top]:
        lines.append(f"| {k} | {gap_n[k]} | {gap_ns[k] / 1e6:.1f} | {gap_ns[k] / gap_n[k] / 1e3:.1f} |")
    return "\n".join(lines)


def summarize_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes):
    """HBM bytes per dispatch from FETCH_SIZE and WRITE_SIZE runs (KiB per dispatch),
    each scaled by what the counter reads for a plain streaming kernel that reads and
    writes copy_bytes."""
    cf = max(pmc_means(copy_fetch_dir, "FETCH_SIZE").values())
    cw = max(pmc_means(copy_write_dir, "WRITE_SIZE").values())
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    fe, wr = pmc_means(fetch_dir, "FETCH_SIZE"), pmc_means(write_dir, "WRITE_SIZE")
    out = {"kernels_hip_sha256": kernel_source_hash(), "fetch_scale": f_scale, "write_scale": w_scale,
           "bytes_per_dispatch": {k: fe[k] * 1024.0 * f_scale + wr.get(k, 0.0) * 1024.0 * w_scale for k in fe},
           "fetch_bytes_per_dispatch": {k: fe[k] * 1024.0 * f_scale for k in fe},
           "write_bytes_per_dispatch": {k: wr[k] * 1024.0 * w_scale for k in wr}}
    return out


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when
    there is none or the kernel source changed after the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernels_hip_sha256") != kernel_source_hash():
        return None
    return t["bytes_per_dispatch"].get(short_name(kernel.split(" (")[0]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lap3d_7pt_128_diagB")
    ap.add_argument("--grid", type=int, default=None)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cg-max-iter", type=int, default=30, help="inner CG iterations per GCG iteration (cap)")
    ap.add_argument("--cg-rel-tol", type=float, default=1e-2,
                    help="inner CG stop at this relative residual (0: always cg-max-iter iterations)")
    ap.add_argument("--shift", type=int, choices=(0, 1), default=1,
                    help="1: inner CG on A - theta B with theta the largest converged eigenvalue; 0: theta = 0")
    ap.add_argument("--precond", type=int, choices=(0, 1), default=0,
                    help="1: STEP 6 as CG preconditioned by the algebraic multigrid V-cycle at theta = 0 "
                         "(the mixed run uses FP32 PCG and V-cycle)")
    ap.add_argument("--orth", type=int, choices=(2, 3), default=3,
                    help="STEP 2 orthogonalization: 3 RecursiveOrthSVD (default), 2 modified block")
    ap.add_argument("--orth-skip-final", type=int, choices=(0, 1), default=0,
                    help="1: Algorithm 3's pass loops stop before the update of a pass that already "
                         "meets the tolerance (the paper's listing applies it)")
    ap.add_argument("--cg-history", type=int, default=32,
                    help="inner CG search-direction history slots (0: update the iterate in every step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-grid", type=int, default=32,
                    help="grid of the reduced input that the CPU oracle and the GPU both solve for cpu_baseline")
    ap.add_argument("--cpu-budget-s", type=float, default=5.0,
                    help="time spent on the SpMM sample of the extrapolated CPU figure")
    ap.add_argument("--summarize-trace", metavar="DIR", help="print a markdown table of a rocprofv3 --stats run")
    ap.add_argument("--summarize-gaps", metavar="DIR",
                    help="print the busy fraction and the idle gaps between kernels of a rocprofv3 --kernel-trace run")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                            "COPY_WRITE_DIR"),
                    help="write the per-kernel HBM traffic of rocprofv3 --pmc runs to profiles/kernel_traffic.json")
    ap.add_argument("--copy-bytes", type=float, default=float(2 ** 30),
                    help="bytes read (and written) by each dispatch of the calibration copy")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return
    if args.summarize_gaps:
        print(summarize_gaps(args.summarize_gaps))
        return
    if args.summarize_traffic:
        t = summarize_traffic(*args.summarize_traffic, args.copy_bytes)
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(t, f, indent=1, sort_keys=True)
        print(json.dumps({k: t[k] for k in ("fetch_scale", "write_scale")}))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU row "
              f"partition is a design, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2111_06552_amd as g
    import workloads as wl

    g._lib.load()
    t0 = time.perf_counter()
    A, bkind, B, p = wl.build_workload(args.workload, args.grid)
    log(f"[bench] workload {args.workload} grid={p['grid']} n={A.n} nnz={A.nnz} built in {time.perf_counter()-t0:.1f}s")
    dev = torch.device("cuda:0")
    Ad = g.DeviceCsr.from_csr(A, dev)
    Bd = None
    if bkind == "diag":
        Bd = torch.as_tensor(B, dtype=torch.float64, device=dev)
    elif bkind == "csr":
        Bd = g.DeviceCsr.from_csr(B, dev)
    nev, bs, tol = p["nev"], p["block_size"], p["tol"]
    evecs = torch.empty((A.n, nev), dtype=torch.float64, device=dev)

    def run(prec, steps, warmup):
        """Timed solves without instrumentation, then one solve with every
        launch of the main kernel classes bracketed by HIP events."""
        opts = dict(block_size=bs, precision=prec, moving=int(p["moving"]), profile=0, orth=args.orth,
                    cg_max_iter=args.cg_max_iter, cg_rel_tol=args.cg_rel_tol, shift=args.shift,
                    precond=args.precond, orth_skip_final=args.orth_skip_final, cg_history=args.cg_history)
        with g.Solver(Ad, Bd, nev, tol, **opts) as s:
            for i in range(warmup):
                lam, _, st = s.solve(evecs)
                log(f"[bench] {prec} warmup {i}: {st['time_ms']['total']:.0f} ms, {st['iterations']} iterations")
            times, stats = [], []
            torch.cuda.synchronize()
            for i in range(steps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                lam, _, st = s.solve(evecs)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t)
                stats.append(st)
                log(f"[bench] {prec} step {i}: {times[-1]*1e3:.0f} ms, {st['iterations']} iterations, "
                    f"{st['cg_iterations']} CG iterations, max rel residual {st['max_rel_residual']:.2e}")
            s.set_options(profile=1)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, _, sp = s.solve(evecs)
            torch.cuda.synchronize()
            tp = time.perf_counter() - t
            log(f"[bench] {prec} instrumented solve: {tp*1e3:.0f} ms")
            return np.array(times), stats, lam.numpy().copy(), sp, tp

    copy_gbs = copy_peak_gbs(dev)
    log(f"[bench] plain device copy: {copy_gbs:.0f} GB/s")
    t64, s64, lam64, sp64, tp64 = run("fp64", args.steps, args.warmup)
    out = {
        "metric": METRIC, "value": float(t64.mean()), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": float(t64.mean() * 1e3), "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "grid": p["grid"], "n": A.n, "nnz": A.nnz, "nev": nev,
                   "block_size": bs, "tol": tol, "B": bkind, "moving": bool(p["moving"]),
                   "orthogonalization": ("Algorithm 3" if args.orth == 3 else "Algorithm 2")
                   + (", final sub-tolerance update skipped" if args.orth_skip_final else ""),
                   "cg_max_iter": args.cg_max_iter, "cg_rel_tol": args.cg_rel_tol, "shift": bool(args.shift),
                   "cg_history": args.cg_history,
                   "inner_preconditioner": "algebraic multigrid V-cycle (theta = 0)" if args.precond else None},
    }
    st = s64[-1]
    out["solve"] = {k: st[k] for k in ("iterations", "nconv", "moves", "cg_iterations", "spmm_columns",
                                       "max_rel_residual", "orth_error")}
    out["solve"]["step_ms"] = {k: round(v, 2) for k, v in st["time_ms"].items()}
    out["solve"]["times_s"] = [round(x, 4) for x in t64.tolist()]
    out["solve"]["instrumented_solve_s"] = round(tp64, 4)
    # rooflines from every launch of the instrumented solve
    prof = sum_prof([sp64])
    lazy = uses_history(prof)
    roof, name = dominant_roofline(prof, A.n, A.nnz, bs=bs, lazy=lazy)
    if roof is not None and roof.get("bound") == "hbm":
        roof["traffic"] = measured_traffic(roof["kernel"])
    out["roofline"] = add_measured_peak(roof, copy_gbs)
    out["kernel_rooflines"] = {c: add_measured_peak(class_roofline(c, prof[c], A.n, A.nnz, bs=bs, lazy=lazy),
                                                    copy_gbs)
                               for c in prof}
    out["kernel_ms_per_solve"] = {c: round(prof[c]["ms"], 2) for c in prof}
    out["cg_iteration_roofline"] = add_measured_peak(cg_iteration_roofline(out["kernel_rooflines"], lazy), copy_gbs)
    out["cg_search_direction_history"] = lazy
    out["copy_peak_gbs"] = copy_gbs
    if not args.no_mixed:
        tm, sm, lamm, spm, tpm = run("mixed", args.steps, args.warmup)
        out["mixed"] = {"value": float(tm.mean()), "unit": "s", "ms_per_step": float(tm.mean() * 1e3),
                        "speedup_vs_fp64": float(t64.mean() / tm.mean()),
                        "max_eig_rel_diff_vs_fp64": float(np.max(np.abs(lamm - lam64) / np.abs(lam64))),
                        "iterations": sm[-1]["iterations"], "cg_iterations": sm[-1]["cg_iterations"],
                        "max_rel_residual": sm[-1]["max_rel_residual"], "dtype": "f32 inner CG, f64 elsewhere"}
        profm = sum_prof([spm])
        lazym = uses_history(profm)
        out["mixed"]["kernel_rooflines"] = {
            c: add_measured_peak(class_roofline(c, profm[c], A.n, A.nnz, s=4, bs=bs, lazy=lazym), copy_gbs)
            for c in ("cg_spmm", "cg_update_r", "cg_update_xp", "cg_fold")}
        out["mixed"]["cg_iteration_roofline"] = add_measured_peak(
            cg_iteration_roofline(out["mixed"]["kernel_rooflines"], lazym), copy_gbs)
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle on the {args.cpu_grid}^3 grid, {host_threads()} threads")
        out["cpu_baseline"] = cpu_baseline(g, args.workload, args.cpu_grid, dev)
        log(f"[bench] cpu baseline: {out['cpu_baseline']['value']:.1f} s (GPU {out['cpu_baseline']['gpu_same_input_s']:.3f} s)")
        out["cpu_spmm_extrapolation"] = spmm_extrapolation(A, int(st["spmm_columns"]), args.cpu_budget_s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
