"""Build libgcge.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgcge.so")

SOURCES = ["kernels.hip", "eig.hip", "noalloc.hip", "operator.cpp", "solver.cpp", "dense.cpp", "amg.cpp"]
ARCH = os.environ.get("GCGE_OFFLOAD_ARCH", "gfx950")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _omp_rpath():
    for d in ("/opt/rocm/lib/llvm/lib", "/opt/rocm/llvm/lib"):
        if os.path.exists(os.path.join(d, "libomp.so")):
            return d
    return None


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 and link libgcge.so; returns its path."""
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-result",
              "-Wno-unused-command-line-argument"]
    objs = []

    def compile_one(src):
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        if src.endswith(".hip"):
            cmd = [hipcc, f"--offload-arch={ARCH}", "-x", "hip", *common,
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-c", path, "-o", obj]
        else:
            cmd = [hipcc, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", *common, "-fopenmp", "-c", path, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-fopenmp", "-o", tmp, *objs]
    rp = _omp_rpath()
    if rp:
        link += [f"-Wl,-rpath,{rp}"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(link)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
