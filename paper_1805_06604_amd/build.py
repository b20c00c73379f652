"""Compile the HIP sources of the package into libnmf.so for gfx950.

All device code is built for gfx950 only. Packed FP32 instructions are
disabled at the target-feature level (the compiler would otherwise form them
from ordinary float code).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnmf.so")
SOURCES = ["sweep_rp64.hip", "sweep_rp48.hip", "sweep_rp32.hip", "sweep_rp16.hip",
           "prod_i8.hip", "prod_x16.hip", "prod_csr.hip",
           "engine.hip", "batch.hip", "noalloc.hip", "kernels_sweep.hip", "kernels_dense.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def compile_flags():
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"),
            "-I", CSRC]


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile each source to an object in parallel, then link the library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC] + compile_flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    if p.wait() != 0:
        raise RuntimeError(f"hipcc failed on {src}")


if __name__ == "__main__":
    print(build(verbose=True))
