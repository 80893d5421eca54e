"""Build libfetdpic.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfetdpic.so")
BUILD = os.path.join(ROOT, "_build")
# (source, object name, extra flags).  The particle kernels are built once
# per precision: FP32 with the compiler's default contraction, FP64 and the
# field kernels with contraction off (each FP64 update is the plain
# sequence of rounded operations of its definition).
SOURCES = [
    ("fetd_kernels.hip", "fetd_kernels", ["-ffp-contract=off"]),
    ("fetd_particles.hip", "fetd_particles_f32", ["-DFETD_REAL=float", "-DFETD_REAL_IS_DOUBLE=0"]),
    ("fetd_particles.hip", "fetd_particles_f64",
     ["-DFETD_REAL=double", "-DFETD_REAL_IS_DOUBLE=1", "-ffp-contract=off"]),
    ("fetd_host.cpp", "fetd_host", []),
    ("fetd_sparse.cpp", "fetd_sparse", []),
    ("fetd3_kernels.hip", "fetd3_kernels", []),
    ("fetd3_host.cpp", "fetd3_host", []),
]
ARCH = os.environ.get("FETD_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()

    def compile_one(item):
        src, name, extra = item
        obj = os.path.join(BUILD, name + ".o")
        cmd = [cc, *flags(), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with cf.ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
