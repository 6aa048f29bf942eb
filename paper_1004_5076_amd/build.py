"""Build libscabs.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libscabs.so")
SOURCES = ["setup.cpp", "toeplitz.cpp", "postproc.cpp", "kernels_fft.hip", "kernels_toeplitz.hip", "kernels_toeplitz_t.hip", "kernels_matvec.hip", "kernels_near.hip", "kernels_krylov.hip", "kernels_precond.hip", "kernels_adjoint.hip", "api.hip"]
ARCH = os.environ.get("SCABS_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 6) -> str:
    """Compile every source to an object (in parallel), then link the shared library."""
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    hipcc = _hipcc()
    procs = []
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(out_dir, src + ".o")
        objs.append(obj)
        cmd = [hipcc] + HIP_FLAGS + ["-c", path, "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "-x", "hip"] + HIP_FLAGS + ["-fopenmp", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-fopenmp", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    if p.returncode:
        raise RuntimeError(f"compiling {src} failed:\n" + out.decode(errors="replace"))
    text = out.decode(errors="replace")
    if "warning" in text and os.environ.get("SCABS_BUILD_VERBOSE"):
        sys.stderr.write(text)


if __name__ == "__main__":
    print(build(verbose=True))
