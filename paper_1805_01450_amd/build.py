"""Build libqgm.so (host C++ + gfx950 HIP kernels) in the package directory.

    python paper_1805_01450_amd/build.py   (the package import would load the library being built)
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqgm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", f"-I{os.path.join(ROOT, 'include')}"]
# Device code: gfx950 only; packed FP32 instructions disabled.
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def hip_runtime_dir() -> str:
    """Directory of the libamdhip64.so that torch uses (torch/lib), else /opt/rocm/lib."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec and spec.origin:
        d = os.path.join(os.path.dirname(spec.origin), "lib")
        if os.path.exists(os.path.join(d, "libamdhip64.so")):
            return d
    return "/opt/rocm/lib"


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []
    for src in sources():
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        objs.append(obj)
        if src.endswith(".hip"):
            cmd = [HIPCC, "-x", "hip", *COMMON, *DEVICE, "-c", src, "-o", obj]
        else:
            # host-only C++: plain g++ against the HIP runtime headers
            cmd = [CXX, *COMMON, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-c", src, "-o", obj]
        jobs.append(cmd)
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r, cmd in zip(ex.map(_run, jobs), jobs):
            if verbose and (r.stdout or r.stderr):
                print(" ".join(cmd), r.stdout, r.stderr, sep="\n")
    tmp = LIB + ".tmp"
    # Link against the HIP runtime that PyTorch loads, so that streams and
    # device memory handed over by torch belong to the same runtime instance.
    rt = hip_runtime_dir()
    _run([CXX, "-shared", "-fPIC", "-o", tmp, *objs, f"-L{rt}", "-l:libamdhip64.so", "-l:libhiprtc.so",
          f"-Wl,-rpath,{rt}"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
