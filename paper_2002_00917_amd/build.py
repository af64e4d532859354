"""Build the PSLR HIP library (libpslr.so) in-tree for gfx950.

    python -m paper_2002_00917_amd.build

Compiles the C++ host setup with g++ and the HIP sources with hipcc
(--offload-arch=gfx950), then links one shared library next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpslr.so")
BUILD = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]
HIP_SOURCES = ("pslr_kernels.hip", "pslr_vec.hip", "pslr_api.hip")
CXX_SOURCES = ("pslr_host.cpp", "pslr_schur.cpp")
CXX_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-sign-compare", "-Wno-unused-function"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd[:3]))
    return r


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    cxx = shutil.which("g++") or "g++"
    os.makedirs(BUILD, exist_ok=True)
    jobs = [[cxx] + CXX_FLAGS + ["-c", os.path.join(CSRC, src), "-o",
                                 os.path.join(BUILD, src.replace(".cpp", ".o"))]
            for src in CXX_SOURCES]
    for src in HIP_SOURCES:
        jobs.append([hipcc] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o",
                                           os.path.join(BUILD, src.replace(".hip", ".o"))])
    objs = [j[-1] for j in jobs]
    # the translation units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for _ in ex.map(lambda j: _run(j, verbose), jobs):
            pass
    tmp = OUT + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
