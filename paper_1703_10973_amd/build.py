"""Builds liblrsdp.so (the HIP library behind include/lrsdp.h) for gfx950 with hipcc.

Usage:  python -m paper_1703_10973_amd.build   (or build() from Python)
Objects go to paper_1703_10973_amd/_build/, the library next to this file.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblrsdp.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["api.hip", "ingest.hip", "hv.hip", "dense.hip", "eig.hip", "spectral.hip", "serve.hip", "factor.hip",
           "apply.hip", "pcg.hip", "ipm.hip", "augsys.hip"]

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-mcode-object-version=5",
    "-ffp-contract=off", "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
    # packed FP32 instructions stay off (see the build notes in the design document)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE,
]


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")
    return exe


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{p.stderr}")
    errs = [ln for ln in p.stderr.splitlines()
            if "warning" in ln and "packed-fp32-ops" not in ln]
    return obj, errs


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every HIP source and link liblrsdp.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    if verbose:
        for obj, warns in results:
            for w in warns:
                print(w, file=sys.stderr)
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
