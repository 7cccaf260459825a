"""Build libptebd.so (and the counter-calibration copy, libhbmcopy.so) for gfx950 with hipcc
(in-tree, next to this file).

Usage: ``python -m paper_2312_02667_amd.build`` or ``paper_2312_02667_amd.build.build()``.
Every HIP source is compiled with packed FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``).
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libptebd.so")
# the copy of known size that calibrates the HBM byte counters (measurement support only)
COPY_LIB = os.path.join(HERE, "libhbmcopy.so")
COPY_SOURCE = "hbm_copy.hip"
SOURCES = ["ptebd_api.hip", "ptebd_kernels.hip", "ptebd_queries.hip", "ptebd_sample.hip",
           "ptebd_precond.hip", "ptebd_noalloc.hip", "ptebd_jacobi64.hip", "ptebd_theta.hip"]
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _run(cmd):
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(line for line in proc.stdout.splitlines()
                    if "unknown target feature" not in line and "packed-fp32-ops" not in line)
    if proc.returncode != 0:
        raise RuntimeError(f"command failed ({proc.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source and link ``libptebd.so``; returns the library path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([HIPCC, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(_run, cmds))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    tmp = COPY_LIB + ".tmp"
    _run([HIPCC, *COMMON, "-shared", "-o", tmp, os.path.join(CSRC, COPY_SOURCE)])
    os.replace(tmp, COPY_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
