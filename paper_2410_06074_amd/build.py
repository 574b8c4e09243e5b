"""Build libsmnn.so (HIP, gfx950) in-tree.

    python -m paper_2410_06074_amd.build

compiles csrc/smnn_kernels.hip once per block size (K = 2..5) and group of
instance forms in parallel,
csrc/smnn_misc.hip, csrc/smnn_noalloc.hip and csrc/smnn_api.cpp, and links them into
paper_2410_06074_amd/libsmnn.so.  Objects go to paper_2410_06074_amd/_build/.
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
LIB = os.path.join(HERE, "libsmnn.so")
ARCH = os.environ.get("SMNN_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          # keep the compiler from forming packed FP32 instructions
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libsmnn")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return cmd[-1]


def build(jobs: int | None = None, verbose: bool = False) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    units = []
    # one translation unit per block size K and group of instance forms:
    # 0 = one variable with scalar weights (and the separator levels),
    # 1 = one variable with per-row weights, 2 = two coupled variables
    for K, forms in ((4, 2), (3, 0), (4, 0), (2, 0), (5, 0), (2, 1), (3, 1), (4, 1), (5, 1)):
        units.append([hipcc, *COMMON, f"-DSMNN_TU_K={K}", f"-DSMNN_TU_FORMS={forms}", "-c",
                      os.path.join(CSRC, "smnn_kernels.hip"), "-o", os.path.join(BUILD, f"smnn_kernels_k{K}f{forms}.o")])
    # wide blocks (K = 6, 9): one 16-lane group per chunk
    for K in (9, 6):
        units.append([hipcc, *COMMON, f"-DSMNN_TU_K={K}", "-c", os.path.join(CSRC, "smnn_wide.hip"),
                      "-o", os.path.join(BUILD, f"smnn_wide_k{K}.o")])
    units.append([hipcc, *COMMON, "-c", os.path.join(CSRC, "smnn_misc.hip"), "-o", os.path.join(BUILD, "smnn_misc.o")])
    units.append([hipcc, *COMMON, "-c", os.path.join(CSRC, "smnn_noalloc.hip"),
                  "-o", os.path.join(BUILD, "smnn_noalloc.o")])
    units.append([hipcc, *COMMON, "-c", os.path.join(CSRC, "smnn_api.cpp"), "-o", os.path.join(BUILD, "smnn_api.o")])
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_run, units))
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
