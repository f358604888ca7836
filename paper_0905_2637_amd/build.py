"""Build libfmm_mi355x.so in-tree with hipcc for gfx950.

Each translation unit is compiled in parallel into ``_build/`` and linked into
``paper_0905_2637_amd/libfmm_mi355x.so``.  Always rebuilds.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfmm_mi355x.so")
# a host program that drives the library through the C ABI alone
EXAMPLE_SRC = os.path.join(HERE, "examples", "fmm_eval_file.cpp")
EXAMPLE = os.path.join(HERE, "fmm_eval_file")
# the register-only FMA loop that measures the sustained FMA rate
FMA_PROBE_SRC = os.path.join(HERE, "examples", "fma_issue_rate.cpp")
FMA_PROBE = os.path.join(HERE, "fma_issue_rate")

SOURCES = ["fmm_api.cpp", "fmm_tables.cpp", "fmm_tree.hip", "fmm_upward.hip", "fmm_downward.hip",
           "fmm_near.hip", "fmm_step.hip", "fmm_fgt.hip", "fmm3d.hip", "fmm3d_api.cpp", "fmm_static.hip", "fmm_batch.hip"]

ARCH = os.environ.get("FMM_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return path


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    cmd = [hipcc(), *COMMON, "-x", "hip", EXAMPLE_SRC, "-o", EXAMPLE + ".tmp", f"-L{HERE}", "-lfmm_mi355x",
           "-Wl,-rpath,$ORIGIN"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"example build failed:\n{r.stderr}")
    os.replace(EXAMPLE + ".tmp", EXAMPLE)
    cmd = [hipcc(), *COMMON, "-x", "hip", FMA_PROBE_SRC, "-o", FMA_PROBE + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"FMA probe build failed:\n{r.stderr}")
    os.replace(FMA_PROBE + ".tmp", FMA_PROBE)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
