"""Build libcgh.so (gfx950) in-tree with hipcc.

    python -m paper_1309_2734_amd.build

Every HIP source under csrc/ is compiled for gfx950 only, with packed-FP32
instruction selection switched off, and linked into
paper_1309_2734_amd/libcgh.so next to this file; microbench.hip becomes the
program paper_1309_2734_amd/cgh_microbench.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcgh.so")
# the rate and accuracy microbenchmarks (a program, not part of the library)
MICROBENCH_SRC = os.path.join(HERE, "microbench.hip")
MICROBENCH = os.path.join(HERE, "cgh_microbench")

SOURCES = ["api.hip", "points.hip", "direct.hip", "spherical.hip", "factors.hip", "gemm.hip",
           "phase.hip", "fresnel.hip", "wrm.hip"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", f"--offload-arch={ARCH}",
         # no packed-FP32 (v_pk_*_f32) instruction selection
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-pass-failed", f"-I{INCLUDE}", f"-I{CSRC}"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "hip-link" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    """Compile every source and link libcgh.so; returns the library path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src.replace(".hip", ".o"))
        jobs.append((os.path.join(CSRC, src), obj))

    def compile_one(job):
        src, obj = job
        return _run([HIPCC, *FLAGS, "-c", src, "-o", obj])

    workers = min(len(jobs), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for log in ex.map(compile_one, jobs):
            if verbose and log:
                print(log)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *[o for _, o in jobs],
          "-o", tmp])
    os.replace(tmp, LIB)
    build_microbench()
    return LIB


def build_microbench() -> str:
    """Compile the microbenchmark program next to the library."""
    tmp = MICROBENCH + ".tmp"
    _run([HIPCC, "-O3", "-std=c++17", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          MICROBENCH_SRC, "-o", tmp])
    os.replace(tmp, MICROBENCH)
    return MICROBENCH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
