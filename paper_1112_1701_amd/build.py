"""Build the gfx950 HIP library libbls_mi355x.so in-tree with hipcc.

    python -m paper_1112_1701_amd.build          # build (always recompiles)

Every HIP source is compiled for gfx950 only, with FP contraction off (the
phase bins must follow the FP64 operation order of their definition) and
packed-FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libbls_mi355x.so")

SOURCES = ["bls_kernels.hip", "bls_unbinned.hip", "bls_detect.hip", "bls_window.hip",
           "bls_variability.hip", "bls_plan.cpp", "bls_autotune.cpp",
           "bls_server.cpp", "bls_noalloc.hip", "bls_recovery.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-ffp-contract=off", "-fno-fast-math", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout,
                                                             r.stderr))
    return obj


PROBES_SRC = "bls_probes.hip"
PROBES_LIB = os.path.join(HERE, "libbls_probes.so")


def build_probes(verbose: bool = False) -> str:
    """The micro-benchmark library libbls_probes.so (bench.py --probes)."""
    obj = _compile(PROBES_SRC)
    tmp = PROBES_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, PROBES_LIB)
    if verbose:
        print("built", PROBES_LIB)
    return PROBES_LIB


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + \
        objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    build_probes(verbose=True)
    sys.exit(0)
