"""Build steps for the native libraries (in-tree, gfx950 only).

libmttkrp.so   HIP kernels + C-ABI host library (hipcc, --offload-arch=gfx950)
libsynth.so    input-generator helpers (gcc, OpenMP)
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmttkrp.so")
SYNTH = os.path.join(HERE, "libsynth.so")

HIP_SOURCES = ["mttkrp_lib.hip"] + [f"inst_n{n}.hip" for n in range(2, 9)]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    subprocess.check_call(cmd)


def build_synth(force: bool = True) -> str:
    if force or not os.path.exists(SYNTH):
        tmp = SYNTH + ".tmp"
        _run(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp,
              os.path.join(CSRC, "synth.c")])
        os.replace(tmp, SYNTH)
    return SYNTH


def build_lib(force: bool = True, extra=(), jobs: int | None = None) -> str:
    """Compile every HIP translation unit (in parallel) and link the library."""
    if force or not os.path.exists(LIB):
        from concurrent.futures import ThreadPoolExecutor
        hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin",
                             "hipcc")
        objdir = os.path.join(CSRC, "_build")
        os.makedirs(objdir, exist_ok=True)

        def one(src):
            obj = os.path.join(objdir, src.replace(".hip", ".o"))
            _run([hipcc, *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, "-c",
                  "-o", obj, os.path.join(CSRC, src)])
            return obj

        n = jobs or min(len(HIP_SOURCES), max(1, (os.cpu_count() or 4)))
        with ThreadPoolExecutor(max_workers=n) as ex:
            objs = list(ex.map(one, HIP_SOURCES))
        tmp = LIB + ".tmp"
        _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp,
              *objs])
        os.replace(tmp, LIB)
    return LIB


def build_all(force: bool = True):
    build_synth(force)
    build_lib(force)
