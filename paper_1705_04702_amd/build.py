"""Builds the HIP library (libmcrt.so, gfx950) and the host lane simulator.

hipcc cross-compiles for gfx950 without a GPU.  Every HIP translation unit is
built with packed-FP32 instructions disabled; the FP64 validation kernel is
built without floating-point contraction so it rounds like an FP64 reference.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmcrt.so")
LANESIM = os.path.join(HERE, "libmcrt_lanesim.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]

UNITS = [
    ("transport_f32.hip", ["-x", "hip"]),
    ("transport_f64.hip", ["-x", "hip", "-ffp-contract=off"]),
    ("aux_kernels.hip", ["-x", "hip"]),
    ("proposal.hip", ["-x", "hip"]),
    ("microbench.hip", ["-x", "hip"]),
    ("dust.hip", ["-x", "hip", "-ffp-contract=off"]),
    ("noalloc.hip", ["-x", "hip", "-ffp-contract=off"]),
    ("mcrt_api.cpp", []),
    ("output.cpp", []),
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout)
        raise RuntimeError(f"build step failed: {cmd[-1] if cmd else ''}")
    return r.stdout


def build_hip(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)

    def compile_unit(u):
        src, extra = u
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        out = _run([HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
        if verbose and out.strip():
            print(out)
        return obj

    with ThreadPoolExecutor(max_workers=len(UNITS)) as ex:
        objs = list(ex.map(compile_unit, UNITS))
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


def build_lanesim() -> str:
    """Serial host build of the per-lane transport logic (test harness)."""
    tmp = LANESIM + ".tmp"
    _run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", f"-I{CSRC}", "-o", tmp, os.path.join(CSRC, "lanesim.cpp")])
    os.replace(tmp, LANESIM)
    return LANESIM


def build(verbose: bool = False):
    build_lanesim()
    return build_hip(verbose)


if __name__ == "__main__":
    print(build(verbose=True))
