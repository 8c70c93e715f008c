"""Builds the HIP library ``librdx.so`` in-tree for gfx950 with hipcc.

Flags: -O3, fp contraction off and no fast-math (every floating-point
operation of the scheme is a single IEEE-754 operation), packed-FP32
instructions disabled, position-independent shared object.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "librdx.so")
SOURCES = ["rdx_setup.cpp", "rdx_engine.cpp", "rdx_api.cpp", "rdx_server.cpp", "rdx_kernels.hip", "rdx_record.hip"]
ARCH = os.environ.get("RDX_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
              "-Wall", "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}"]
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(build_dir, src + ".o")
        cmd = [hipcc(), *common, "-c", path, "-o", obj]
        if src.endswith(".hip"):
            cmd += [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops"]
        else:
            cmd += ["-D__HIP_PLATFORM_AMD__"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
