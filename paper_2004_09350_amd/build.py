"""Build the HIP libraries in-tree for gfx950 (cross-compiles without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MS_OFFLOAD_ARCH", "gfx950")
# Packed FP32 instructions are kept out of every code object.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]

LIBS = {
    "libmorphgpu.so": ["ms_kernels.hip", "ms_api.hip", "ms_plan.hip"],
    "libmsgen.so": ["datagen.hip"],
}


def build_lib(name: str, verbose: bool = True) -> str:
    out = os.path.join(HERE, name)
    srcs = [os.path.join(CSRC, s) for s in LIBS[name]]
    objs = []
    for s in srcs:
        o = os.path.join(CSRC, "_build", os.path.basename(s) + ".o")
        os.makedirs(os.path.dirname(o), exist_ok=True)
        cmd = [HIPCC, *COMMON, "-c", s, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(o)
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build_all(verbose: bool = True) -> None:
    for name in LIBS:
        build_lib(name, verbose)


if __name__ == "__main__":
    build_all(verbose="-q" not in sys.argv)
