"""Build the HIP libraries in-tree for gfx950 (cross-compiles without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MS_OFFLOAD_ARCH", "gfx950")
# Packed FP32 instructions are kept out of every code object.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]

# (source, extra flags): morph and project are compiled once per output kind
# (MS_OK = UNCOMPR 0 .. FOR_DYN_BP 4) so that the instantiations build in parallel.
_PER_KIND = [(src, [f"-DMS_OK={k}"]) for src in ("ms_project.hip", "ms_morph.hip") for k in range(5)]
LIBS = {
    "libmorphgpu.so": _PER_KIND + [("ms_kernels.hip", []), ("ms_api.hip", []), ("ms_plan.hip", []),
                                   ("ms_selector.hip", []), ("ms_pred.hip", []),
                                   ("ms_ops2.hip", []), ("ms_batch.hip", [])],
    "libmsgen.so": [("datagen.hip", [])],
}
JOBS = max(1, min(16, int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))


def _object(src: str, flags) -> str:
    tag = "".join("." + f[2:].replace("=", "").lower() for f in flags)
    return os.path.join(CSRC, "_build", os.path.basename(src) + tag + ".o")


def build_lib(name: str, verbose: bool = True) -> str:
    out = os.path.join(HERE, name)
    jobs = []
    for src, flags in LIBS[name]:
        o = _object(src, flags)
        os.makedirs(os.path.dirname(o), exist_ok=True)
        jobs.append([HIPCC, *COMMON, *flags, "-c", os.path.join(CSRC, src), "-o", o])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return cmd[-1]

    with ThreadPoolExecutor(max_workers=JOBS) as ex:
        objs = list(ex.map(run, jobs))
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
