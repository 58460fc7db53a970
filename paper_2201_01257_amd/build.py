"""Build the native libraries in-tree: the HIP library (gfx950) and the input generator."""

from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtamm_mi.so")
SOURCES = ["capi_core.cpp", "plan.cpp", "denominator.cpp", "addop.cpp", "sched.cpp", "cholesky.cpp", "kernels.hip", "kernels_mixed.hip",
           "kernels_elem.hip", "diag.hip", "noalloc.hip"]
HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions are never generated (see the design notes on gfx950 hazards)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in architectural VGPRs: without it the loop-carried accumulators are
    # copied between VGPRs and AGPRs on every K chunk
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-I" + os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found; the HIP library cannot be built")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build_hip(verbose: bool = False) -> str:
    """Compile every source to an object in parallel, then link the shared library in place."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="tamm_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in sources()]
        cmds = [[hipcc()] + compile_flags + ["-c", "-o", obj, src] for src, obj in zip(sources(), objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            for f in [ex.submit(subprocess.check_call, c) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp%d" % os.getpid()
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(tmp, LIB)
    return LIB


def build_all(verbose: bool = False):
    from .synth import build_library

    build_library(force=True)
    return build_hip(verbose)


if __name__ == "__main__":
    build_all(verbose=True)
