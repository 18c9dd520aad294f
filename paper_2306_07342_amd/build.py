"""Build libvqd.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2306_07342_amd.build        # or build() from Python

Objects go to paper_2306_07342_amd/_build/, the library to
paper_2306_07342_amd/libvqd.so.  Every call recompiles every source.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvqd.so")
ARCH = os.environ.get("VQD_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.cpp", "builders.cpp", "planner.cpp", "batch.cpp", "traj.cpp", "measure.cpp", "device.cpp",
           "presets.cpp",
           "kernels.hip",
           "mlp.hip", "traj.hip", "measure.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-fcx-limited-range",
          "-I", os.path.join(HERE, "..", "include")]
# packed FP32 instructions stay off in all device code
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [hipcc(), *COMMON, "-c", path, "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = DEVICE
    else:
        # host sources: hipcc still runs a device pass over them, so name the
        # target rather than take its default
        cmd[1:1] = ["-D__HIP_PLATFORM_AMD__", "--offload-arch=" + ARCH]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
