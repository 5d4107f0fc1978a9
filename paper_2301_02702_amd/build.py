"""Build ``libkomahip.so`` (HIP kernels + C-ABI host code) for gfx950 in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", f)
       for f in ("komahip_host.cpp", "komahip_discretize.cpp", "komahip_kernels.hip", "komahip_mrf.hip",
                 "komahip_lowrank.hip", "komahip_scratch.hip")]
DEPS = SRC + [os.path.join(HERE, "csrc", h) for h in ("komahip_internal.h", "komahip_mrf.h", "komahip_lowrank.h",
                                                           "komahip_scratch.h")] + \
    [os.path.join(ROOT, "include", "komahip.h")]
LIB = os.path.join(HERE, "libkomahip.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 (v_pk_*) stays off: the compiler would otherwise form it
    # from plain float code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # host code (sequence packing): AVX2 and FMA, present on every x86-64
    # host of this GPU generation
    "-Xarch_host", "-mavx2", "-Xarch_host", "-mfma",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    """Compile the library (always recompiles) and return its path."""
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), *SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build libkomahip.so")
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
