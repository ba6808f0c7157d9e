"""Build the gfx950 HIP library libld.so in-tree (hipcc cross-compiles without a GPU)."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libld.so")

# -ffp-contract=off: every multiply-add in the decision arithmetic is rounded as written
# (explicit fma() only where the method's step says so), so the FP64 bins, gates, fits and
# track columns follow a fixed operation sequence.  Packed FP32 instructions are disabled.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp,
           os.path.join(CSRC, "ld.hip"), os.path.join(CSRC, "ld_server.hip"),
           os.path.join(CSRC, "ld_cnn.hip"), os.path.join(CSRC, "ld_filter.hip"),
           os.path.join(CSRC, "ld_track.hip"), os.path.join(CSRC, "ld_stereo.hip"),
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
