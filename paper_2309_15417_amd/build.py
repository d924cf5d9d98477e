"""Build libmcd.so (gfx950 HIP kernels + host runtime behind include/mcd.h)."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmcd.so")
SOURCES = ["mcd_kernels.hip", "mcd_toi.hip", "mcd_broad.hip", "mcd_narrow.hip", "mcd_fuse.hip", "mcd_impulse.hip", "mcd_runtime.hip"]
ARCH = os.environ.get("MCD_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are switched off for every HIP translation unit.
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-Wno-bitwise-instead-of-logical"]


def build(verbose=False):
    """Compile every source and link the shared library in place."""
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = ["hipcc"] + HIPFLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
