"""Builds libcr.so (HIP, gfx950) in-tree with hipcc.

Flags that matter for correct rounding:
  -ffp-contract=off           no implicit a*b+c fusion (error-free transforms
                              rely on exact operation order; every fma is
                              written explicitly)
  -fno-gpu-flush-denormals-to-zero
                              IEEE gradual underflow for binary32 as well
  -Xclang -target-feature -Xclang -packed-fp32-ops
                              no packed binary32 instructions
No fast-math, no approximate library functions.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcr.so")
REF_LIB = os.path.join(PKG, "libcr_ulpref.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def build(verbose=False, extra=()):
    src = os.path.join(CSRC, "cr_lib.hip")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra) + [src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


def build_ref(verbose=False):
    """The platform's ~1-ulp functions as maps (benchmark comparison only)."""
    src = os.path.join(CSRC, "ulp_ref.hip")
    tmp = REF_LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + [src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, REF_LIB)
    return REF_LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
    build_ref(verbose=True)
