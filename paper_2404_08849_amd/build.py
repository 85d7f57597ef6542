"""Build the mpdc HIP library (libmpdc.so) in-tree for gfx950.

Usage: python -m paper_2404_08849_amd.build   (or build() from Python)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpdc.so")
SOURCES = ["abi.cpp", "mesh.cpp", "dycore_kernels.hip", "tracer_kernels.hip", "stream_kernels.hip",
           "norms_static.hip", "term_kernels.hip"]
ARCH = os.environ.get("MPDC_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    """Compile every source into libmpdc.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=" + ARCH,
           # no packed-FP32 instructions (v_pk_*_f32) anywhere in the device code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           # no FMA contraction: every value is computed by the same operations whatever
           # the launch shape (bitwise-reproducible across shapes and the autotuner)
           "-ffp-contract=off",
           "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
           # every change of floating-point kind is written out (the mixed-kind
           # hazard of Section 2.2 (ii)): implicit float <-> double and
           # integer -> float conversions are errors
           "-Werror=double-promotion", "-Werror=implicit-float-conversion",
           "-x", "hip"] + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
