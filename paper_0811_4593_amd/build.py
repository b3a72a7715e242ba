"""Build the HIP library liblbm.so for gfx950, in-tree.

Every HIP source is compiled with packed FP32 instructions disabled
(-target-feature -packed-fp32-ops): float code is emitted as ordinary VALU
operations.
"""
import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "liblbm.so")
SOURCES = ["csrc/lbm_kernels.hip", "csrc/lbm_sweep2.hip", "csrc/lbm_capi.hip", "csrc/lbm_batch.hip",
           "csrc/lbm_static.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # Keep the 19 populations of a node in registers: sinking the common
    # stores of the boundary rule's select arms into one store through a
    # selected address would force the population array into scratch memory.
    "-mllvm", "-simplifycfg-sink-common=false",
    "-Wall", "-Wno-unused-function",
    f"-I{os.path.join(_ROOT, 'include')}",
]


def build(verbose: bool = False, extra=()) -> str:
    srcs = [os.path.join(_HERE, s) for s in SOURCES]
    tmp = LIB_PATH + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
