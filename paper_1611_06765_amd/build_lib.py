"""Build the CCD shared library for gfx950 with hipcc (in-tree).

    python -m paper_1611_06765_amd.build_lib

Produces paper_1611_06765_amd/libccd.so from csrc/ccd_plan.cpp,
csrc/ccd_device.hip, csrc/ccd_mlp.hip, csrc/ccd_ceil.hip, csrc/ccd_dense.hip
and csrc/ccd_nm.hip.  Packed FP32 instructions are disabled for all device
code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libccd.so")
ARCH = "gfx950"

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-pthread", *DEVICE_FLAGS,
           "-I", os.path.join(HERE, "..", "include"),
           os.path.join(CSRC, "ccd_plan.cpp"), os.path.join(CSRC, "ccd_device.hip"),
           os.path.join(CSRC, "ccd_mlp.hip"), os.path.join(CSRC, "ccd_ceil.hip"),
           os.path.join(CSRC, "ccd_dense.hip"), os.path.join(CSRC, "ccd_nm.hip"),
           "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
