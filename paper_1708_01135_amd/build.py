"""Build the gfx950 HIP library ``libewald_mi355x.so`` in-tree with hipcc.

All HIP sources are compiled with packed-FP32 instruction selection disabled
(``-target-feature -packed-fp32-ops``); the kernels are written for plain
64-wide wavefront VALU/scalar execution on CDNA4.  MFMA results are kept in
VGPRs (``-amdgpu-mfma-vgpr-form``): the gather's epilogue reads every
accumulator, and the AGPR form cost a copy per value and two waves per SIMD.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libewald_mi355x.so")
ARCH = os.environ.get("EWALD_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra=None) -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-mllvm", "-amdgpu-mfma-vgpr-form=1",
           "-Wall", "-Wno-unused-function",
           "-I", os.path.join(ROOT, "include"), "-o", LIB + ".tmp"] + srcs + list(extra or [])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


RSA_LIB = os.path.join(HERE, "librsa_accept.so")


def build_host_helpers(verbose: bool = False) -> str:
    """The input generator's C helper (random sequential addition); no GPU code."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off", "-Wall", "-Wextra",
           "-o", RSA_LIB + ".tmp", os.path.join(HERE, "csrc_host", "rsa_accept.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(RSA_LIB + ".tmp", RSA_LIB)
    return RSA_LIB


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_host_helpers(verbose=True))
