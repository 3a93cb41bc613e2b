"""Compile the HIP library for gfx950 (in-tree, no JIT cache).

The shared library exports the C ABI declared in include/relres.h.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librelres_hip.so")
SOURCES = [os.path.join(CSRC, "relres_kernels.hip"), os.path.join(CSRC, "relres_md.hip"),
           os.path.join(CSRC, "relres_host.cpp")]
ARCH = os.environ.get("RELRES_OFFLOAD_ARCH", "gfx950")


def hipcc_command(out: str):
    return ["/opt/rocm/bin/hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-shared", "-Wall", "-Wno-unused-function",
            # no packed FP32 instructions (v_pk_*_f32) anywhere in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC,
            *SOURCES, "-o", out]


def build(verbose: bool = False) -> str:
    cmd = hipcc_command(LIB + ".tmp")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
