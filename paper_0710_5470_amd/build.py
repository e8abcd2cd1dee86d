"""Build the HIP library paper_0710_5470_amd/_lib/liblbm.so for gfx950.

hipcc, -O3, no fast-math; packed-FP32 instruction selection is disabled
(-packed-fp32-ops) for every HIP translation unit.  FMA contraction only
within a source expression (-ffp-contract=on), so every kernel instance of
the same arithmetic rounds the same way whatever its launch shape.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "liblbm.so")
SOURCES = [os.path.join(HERE, "csrc", "lbm_capi.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=on", "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose=False, extra=(), out=LIB):
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    cmd = [HIPCC] + HIP_FLAGS + list(extra) + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
