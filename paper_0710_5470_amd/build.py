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
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=on", "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"),
]
# translation units and their extra flags: the D3Q19 step kernels are
# scheduled for instruction-level parallelism (faster there, slower for the
# batched D2Q9 kernels of the main unit)
UNITS = [(os.path.join(HERE, "csrc", "lbm_capi.hip"), []),
         (os.path.join(HERE, "csrc", "lbm_step3d.hip"), ["-mllvm", "--amdgpu-sched-strategy=max-ilp"])]
SOURCES = [u[0] for u in UNITS]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False, extra=(), out=LIB):
    """Compile every unit to an object (in parallel) and link the library."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    objs, procs = [], []
    for src, flags in UNITS:
        obj = "%s.%s.o" % (out, os.path.splitext(os.path.basename(src))[0])
        cmd = [HIPCC] + HIP_FLAGS + flags + list(extra) + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    _run([HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared"] + objs + ["-o", tmp], verbose)
    for obj in objs:
        os.remove(obj)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
