"""Build libgsis.so (HIP for gfx950) in-tree.

``python -m paper_2507_03975_amd.build`` or ``build()`` compiles every HIP
source under ``csrc/`` with hipcc and links the shared library next to this
file. Packed-FP32 instructions are disabled for all device code. Kernel
arguments (the first 16 dwords) are preloaded into scalar registers at wave
launch: every kernel here starts with a chain of dependent scalar loads
(arguments, then a descriptor, then what it points to) before its first
vector load, and the preload takes the first link out of it (the synthetic
solve of a 256 x 256 x 128 step 0.115 -> 0.111 ms). The code object keeps a
prologue that loads them itself where the firmware does not preload.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build", "gsis")
LIB = os.path.join(HERE, "libgsis.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-amdgpu-kernarg-preload-count=16",
          "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]

SOURCES = ["capi.cpp", "batch.cpp", "adjoint.cpp", "kernels_transport.hip",
           "kernels_synth.hip", "kernels_adjoint.hip"]


def _compile(src):
    out = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return out


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
