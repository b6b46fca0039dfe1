"""Build the native library libs2mi.so in-tree (hipcc for gfx950, g++ for the
quad-precision host constant generator).

    python -m paper_2311_14670_amd.build
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libs2mi.so")
ARCH = os.environ.get("S2MI_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
             # packed-FP32 instructions stay off (hipcc's host pass warns about the feature; harmless)
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in ["s2mi_kernels.hip", "s2mi_mfma.hip", "s2mi_capi.hip"]:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        _run(["hipcc", "-c", "-x", "hip"] + HIP_FLAGS + [os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    obj = os.path.join(BUILD, "s2mi_consts.o")
    _run(["g++", "-c", "-O2", "-fPIC", "-std=gnu++17", "-I", CSRC, os.path.join(CSRC, "s2mi_consts.cpp"), "-o", obj])
    objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + ["-lquadmath", "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
