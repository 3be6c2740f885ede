"""Build liboat.so (HIP kernels for gfx950 + host plan + C ABI) in-tree."""
import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liboat.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_SOURCES = ["oat_srt.hip", "oat_aux.hip", "oat_cnn.hip", "oat_eir.hip", "oat_sph.hip"]
HOST_SOURCES = ["oat_plan.cpp"]
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def sources():
    return ([os.path.join(CSRC, f) for f in DEVICE_SOURCES + HOST_SOURCES]
            + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
            + [os.path.join(INCLUDE, f) for f in ("oat.h", "oat_cnn.h")])


def build(verbose: bool = False) -> str:
    tmp = tempfile.mkdtemp(prefix="oat_build_")
    try:
        objs = []
        for f in DEVICE_SOURCES:
            o = os.path.join(tmp, f + ".o")
            cmd = [HIPCC, "-x", "hip", "-c", os.path.join(CSRC, f), "-o", o,
                   "-I", INCLUDE, "-I", CSRC] + DEVICE_FLAGS
            if verbose:
                print(" ".join(cmd))
            subprocess.run(cmd, check=True)
            objs.append(o)
        for f in HOST_SOURCES:
            o = os.path.join(tmp, f + ".o")
            cmd = [HIPCC, "-c", os.path.join(CSRC, f), "-o", o, "-I", INCLUDE,
                   "-I", CSRC] + HOST_FLAGS
            if verbose:
                print(" ".join(cmd))
            subprocess.run(cmd, check=True)
            objs.append(o)
        out = LIB + ".tmp"
        cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", out] + objs
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
