"""Build the HIP/C++ library libsphpoisson.so in-tree for gfx950.

    python paper_1806_06623_amd/build.py

compiles every source under ``csrc/`` with hipcc and links one shared
library next to this file.  Packed FP32 instructions are disabled for all
device code (``-packed-fp32-ops``).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsphpoisson.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = ["plan.cpp", "eigen_ql.cpp", "solve.hip", "batch.cpp", "server.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}", "-Wall", "-Wno-unused-result"]
# code object v5 is loadable by the HIP runtime bundled with PyTorch as well as
# by the system ROCm runtime
DEVICE = ["--offload-arch=gfx950", "-mcode-object-version=5", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True):
    os.makedirs(OBJDIR, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(OBJDIR, src.replace(".", "_") + ".o")
        lang = ["-x", "hip"] + DEVICE if src.endswith(".hip") else ["-x", "hip"] + DEVICE
        _run([HIPCC] + COMMON + lang + ["-c", path, "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
