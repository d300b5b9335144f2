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

SOURCES = ["plan.cpp", "eigen_ql.cpp", "solve.hip", "batch.cpp", "server.cpp", "noalloc.hip"]

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
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(OBJDIR, src.replace(".", "_") + ".o")
        # every source is compiled as HIP for gfx950 (host code included)
        jobs.append(([HIPCC] + COMMON + ["-x", "hip"] + DEVICE + ["-c", path, "-o", obj], obj))
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        list(ex.map(lambda j: _run(j[0]), jobs))
    objs = [o for _, o in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
