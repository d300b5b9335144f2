"""Build the HIP/C++ library libsphpoisson.so in-tree for gfx950.

    python paper_1806_06623_amd/build.py [--sanitize]

compiles every source under ``csrc/`` with hipcc and links one shared
library next to this file.  Packed FP32 instructions are disabled for all
device code (``-packed-fp32-ops``).

``--sanitize`` builds libsphpoisson_san.so instead: the same sources with
AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (device
code is built as usual), linked against the shared sanitizer runtime, for the
host-side tests (load it with SPP_LIB and preload the ASan runtime, as
tests/test_sanitized_host.py does).
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
LIB_SAN = os.path.join(HERE, "libsphpoisson_san.so")
OBJDIR_SAN = os.path.join(HERE, "_build_san")

SOURCES = ["plan.cpp", "eigen_ql.cpp", "solve.hip", "batch.cpp", "server.cpp", "noalloc.hip", "stream.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}", "-Wall", "-Wno-unused-result"]
# code object v5 is loadable by the HIP runtime bundled with PyTorch as well as
# by the system ROCm runtime
DEVICE = ["--offload-arch=gfx950", "-mcode-object-version=5", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"]
# host-only sanitizers (each flag after -Xarch_host: device code is not instrumented)
SANITIZE = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fno-sanitize-recover=undefined -Xarch_host -fno-omit-frame-pointer -Xarch_host -g").split()
CLANGXX = os.environ.get("SPP_CLANGXX", "/opt/rocm/llvm/bin/clang++")


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True, sanitize=False):
    from concurrent.futures import ThreadPoolExecutor
    objdir, lib = (OBJDIR_SAN, LIB_SAN) if sanitize else (OBJDIR, LIB)
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src.replace(".", "_") + ".o")
        # every source is compiled as HIP for gfx950 (host code included)
        cmd = [HIPCC] + COMMON + ["-x", "hip"] + DEVICE + (SANITIZE if sanitize else []) + ["-c", path, "-o", obj]
        jobs.append((cmd, obj))
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        list(ex.map(lambda j: _run(j[0]), jobs))
    objs = [o for _, o in jobs]
    tmp = lib + ".tmp"
    if sanitize:
        # each object already carries its device code: a host link with the
        # shared sanitizer runtime and the HIP runtime library
        rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
        _run([CLANGXX, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libsan", "-o", tmp] + objs
             + [f"-L{rocm}/lib", "-lamdhip64", "-lpthread", f"-Wl,-rpath,{rocm}/lib"])
    else:
        _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
