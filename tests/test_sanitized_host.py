"""The host-side ABI tests under AddressSanitizer and UndefinedBehaviorSanitizer.

`python paper_1806_06623_amd/build.py --sanitize` (also run by
__graft_entry__.build()) builds libsphpoisson_san.so: the library's host code
instrumented with ASan and UBSan (UB is fatal), its device code as usual.
This test runs tests/test_abi.py in a child process that loads that library
(SPP_LIB) with the ASan runtime preloaded (Python itself is not
instrumented).  Leak detection is off: the interpreter and the HIP runtime
keep allocations until exit by design.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_LIB = os.path.join(ROOT, "paper_1806_06623_amd", "libsphpoisson_san.so")


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_abi_tests_pass_under_asan_and_ubsan(tmp_path):
    rt = _asan_runtime()
    if not os.path.exists(SAN_LIB) or rt is None:
        pytest.skip("sanitized library not built (python paper_1806_06623_amd/build.py --sanitize)")
    env = dict(os.environ)
    env.update({
        "SPP_LIB": SAN_LIB,
        "LD_PRELOAD": rt,
        "ASAN_OPTIONS": f"detect_leaks=0:abort_on_error=0:log_path={tmp_path}/asan",
        "UBSAN_OPTIONS": f"print_stacktrace=1:halt_on_error=1:log_path={tmp_path}/ubsan",
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = ""
    for f in sorted(glob.glob(str(tmp_path / "asan*")) + glob.glob(str(tmp_path / "ubsan*"))):
        reports += open(f).read()[:4000]
    assert r.returncode == 0 and not reports, (r.stdout[-3000:] + r.stderr[-3000:] + reports)
    assert " passed" in r.stdout
