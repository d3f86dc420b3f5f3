"""The C-ABI sources under host AddressSanitizer and UndefinedBehaviorSanitizer.

The api*.cpp files (validation, workspace layout, schedules, every entry
point's host code) are rebuilt with ASan + UBSan on their host code (device
code unchanged, errors fatal) and the CPU ABI tests run against that build in
a child process with the clang ASan runtime preloaded.  Nothing here touches
a GPU.
"""

import os
import subprocess
import sys

import pytest

from paper_2305_14566_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    src = [os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC)] + [os.path.join(ROOT, "include", "omniseg.h")]
    return any(os.path.getmtime(p) > t for p in src)


@pytest.fixture(scope="module")
def sanitized_lib():
    lib = B.SANITIZED_LIB
    if _stale(lib):
        B.build_sanitized()
    return lib


def test_sanitized_build_is_instrumented(sanitized_lib):
    syms = subprocess.run(["nm", "-D", sanitized_lib], capture_output=True, text=True).stdout
    assert "__asan_report_load" in syms
    assert "__ubsan_handle_" in syms


def test_abi_tests_clean_under_asan_ubsan(sanitized_lib):
    env = dict(os.environ)
    env["OMNISEG_LIBRARY"] = sanitized_lib
    env["LD_PRELOAD"] = B.sanitizer_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_abi.py"), os.path.join(HERE, "test_stream_schedule.py"),
                        os.path.join(HERE, "test_zz_no_alloc.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out
    assert " passed" in out
