"""The host code of libgccd under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is rebuilt with its host code instrumented (libgccd_san.so, see
paper_2203_11043_amd/build.py) and the C-ABI tests of test_abi_cpu.py run
against it in a child process with the ASan runtime preloaded: argument
validation, NULL handling, struct layout, error strings and the device-less
init path.  Any sanitizer report aborts the child and fails this test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def san_lib():
    from paper_2203_11043_amd import build
    if not os.path.exists(build.SAN_LIB):
        build.build_sanitized()
    return build.SAN_LIB, build.asan_runtime()


def test_abi_suite_under_sanitizers(san_lib):
    lib, rt = san_lib
    env = dict(os.environ)
    env.update(
        GCCD_LIB=lib,
        LD_PRELOAD=rt,
        # Python and the HIP runtime keep allocations to the end of the process
        ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
        UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
    )
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_abi_cpu.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert "AddressSanitizer" not in out and "runtime error" not in out
    assert r.returncode == 0, out[-3000:]
    assert " passed" in out


def test_sanitized_library_is_instrumented(san_lib):
    lib, _ = san_lib
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_" in syms and "__ubsan_" in syms
