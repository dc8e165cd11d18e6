"""The host code of the library under AddressSanitizer and
UndefinedBehaviorSanitizer: the host-sanitizer build (host code
instrumented, device code as usual) runs the host-side C-ABI tests
(tests/test_abi_host.py: local bases, tree and sector allocation, block
tables, argument and error checks, checkpoint file checks) in a child
process with the clang ASan runtime preloaded.  Any sanitizer report ends
the child with an error."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_host_under_asan_and_ubsan():
    from paper_2011_10658_amd import build as B
    rt = B.asan_runtime()
    if rt is None:
        pytest.skip("no clang ASan runtime in this toolchain")
    lib = B.build_sanitized()
    env = dict(os.environ, LD_PRELOAD=rt, QEDTTN_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, out
    assert " passed" in r.stdout, out
