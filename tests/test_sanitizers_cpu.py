"""The library's host code (validation, minimal presolve, row blocks and
tiles, option checks) under AddressSanitizer and UndefinedBehaviorSanitizer:
a host-instrumented build of libuclp runs the CPU tests of the library in a
child process with the sanitizer runtime preloaded."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_library_host_code_is_clean_under_asan_and_ubsan():
    from paper_2607_03627_amd import build as b

    lib = b.build(sanitize=True)
    env = dict(os.environ, UCLP_LIB=lib, LD_PRELOAD=b.sanitizer_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    code = ("import sys, pytest\n"
            "from paper_2607_03627_amd import uclp\n"
            "rc = pytest.main(['-q', '-p', 'no:cacheprovider', '-m', 'not gpu', 'tests/test_lib_cpu.py'])\n"
            f"assert uclp.load()._name == {lib!r}, uclp.load()._name\n"
            "sys.exit(int(rc))\n")
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, out
