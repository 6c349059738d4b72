"""The host C++ of the library under AddressSanitizer and UndefinedBehavior-
Sanitizer (tests/host_check.cpp, built by build()): argument validation of
every entry point, the host helpers over wide input ranges, and the tuner-cache
and model-file parsers on malformed files.  CPU only."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECK = os.path.join(ROOT, "_build", "host_check", "host_check")


@pytest.mark.skipif(not os.path.exists(CHECK), reason="host check not built (run build())")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    env = dict(os.environ, HOST_CHECK_DIR=str(tmp_path), HIP_VISIBLE_DEVICES="",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([CHECK], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.returncode == 0 and "PASSED" in r.stdout
