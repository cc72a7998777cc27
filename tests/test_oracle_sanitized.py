"""The oracle's host code under AddressSanitizer and UndefinedBehaviorSanitizer: every exported
entry point on small problems of each network shape, with empty, single, moving and blocking
obstacle points and every rounding mode (oracle/sanitize_check.c)."""
import os
import shutil
import subprocess

import pytest

import oracle


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = oracle.build_sanitized(str(tmp_path / "orc_sanitize"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    assert "oracle sanitizer run: ok" in r.stdout
