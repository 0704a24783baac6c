"""The host code of the library (clustering, local regrid, plan builders, argument checks
and error paths of the C ABI) under AddressSanitizer and UndefinedBehaviorSanitizer: the
library is built a second time with both sanitizers on every host translation unit and
the host-side tests run against that build in a child process (CPU only).  Any sanitizer
report aborts the child and fails this test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(900)
def test_host_code_is_clean_under_asan_and_ubsan():
    from paper_2404_02950_amd import build_lib, sanitize_check
    try:
        build_lib._hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    try:
        sanitize_check._asan_runtime()
    except SystemExit:
        pytest.skip("no AddressSanitizer runtime beside ROCm's clang")
    r = subprocess.run([sys.executable, "-m", "paper_2404_02950_amd.sanitize_check", "--build"], cwd=ROOT,
                       capture_output=True, text=True, timeout=840)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "failed" not in r.stdout, tail
