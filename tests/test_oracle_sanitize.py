"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sanitize_check.c runs every oracle entry point on small inputs,
including integer sums that wrap many times: signed overflow is undefined
in C, so a clean UBSan run is what enforces the modulo-2^32 rule of the
scan and the reduction.  Host code only; nothing of the HIP path is built.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    import oracle

    exe = str(tmp_path / "sanitize_check")
    srcs = [os.path.join(ORACLE, s) for s in oracle._SOURCES] + [os.path.join(ORACLE, "sanitize_check.c")]
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-strict-aliasing",
           "-fopenmp", "-pthread", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-o", exe] + srcs
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitize ok" in r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
