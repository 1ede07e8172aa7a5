"""The CPU oracle built under AddressSanitizer and UndefinedBehaviorSanitizer (host code
only): oracle/sanitize_driver.c calls every exported routine on small ragged inputs,
including breakdowns; any memory error, leak or undefined behaviour aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-ffp-contract=off", "-D_GNU_SOURCE", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-o", str(exe),
           os.path.join(ROOT, "oracle", "sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "tsqr_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-3000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out
    assert out.count("done") == 5
