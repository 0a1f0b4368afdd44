"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds oracle/act_oracle.c together with tests/sanitize/oracle_driver.c with
gcc, -fsanitize=address,undefined and no recovery, and runs the driver: the
core cases (correlation, batched correlation, arg-max, objective and
gradient, refinement, residue-based, prior and complex pursuits, the
hierarchical search, reconstruction) must run without a sanitizer report and
with their identities holding.  Host code only; no GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "act_oracle.c"), os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
           "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "driver ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
