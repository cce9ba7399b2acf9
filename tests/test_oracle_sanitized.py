"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a C
driver (tests/native/oracle_sanitize_driver.c) that includes the oracle
source and runs every option on tiny cases is built with gcc and run; any
invalid access, leak or undefined behaviour fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = tmp_path / "oracle_sanitized"
    src = os.path.join(HERE, "native", "oracle_sanitize_driver.c")
    cmd = [gcc, "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", src, "-o", str(exe), "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and ("-lasan" in build.stderr or "-lubsan" in build.stderr):
        pytest.skip("sanitizer runtimes not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "oracle sanitized run: ok" in run.stdout
