"""The FP64 oracle built with the address and undefined-behaviour sanitizers
(gcc) and run over every exported routine on a tiny case
(oracle/sanitize_driver.c): no sanitizer report, exit status 0."""
import os
import shutil
import subprocess

import pytest

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_sanitized")
    flags = ["-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    build = subprocess.run(["gcc", *flags, "-o", exe, os.path.join(ORACLE, "sanitize_driver.c"),
                            "-lm"], capture_output=True, text=True)
    if build.returncode != 0 and "asan" in (build.stderr + build.stdout).lower():
        pytest.skip("sanitizer runtime not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    print(run.stdout, run.stderr[-2000:])
    assert run.returncode == 0
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr
    assert "ok" in run.stdout
