"""Host sanitizers on the CPU oracle: every oracle entry point, built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code only), on
small inputs of awkward sizes (1x1, single rows and columns, windows of 1 to
256)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    build = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-o", exe, os.path.join(HERE, "sanitize", "oracle_driver.c"),
             os.path.join(ROOT, "oracle", "sgm_oracle.c"), "-lm"]
    res = subprocess.run(build, capture_output=True, text=True)
    if res.returncode != 0 and "sanitize" in (res.stderr or ""):
        pytest.skip("sanitizer runtime not available: " + res.stderr[-200:])
    assert res.returncode == 0, res.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "clean" in run.stdout
