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


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    """The library's C-ABI layer (plans, validation, workspace layouts, the
    batch descriptor tables and queue, graphs, the autotuners and their
    caches) built for the host with AddressSanitizer and
    UndefinedBehaviorSanitizer, its device side replaced by a host stand-in
    that checks every launch configuration and touches the ends of every
    buffer a kernel would use; driven through every call with valid and
    invalid arguments."""
    exe = str(tmp_path / "host_api_asan")
    csrc = os.path.join(ROOT, "paper_2012_10802_amd", "csrc")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    build = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(rocm, "include"),
             "-Wno-unused-result", "-Wno-format-truncation", "-o", exe,
             os.path.join(HERE, "sanitize", "host_api_driver.cpp"), os.path.join(HERE, "sanitize", "fake_device.cpp"),
             os.path.join(csrc, "sgm_api.cpp"), os.path.join(csrc, "sgm_batch_api.cpp")]
    res = subprocess.run(build, capture_output=True, text=True)
    if res.returncode != 0 and "sanitize" in (res.stderr or "") and "undefined reference" not in res.stderr:
        pytest.skip("sanitizer runtime not available: " + res.stderr[-200:])
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300, cwd=str(tmp_path))
    assert run.returncode == 0, run.stdout + run.stderr
    assert "clean" in run.stdout
