"""The benchmark's command line on the CPU: it refuses more than one GPU
with a message before touching a device, and its kernel-source digest is
stable."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    for n in ("2", "8"):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", n], capture_output=True,
                           text=True, timeout=120, cwd=ROOT)
        assert r.returncode == 2
        assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_source_digest_is_stable():
    sys.path.insert(0, ROOT)
    import bench
    a, b = bench.kernel_source_digest(), bench.kernel_source_digest()
    assert a == b and len(a) == 16 and int(a, 16) >= 0
