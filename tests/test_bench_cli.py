"""bench.py with more than one GPU asked for: it exits with a message and
prints no result line (the library has no multi-GPU path), without touching
a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert r.stdout.strip() == ""
    assert "one GPU" in r.stderr and "multi-GPU" in r.stderr
