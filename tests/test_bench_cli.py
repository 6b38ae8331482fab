"""The benchmark's command line, on the CPU: it refuses any device count
other than one before it touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    for n in ("2", "8"):
        p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", n],
                           cwd=ROOT, capture_output=True, text=True, timeout=120)
        assert p.returncode == 2
        assert "exactly one GPU" in p.stderr
        assert p.stdout == ""
