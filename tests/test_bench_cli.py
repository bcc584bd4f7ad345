"""The benchmark's command-line contract on the CPU: more than one GPU is
refused with a message and a non-zero exit before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_second_order_needs_only():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--second-order"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "--only" in r.stderr
    assert r.stdout == ""
