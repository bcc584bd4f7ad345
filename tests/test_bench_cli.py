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


def test_traffic_digest_follows_code_not_comments():
    """The counters' traffic is reported only for the kernel code it was
    taken on: the digest ignores comments and blank lines, not code."""
    sys.path.insert(0, ROOT)
    import bench
    a = "int f(int x) {\n  return x + 1;  // one more\n}\n"
    b = "// header\nint f(int x) {\n\n  /* the sum */ return x + 1;\n}\n"
    c = "int f(int x) {\n  return x + 2;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)
    for tag in ("k_step3_fp64", "k_step3_mixed"):
        traffic, source = bench.load_traffic(tag, "box3d_128cube_S8")
        if traffic is not None:   # the committed summaries match the built code
            assert source.startswith("profiles/traffic_") and traffic > 0
