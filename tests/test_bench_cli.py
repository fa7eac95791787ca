"""Command-line contract of bench.py that holds without a GPU: the path runs on
one GPU, so asking for more exits at once with a non-zero status and a message."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 2
    assert "one GPU only" in out.stderr
    assert out.stdout == ""
