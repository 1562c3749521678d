"""bench.py's command line on the CPU: more than one GPU, or an unknown render path of the
large scene, is refused with a message before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_unknown_large_path_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--large-paths", "fp8,fp16_ess"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "fp16_ess" in p.stderr
    assert p.stdout == ""
