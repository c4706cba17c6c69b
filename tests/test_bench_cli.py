"""Host-side contract of bench.py (no GPU): one GPU only, with a message for
more, and the documented options present."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    p = run("--gpus", "2")
    assert p.returncode != 0
    assert "one GPU" in p.stdout + p.stderr


def test_documented_options():
    p = run("--help")
    assert p.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--workload", "--serve", "--ncy-scan", "--sap-half-fields",
                "--no-cpu-baseline"):
        assert opt in p.stdout
