"""Host-side checks of bench.py's command line (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    for n in ("2", "8"):
        p = _run("--gpus", n)
        assert p.returncode == 2
        assert "one GPU" in p.stderr and f"--gpus {n}" in p.stderr
        assert p.stdout == ""  # no JSON line for a run that did not happen


def test_unknown_workload_is_rejected():
    p = _run("--workload", "no-such-workload")
    assert p.returncode != 0
    assert "invalid choice" in p.stderr
