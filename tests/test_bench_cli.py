"""The benchmark script's command line, checked on the CPU: it parses, documents its options, and refuses a
GPU count other than one with a message (this build measures one GPU's share)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_help_lists_the_workloads_and_solver_options():
    r = _run("--help")
    assert r.returncode == 0, r.stderr
    for opt in ("--workload", "--batched", "--krylov-poly", "--gmres-m", "--eps-r", "--autotune", "--reorder"):
        assert opt in r.stdout


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
