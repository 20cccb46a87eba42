"""bench.py command line, on the CPU: more than one GPU is refused with a message and
exit status 2 before anything touches a device; --help lists the workloads."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_help_lists_workloads():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("C2", "C3", "C3darcy", "C4", "C5", "D3"):
        assert w in r.stdout
