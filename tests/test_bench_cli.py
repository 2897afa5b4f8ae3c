"""bench.py's command line on a machine without a GPU: the one-GPU contract
(more than one GPU is refused with a message) and the help text."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_workloads():
    r = run("--help")
    assert r.returncode == 0
    for w in ("pool", "batch", "large", "policy", "bnb"):
        assert w in r.stdout
