"""bench.py's argument checks, which run before anything touches a GPU."""
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


def test_unknown_ensemble_mode_is_refused():
    r = run("--ensemble-only", "--ensemble-modes", "ensemble,bogus")
    assert r.returncode == 2
    assert "--ensemble-modes" in r.stderr
