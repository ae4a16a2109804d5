"""bench.py's command line on the host (no GPU work): the single-GPU
refusal and the workload list."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_workloads_listed():
    r = run("--help")
    assert r.returncode == 0
    for w in ("stack1k", "slices2048", "stack4k-f16", "learned2k", "npr-video", "ad1k-dct", "stack1k-streamed"):
        assert w in r.stdout
    for opt in ("--steps", "--warmup", "--discretization", "--prolong"):
        assert opt in r.stdout
