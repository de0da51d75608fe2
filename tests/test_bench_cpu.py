"""bench.py's command-line contract, checked without a GPU: it refuses more
than one GPU with a message (before touching the GPU) and offers the launch
and step-kernel choices."""

import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def run(*args):
    return subprocess.run([sys.executable, str(ROOT / "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_options():
    r = run("--help")
    assert r.returncode == 0
    for opt in ("--launch", "--step-kernel", "--workload", "--table1", "--cpu-pulses"):
        assert opt in r.stdout, opt
    r = run("--launch", "nonsense")
    assert r.returncode != 0

