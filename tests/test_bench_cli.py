"""bench.py's command-line contract, checked without a GPU: it refuses more
than one GPU and step counts that do not split over the eight force forms,
before touching the device."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("steps", ["12", "0"])
def test_steps_must_split_over_the_forms(steps):
    r = _run("--steps", steps)
    assert r.returncode == 2
    assert "multiple of 8" in r.stderr
