"""bench.py's command-line contract, checked without a GPU: any positive
step count is accepted and split over the eight force forms; more than one
GPU and non-positive step counts are refused before touching the device."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("steps", ["0", "-3"])
def test_non_positive_steps_are_refused(steps):
    r = _run("--steps", steps)
    assert r.returncode == 2
    assert "positive" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("steps,expect", [
    ("20", [3, 3, 3, 3, 2, 2, 2, 2]),
    ("12", [2, 2, 2, 2, 1, 1, 1, 1]),
    ("5", [1, 1, 1, 1, 1, 0, 0, 0]),
    ("1600", [200] * 8),
])
def test_any_positive_step_count_splits_over_the_forms(steps, expect):
    r = _run("--gpus", "1", "--steps", steps, "--warmup", "5", "--check-args")
    assert r.returncode == 0, r.stderr
    got = json.loads(r.stdout.strip().splitlines()[-1])["steps_per_form"]
    assert list(got.values()) == expect
    assert sum(got.values()) == int(steps)


def test_split_function():
    import bench
    for k in range(1, 40):
        c = bench.split_steps(k)
        assert sum(c) == k and max(c) - min(c) <= 1 and c == sorted(c, reverse=True)
