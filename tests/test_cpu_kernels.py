"""The library's own kernels, built for the host and run on the CPU under
AddressSanitizer, against the oracle (no GPU needed).

tests/cpu_hip holds a CPU stand-in for the part of the HIP runtime the
sources use (hip/hip_runtime.h, hip_cpu_runtime.cpp: one OS thread per GPU
thread, __syncthreads as a barrier).  g++ builds lbm_api.hip, lbm_kernels.hip
and lbm_adjoint.hip with it into a shared library; tests/cpu_hip/driver.py
runs the step and the adjoint step through the same C ABI with host arrays
as device memory, in a subprocess that preloads the sanitizer runtime.  Any
out-of-bounds or use-after-free access in a kernel aborts that subprocess
with a report; the results must also match the oracle:
  * forward: 6 steps, every force form, the boundary set-ups (periodic,
    moving y-walls, walls on both axes with gravity) in turn, phi and u
    within 1e-6 relative;
  * adjoint: one adjoint step against the oracle's vector-Jacobian product
    for every force form on each of the three set-ups, lambda within 1e-6, dL/dsigma and dL/dM within
    1e-6 relative.
"""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "cpu_hip")
OUT = os.path.join(ROOT, "_build", "cpu_harness")
SOURCES = ("lbm_api.hip", "lbm_kernels.hip", "lbm_adjoint.hip")
FLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "-fsanitize=address", "-fno-omit-frame-pointer", "-Wno-attributes",
         "-Wno-unknown-pragmas", "-I", HARNESS]


def _asan_runtime():
    gxx = shutil.which("g++")
    if gxx is None:
        return None
    r = subprocess.run([gxx, "-print-file-name=libasan.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def cpu_lib():
    if _asan_runtime() is None:
        pytest.skip("g++ with AddressSanitizer is not available")
    os.makedirs(OUT, exist_ok=True)
    csrc = os.path.join(ROOT, "paper_2012_14729_amd", "csrc")
    jobs = [(os.path.join(HARNESS, "hip_cpu_runtime.cpp"), os.path.join(OUT, "rt.o"), [])]
    jobs += [(os.path.join(csrc, s), os.path.join(OUT, s + ".o"), ["-x", "c++"]) for s in SOURCES]
    procs = [(src, subprocess.Popen(["g++", *FLAGS, *lang, "-c", src, "-o", obj], stdout=subprocess.PIPE,
                                    stderr=subprocess.PIPE, text=True)) for src, obj, lang in jobs]
    for src, p in procs:
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, f"g++ failed on {src}:\n{err}"
    lib = os.path.join(OUT, "libpflbm_cpu.so")
    r = subprocess.run(["g++", "-shared", "-fsanitize=address", *[o for _, o, _ in jobs], "-o", lib, "-lpthread"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    return lib


def _run(lib, what):
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, os.path.join(HARNESS, "driver.py"), lib, what], capture_output=True,
                       text=True, env=env, timeout=1200)
    assert r.returncode == 0 and "DONE" in r.stdout, f"driver failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    assert "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    return [json.loads(line) for line in r.stdout.splitlines() if line.startswith("{")]


def test_cpu_build_of_the_step_matches_the_oracle(cpu_lib):
    rows = _run(cpu_lib, "forward")
    assert len(rows) == 8
    for r in rows:
        assert r["phi"] < 1e-6 and r["u"] < 1e-6, r


def test_cpu_build_of_the_adjoint_matches_the_oracle_vjp(cpu_lib):
    rows = _run(cpu_lib, "adjoint")
    assert len(rows) == 24
    for r in rows:
        assert r["lambda"] < 1e-6, r
        for key in ("dsigma", "dM"):
            got, ref = r[key]
            assert abs(got - ref) <= 1e-6 * abs(ref) + 1e-12, r
