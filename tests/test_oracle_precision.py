"""The precision floor behind the kernels' storage format (CPU, oracle only).

The stationary droplet's velocity is the small residual of large, balanced
terms (Sec. V.A: max|u| of 4.5e-6 on the 64x64 droplet against |mu grad phi|
near 1.5e-4), so where rounding enters decides whether the 1e-5 parity bar on
u (relative to max|u|) can be met at all.  Runs of the oracle, 64x64 droplet,
CPF-1, 1000 steps, against the same run in float64:

- end to end in float32: e_u near 3e-3, far above the bar, so the kernels do
  their arithmetic in FP64;
- float64 with the populations f rounded to float32 after every step (what
  FP32 storage of f costs): e_u near 2e-6, inside the bar;
- float64 with the populations h rounded to float32 after every step (phi is
  their sum): e_u near 4e-4, so phi keeps an FP64 plane and slot 0 of h
  stores only the small deviation from phi.
"""
import numpy as np
import pytest
import torch

import workloads as WL
from oracle import lbm_ref as R

STEPS = 1000
FORM = "cpf1"
BAR = 1e-5


def _run(dtype, round_f=False, round_h=False):
    p, phi0, _, _ = WL.config_droplet64()
    d = p.as_dict()
    d["rho0"] = None
    op = R.Params(**d)
    st = R.init(op, torch.tensor(np.asarray(phi0, np.float32), dtype=dtype))
    for _ in range(STEPS):
        st = R.step(st, FORM, op)
        if round_f:
            st["f"] = st["f"].float().double()
        if round_h:
            st["h"] = st["h"].float().double()
    return {k: v.double().numpy() for k, v in R.moments(st, FORM, op).items()}


def _e_u(ref, got):
    umax = np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2).max()
    return max(np.abs(got["ux"] - ref["ux"]).max(), np.abs(got["uy"] - ref["uy"]).max()) / umax


@pytest.fixture(scope="module")
def reference():
    prev = torch.get_num_threads()
    torch.set_num_threads(min(prev, 4))
    try:
        yield _run(torch.float64)
    finally:
        torch.set_num_threads(prev)


def test_velocity_is_a_small_residual(reference):
    umax = np.sqrt(reference["ux"] ** 2 + reference["uy"] ** 2).max()
    print(f"[precision] max|u| after {STEPS} steps: {umax:.3e}", flush=True)
    assert 1e-6 < umax < 2e-5


def test_float32_arithmetic_misses_the_bar(reference):
    e = _e_u(reference, _run(torch.float32))
    print(f"[precision] oracle in float32: e_u = {e:.3e}", flush=True)
    assert e > 100 * BAR


def test_float32_storage_of_f_meets_the_bar(reference):
    e = _e_u(reference, _run(torch.float64, round_f=True))
    print(f"[precision] f rounded to float32 each step: e_u = {e:.3e}", flush=True)
    assert e < 0.5 * BAR


def test_float32_storage_of_h_misses_the_bar(reference):
    e = _e_u(reference, _run(torch.float64, round_h=True))
    print(f"[precision] h rounded to float32 each step: e_u = {e:.3e}", flush=True)
    assert e > 10 * BAR
