"""Pins of the closed-form capillary-wave amplitude (Sec. V.C, Eqs. 44-46)
against what the solution must satisfy whatever its algebra: the wave
starts at h0 from rest, it oscillates as cos(w0 t) when the viscosity
vanishes, and the quartic's roots are roots."""
import math

import numpy as np
import pytest

from paper_2012_14729_amd import theory as T

K = 2 * math.pi
SIG = 0.25


@pytest.mark.parametrize("rho2", [1.0, 0.1])
@pytest.mark.parametrize("nu", [0.01, 0.05])
def test_released_from_rest_at_unit_amplitude(rho2, nu):
    h0 = T.capillary_wave([0.0], nu, K, 1.0, rho2, SIG)[0]
    assert abs(h0 - 1.0) < 1e-10
    w0 = T.capillary_frequency(K, 1.0, rho2, SIG)
    dt = 1e-7 / w0
    assert abs(T.capillary_wave([dt], nu, K, 1.0, rho2, SIG)[0] - 1.0) / (w0 * dt) < 1e-4   # dh/dt(0) = 0


@pytest.mark.parametrize("rho2", [1.0, 0.1])
def test_inviscid_limit_is_the_linear_capillary_wave(rho2):
    w0 = T.capillary_frequency(K, 1.0, rho2, SIG)
    t = np.linspace(0.0, 3 * 2 * math.pi / w0, 200)
    h = T.capillary_wave(t, 1e-10, K, 1.0, rho2, SIG)
    assert np.abs(h - np.cos(w0 * t)).max() < 2e-3


def test_viscosity_damps_and_the_error_norm_vanishes_on_the_exact_curve():
    nu = 0.01
    w0 = T.capillary_frequency(K, 1.0, 1.0, SIG)
    t = np.linspace(0.0, 25.0 / w0, 2001)
    h = T.capillary_wave(t, nu, K, 1.0, 1.0, SIG)
    assert np.abs(h[-200:]).max() < 0.1 < np.abs(h[:200]).max()
    assert T.capillary_error(t, h, nu, K, 1.0, 1.0, SIG) < 1e-12
    assert abs(T.capillary_error(t, h + 0.01, nu, K, 1.0, 1.0, SIG) - 0.01) < 1e-6


@pytest.mark.parametrize("h0", [0.0, -0.01, 0.5])
def test_capillary_benchmark_rejects_amplitudes_outside_the_box(h0):
    """The benchmark validates its amplitude before touching the GPU."""
    from paper_2012_14729_amd.benchmarks import capillary_wave
    with pytest.raises(ValueError):
        capillary_wave("stf2", H=16, h0=h0)
