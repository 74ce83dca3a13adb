"""Closed-form references of the Sec. V benchmarks (host side, NumPy/SciPy).

capillary_wave: the amplitude of a small standing wave on the interface
between two viscous fluids of equal kinematic viscosity released from rest
(Sec. V.C, Eqs. 44-46):

    h(t)/h0 = 4 (1 - 4 b) nu^2 k^4 / (8 (1 - 4 b) nu^2 k^4 + w0^2) erfc(sqrt(nu k^2 t))
            + sum_i  z_i / Z_i  *  w0^2 / (z_i^2 - nu k^2)  *  exp((z_i^2 - nu k^2) t) erfc(z_i sqrt(t))

with b = rho1 rho2 / (rho1 + rho2)^2, w0^2 = sigma k^3 / (rho1 + rho2), z_i the
four roots of

    z^4 - 4 b sqrt(nu k^2) z^3 + 2 (1 - 6 b) nu k^2 z^2 + 4 (1 - 3 b) (nu k^2)^(3/2) z
        + (1 - 4 b) nu^2 k^4 + w0^2 = 0

and Z_i = prod_{j != i} (z_j - z_i).  The product exp(z^2 t) erfc(z sqrt(t)) is
evaluated as the Faddeeva function w(i z sqrt(t)), which stays finite where
the two factors separately overflow.

capillary_error: the time-averaged L2 error of Eq. (47) over 0 <= t <= 25 / w0.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc, wofz


def capillary_wave(t, nu: float, k: float, rho1: float, rho2: float, sigma: float):
    """h(t) / h0 at the times t (array-like, same time unit as nu and sigma)."""
    t = np.asarray(t, dtype=np.float64)
    b = rho1 * rho2 / (rho1 + rho2) ** 2
    w02 = sigma * k ** 3 / (rho1 + rho2)
    nk2 = nu * k * k
    coeffs = [1.0, -4.0 * b * math.sqrt(nk2), 2.0 * (1.0 - 6.0 * b) * nk2, 4.0 * (1.0 - 3.0 * b) * nk2 ** 1.5,
              (1.0 - 4.0 * b) * nk2 * nk2 + w02]
    z = np.roots(coeffs).astype(np.complex128)
    first = 4.0 * (1.0 - 4.0 * b) * nk2 * nk2 / (8.0 * (1.0 - 4.0 * b) * nk2 * nk2 + w02)
    h = first * erfc(np.sqrt(nk2 * t))
    decay = np.exp(-nk2 * t)
    st = np.sqrt(t)
    for i in range(4):
        Zi = np.prod([z[j] - z[i] for j in range(4) if j != i])
        h = h + (z[i] / Zi * w02 / (z[i] ** 2 - nk2) * decay * wofz(1j * z[i] * st)).real
    return h


def capillary_frequency(k: float, rho1: float, rho2: float, sigma: float) -> float:
    """Inviscid angular frequency w0 = sqrt(sigma k^3 / (rho1 + rho2))."""
    return math.sqrt(sigma * k ** 3 / (rho1 + rho2))


def capillary_error(t, h, nu: float, k: float, rho1: float, rho2: float, sigma: float) -> float:
    """E2 of Eq. (47): sqrt((w0 / 25) int_0^{25 / w0} |h(t) - h_exact(t)|^2 dt)
    for sampled normalised amplitudes h(t) (trapezoidal rule over the samples,
    which must cover [0, 25 / w0])."""
    t = np.asarray(t, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    w0 = capillary_frequency(k, rho1, rho2, sigma)
    t_end = 25.0 / w0
    if t[0] > 1e-12 * t_end or t[-1] < t_end * (1.0 - 1e-9):
        raise ValueError("samples must cover [0, 25 / w0]")
    keep = t < t_end
    # close the interval at t_end, interpolating the sampled amplitude
    h_end = float(np.interp(t_end, t, h))
    t, h = np.append(t[keep], t_end), np.append(h[keep], h_end)
    d2 = (h - capillary_wave(t, nu, k, rho1, rho2, sigma)) ** 2
    return math.sqrt(w0 / 25.0 * float(np.trapezoid(d2, t)))
