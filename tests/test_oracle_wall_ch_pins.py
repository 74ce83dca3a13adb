"""Pins of two terms of the oracle that conservation and the brute-force
twin cannot see, fixed by the mathematics of the method (arXiv:2012.14729):

* the moving-wall term of the order-parameter bounce-back (Sec. IV, Eq. 43,
  second line).  Its corrections come in opposite pairs along a flat wall,
  so they cancel in sum_i h_i (phi is blind to their sign and size), but
  not in the first moment sum_i c_i h_i, the flux of phi.  In steady plane
  Couette flow of a uniform phase (phi constant, so mu_phi is constant and
  div(phi u) = d_t(phi u) = 0) the order-parameter equation is pure
  advection and its flux is exactly phi u at every node, the wall rows
  included (half-way bounce-back is exact for the linear profile);
* the A_H div(phi u) term of the order-parameter forcing (Eq. 36, with
  A_H = 3 tau_2/(tau_h tau_1)).  With sigma = 0 (mu_phi = 0) and a uniform
  velocity the order-parameter equation reduces to pure advection, whose
  exact solution is the translated initial field.  The scheme's remaining
  error is dispersive; the printed A_H term removes part of it, so the
  printed coefficient must do measurably better than the term dropped or
  with its sign flipped.

Each pin is checked to fail on a planted mistake (a flipped sign) in the
oracle, on the CPU.
"""
import math

import pytest
import torch

from oracle import lbm_ref as R
from oracle.brute import Brute

torch.set_default_dtype(torch.float64)


def _couette_params(axis, U, nx, ny):
    if axis == "y":   # walls at y = -1/2 (-U) and ny - 1/2 (+U), moving along x
        return R.Params(nx=nx, ny=ny, wall_y=1, u_wall_lo=-U, u_wall_hi=U, rho1=1.0, rho2=1.0, nu1=0.1, nu2=0.1,
                        sigma=0.01, W=4.0, M=0.1, tau_h=0.8)
    return R.Params(nx=nx, ny=ny, wall_x=1, u_wall_lo=-U, u_wall_hi=U, rho1=1.0, rho2=1.0, nu1=0.1, nu2=0.1,
                    sigma=0.01, W=4.0, M=0.1, tau_h=0.8)


def _couette_profile(axis, U, nx, ny):
    y, x = torch.meshgrid(torch.arange(ny, dtype=torch.float64), torch.arange(nx, dtype=torch.float64),
                          indexing="ij")
    if axis == "y":
        return U * (2.0 * (y + 0.5) / ny - 1.0), torch.zeros(ny, nx)
    return torch.zeros(ny, nx), U * (2.0 * (x + 0.5) / nx - 1.0)


def _flux_error(f, h, phi_val, ux, uy):
    """max |sum_i c_i h_i - phi u| over the lattice, both components."""
    hx = sum(R.CX[i] * h[i] for i in range(9))
    hy = sum(R.CY[i] * h[i] for i in range(9))
    return max(float((hx - phi_val * ux).abs().max()), float((hy - phi_val * uy).abs().max()))


class _FlipHWallTerm:
    """Planted mistake: the order-parameter wall term of Eq. (43) with its
    sign flipped (the oracle streams f, then h, once per step)."""

    def __enter__(self):
        self.orig = R._stream
        calls = [0]

        def patched(post, wall_value, p):
            calls[0] += 1
            if calls[0] % 2 == 0:
                return self.orig(post, lambda i, cu: -wall_value(i, cu), p)
            return self.orig(post, wall_value, p)

        R._stream = patched
        return self

    def __exit__(self, *exc):
        R._stream = self.orig


def _couette_flux_error(axis, phi_val, U=0.01, nx=12, ny=16, steps=400):
    if axis == "x":
        nx, ny = ny, nx
    p = _couette_params(axis, U, nx, ny)
    ux0, uy0 = _couette_profile(axis, U, nx, ny)
    st = R.init(p, torch.full((ny, nx), phi_val), ux0, uy0)
    st = R.run(st, "cpf2", p, steps)
    m = R.moments(st, "cpf2", p)
    # the flow itself is the exact Couette profile (f is not affected by h)
    assert float((m["ux"] - ux0).abs().max()) < 1e-12 * U + 1e-15
    assert float((m["uy"] - uy0).abs().max()) < 1e-12 * U + 1e-15
    return _flux_error(st["f"], st["h"], phi_val, m["ux"], m["uy"]) / U


@pytest.mark.parametrize("axis", ["y", "x"])
@pytest.mark.parametrize("phi_val", [1.0, -1.0, 0.3])
def test_order_parameter_flux_at_moving_walls(axis, phi_val):
    assert _couette_flux_error(axis, phi_val) < 1e-12


@pytest.mark.parametrize("axis", ["y", "x"])
def test_flux_pin_fails_with_flipped_wall_term(axis):
    with _FlipHWallTerm():
        err = _couette_flux_error(axis, 1.0, steps=40)
    # the two corrected links carry 2 * 6 w phi c.u_w each: 2/3 of phi U
    assert err > 0.5


@pytest.mark.parametrize("axis", ["y", "x"])
def test_brute_force_twin_meets_the_flux_pin(axis):
    """The independent per-cell stepper satisfies the same pin."""
    U, nx, ny, phi_val = 0.01, 8, 10, 1.0
    if axis == "x":
        nx, ny = ny, nx
    wx, wy = (0, 1) if axis == "y" else (1, 0)
    ux0, uy0 = _couette_profile(axis, U, nx, ny)
    b = Brute(nx, ny, wx, wy, -U, U, 1.0, 1.0, 0.1, 0.1, 0.01, 4.0, 0.1, 0.8, 0.0, 0.0)
    f, h, J = b.init([[phi_val] * nx for _ in range(ny)], ux0.tolist(), uy0.tolist())
    for _ in range(30):
        f, h, J = b.step(f, h, J, "cpf2")
    mb = b.moments(f, h, "cpf2")
    err = _flux_error(None, torch.tensor(h), phi_val, torch.tensor(mb["ux"]), torch.tensor(mb["uy"]))
    assert err / U < 1e-12


def _advection_error(tau_h, a_h_scale, nx=32, ny=2, U=0.05, amp=0.5):
    """Max error, relative to the amplitude, of a sine advected once across
    the periodic lattice at uniform velocity U with sigma = 0, against the
    exact translated field (which after one period is the initial field)."""
    p = R.Params(nx=nx, ny=ny, rho1=1.0, rho2=1.0, nu1=0.1, nu2=0.1, sigma=0.0, W=4.0, M=0.1, tau_h=tau_h)
    x = torch.arange(nx, dtype=torch.float64).view(1, nx).expand(ny, nx)
    phi0 = amp * torch.sin(2.0 * math.pi * x / nx)
    st = R.init(p, phi0, torch.full_like(phi0, U), torch.zeros_like(phi0))
    orig = R.constants

    def scaled(pp):
        c = orig(pp)
        c.a_h = c.a_h * a_h_scale
        return c

    R.constants = scaled
    try:
        st = R.run(st, "cpf2", p, int(round(nx / U)))
    finally:
        R.constants = orig
    m = R.moments(st, "cpf2", p)
    assert float((m["ux"] - U).abs().max()) < 1e-13 and float(m["uy"].abs().max()) < 1e-13   # sigma = 0: u stays uniform
    return float((st["h"].sum(0) - phi0).abs().max()) / amp


@pytest.mark.parametrize("tau_h", [0.8, 1.0, 1.2])
def test_a_h_term_reduces_the_advection_error(tau_h):
    printed = _advection_error(tau_h, 1.0)
    dropped = _advection_error(tau_h, 0.0)
    flipped = _advection_error(tau_h, -1.0)
    assert printed < 0.65 * dropped, (printed, dropped)
    assert printed < 0.5 * flipped, (printed, flipped)


def test_advection_translates_the_field():
    """At tau_h = 1 (A_H = 1) one period of advection over 32 nodes keeps the
    sine within 2.5 % of its amplitude (second order in the grid spacing)."""
    assert _advection_error(1.0, 1.0) < 0.025
    assert _advection_error(1.0, 1.0, nx=64) < 0.3 * _advection_error(1.0, 1.0)
