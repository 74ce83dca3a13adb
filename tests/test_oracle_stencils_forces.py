"""Pins of the oracle's difference operators and interfacial forces.

* The isotropic stencils of Eqs. (41)-(42) are exact on low-order
  polynomials (gradient on quadratics, Laplacian on cubics).
* Each of the eight discrete interfacial forces (Eqs. 17, 18, 20, 24, 25)
  converges at second order to its continuum value, computed here from exact
  derivatives of a smooth, non-symmetric test field and written in an
  expanded form (not the divergence/gradient form the oracle uses).
* On a radial tanh profile F_stf-2, F_cpf-2 and F_csf-1 converge to each
  other (Sec. II.B, Eq. 28).
"""
import math

import pytest
import torch

from oracle import lbm_ref as R

torch.set_default_dtype(torch.float64)


def grid(n, m, x0=-3.0, y0=5.0):
    y, x = torch.meshgrid(torch.arange(m) + y0, torch.arange(n) + x0, indexing="ij")
    return x, y


def test_gradient_exact_on_quadratics():
    x, y = grid(12, 10)
    e = 0.3 + 1.7 * x - 0.9 * y + 0.25 * x * x - 0.4 * x * y + 0.6 * y * y
    gx, gy = R.grad(e)
    xi, yi = x[1:-1, 1:-1], y[1:-1, 1:-1]
    assert torch.allclose(gx, 1.7 + 0.5 * xi - 0.4 * yi, atol=1e-12, rtol=0)
    assert torch.allclose(gy, -0.9 - 0.4 * xi + 1.2 * yi, atol=1e-12, rtol=0)


def test_laplacian_exact_on_cubics():
    x, y = grid(12, 10)
    e = x * x + y * y
    assert torch.allclose(R.lap(e), torch.full_like(R.lap(e), 4.0), atol=1e-11, rtol=0)
    e = 0.5 * x ** 3 - 0.2 * x * x * y + 0.7 * y ** 3 + 0.1 * x * y
    xi, yi = x[1:-1, 1:-1], y[1:-1, 1:-1]
    assert torch.allclose(R.lap(e), 3.0 * xi - 0.4 * yi + 4.2 * yi, atol=1e-10, rtol=0)


def test_divergence_exact_on_quadratic_fields():
    x, y = grid(9, 11)
    vx = 0.2 * x * x - 0.5 * x * y + y
    vy = -0.3 * y * y + 0.8 * x * y - x
    d = R.div(vx, vy)
    xi, yi = x[1:-1, 1:-1], y[1:-1, 1:-1]
    assert torch.allclose(d, 0.4 * xi - 0.5 * yi - 0.6 * yi + 0.8 * xi, atol=1e-12, rtol=0)


# ----------------------------------------------------------------------------
# Manufactured solution for the eight forces
# ----------------------------------------------------------------------------
def field(X, Y):
    """Smooth test field without x<->y symmetry.  phi = 0.9 tanh(q) + 0.05 with
    dq/dX >= 0.3 on the window |X|, |Y| <= 3, so grad(phi) never vanishes and
    the interface normal grad(q)/|grad(q)| is smooth."""
    q = 0.6 * X + 0.3 * Y + 0.15 * torch.sin(0.7 * Y) * torch.cos(0.4 * X) + 0.08 * X * Y - 0.1
    return 0.9 * torch.tanh(q) + 0.05


def exact_derivatives(X, Y):
    X = X.clone().requires_grad_(True)
    Y = Y.clone().requires_grad_(True)
    phi = field(X, Y)
    gx, gy = torch.autograd.grad(phi.sum(), (X, Y), create_graph=True)
    gxx, gxy = torch.autograd.grad(gx.sum(), (X, Y), create_graph=True)
    _, gyy = torch.autograd.grad(gy.sum(), (X, Y), create_graph=True)
    L = gxx + gyy
    Lx, Ly = torch.autograd.grad(L.sum(), (X, Y), create_graph=True)
    return {k: v.detach() for k, v in dict(phi=phi, gx=gx, gy=gy, gxx=gxx, gxy=gxy, gyy=gyy, L=L, Lx=Lx, Ly=Ly).items()}


def continuum_force(form, d, beta, kappa, sigma, eps):
    gx, gy, gxx, gxy, gyy, L = d["gx"], d["gy"], d["gxx"], d["gxy"], d["gyy"], d["L"]
    phi = d["phi"]
    adv_x = gx * gxx + gy * gxy            # (grad phi . grad) grad phi
    adv_y = gx * gxy + gy * gyy
    if form == "stf1":
        return -kappa * (L * gx + adv_x), -kappa * (L * gy + adv_y)
    if form == "stf2":
        return kappa * (adv_x - L * gx), kappa * (adv_y - L * gy)
    mu = 4 * beta * phi * (phi * phi - 1) - kappa * L
    if form == "cpf1":
        dmu_x = 4 * beta * (3 * phi * phi - 1) * gx - kappa * d["Lx"]
        dmu_y = 4 * beta * (3 * phi * phi - 1) * gy - kappa * d["Ly"]
        return -phi * dmu_x, -phi * dmu_y
    if form == "cpf2":
        return mu * gx, mu * gy
    if form == "pf1":
        return -kappa * gx * L, -kappa * gy * L
    if form == "pf2":
        return kappa * phi * d["Lx"], kappa * phi * d["Ly"]
    s = torch.sqrt(gx * gx + gy * gy + eps * eps)
    hess_gg = gx * gx * gxx + 2 * gx * gy * gxy + gy * gy * gyy
    divn = L / s - hess_gg / s ** 3
    if form == "csf1":
        g2 = gx * gx + gy * gy
        return -kappa * g2 * gx / s * divn, -kappa * g2 * gy / s * divn
    return -0.5 * sigma * gx * divn, -0.5 * sigma * gy * divn


@pytest.mark.parametrize("form", R.FORMS)
def test_force_second_order_convergence(form):
    """Discrete force on phi(x/s) -> continuum force with relative error O(1/s^2)."""
    p = R.Params(nx=8, ny=8, sigma=0.02, W=4.0, eps_n=1e-6)
    c = R.constants(p)
    errs = []
    for s in (4.0, 8.0, 16.0):
        n = int(6 * s)
        xs, ys = grid(n + 4, n + 4, x0=-2, y0=-2)
        X, Y = (xs - n / 2) / s, (ys - n / 2) / s
        phie2 = field(X, Y)
        fx, fy = R.interfacial_force(phie2, form, p, c)
        d = exact_derivatives(X[2:-2, 2:-2], Y[2:-2, 2:-2])
        # scale derivatives from X to lattice coordinates (d/dx = (1/s) d/dX)
        sc = dict(phi=1, gx=1 / s, gy=1 / s, gxx=1 / s ** 2, gxy=1 / s ** 2, gyy=1 / s ** 2, L=1 / s ** 2,
                  Lx=1 / s ** 3, Ly=1 / s ** 3)
        d = {k: v * sc[k] for k, v in d.items()}
        ex, ey = continuum_force(form, d, c.beta, c.kappa, p.sigma, p.eps_n)
        scale = float(torch.maximum(ex.abs().max(), ey.abs().max()))
        errs.append(float(torch.maximum((fx - ex).abs().max(), (fy - ey).abs().max())) / scale)
    assert errs[-1] < 0.02, errs
    assert errs[0] > errs[1] > errs[2], errs
    assert 3.3 < errs[1] / errs[2] < 4.8, errs


def test_equivalent_forms_at_equilibrium():
    """On a radial equilibrium tanh profile F_stf-2 = F_cpf-2 = F_csf-1
    (Eq. 28); the discrete versions approach each other as W grows."""
    diffs = []
    for W in (4.0, 8.0, 16.0):
        Rr = 6 * W
        n = int(2 * Rr + 4 * W)
        p = R.Params(nx=n, ny=n, sigma=0.05, W=W)
        c = R.constants(p)
        xs, ys = grid(n + 4, n + 4, x0=-2, y0=-2)
        r = torch.sqrt((xs - n / 2 + 0.37) ** 2 + (ys - n / 2 + 0.21) ** 2)
        phie2 = torch.tanh(2 * (Rr - r) / W)
        f = {k: R.interfacial_force(phie2, k, p, c) for k in ("stf2", "cpf2", "csf1")}
        scale = float(torch.sqrt(f["csf1"][0] ** 2 + f["csf1"][1] ** 2).max())
        d = max(float(torch.sqrt((f[a][0] - f["csf1"][0]) ** 2 + (f[a][1] - f["csf1"][1]) ** 2).max())
                for a in ("stf2", "cpf2")) / scale
        diffs.append(d)
    # the three differ only by discretisation error, which falls as (dx/W)^2
    assert diffs[-1] < 0.08, diffs
    assert diffs[0] / diffs[1] > 3.5 and diffs[1] / diffs[2] > 3.5, diffs
