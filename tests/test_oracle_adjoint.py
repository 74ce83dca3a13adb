"""Pins of the oracle's adjoint (torch autograd through the FP64 oracle) for
the misfit L = 1/2 sum (phi_T - phi*)^2 (reading A19): dL/dsigma, dL/dM and
dL/dphi0 against FP64 central finite differences (h = 1e-6 relative) and,
for sigma, against a complex-step derivative (every step is analytic under
readings A8 and A9)."""
import numpy as np
import pytest
import torch

import workloads as WL
from oracle import lbm_ref as R

torch.set_default_dtype(torch.float64)
T = 40


def setup(form):
    p, phi0, ux0, uy0 = WL.config_shear(nx=32, ny=16, R=4.0, Re=1.0, Ca=0.2)
    d = p.as_dict()
    d["rho0"] = None
    base = R.Params(**d)
    t = lambda a: torch.tensor(np.asarray(a, np.float32), dtype=torch.float64)
    phi0, ux0, uy0 = t(phi0), t(ux0), t(uy0)
    with torch.no_grad():
        q = R.Params(**{**base.__dict__, "sigma": base.sigma * 1.1})
        target = R.run(R.init(q, phi0, ux0, uy0), form, q, T)["h"].sum(0)
    return base, phi0, ux0, uy0, target


def loss(base, sigma, M, phi0, ux0, uy0, target, form):
    q = R.Params(**{**base.__dict__, "sigma": sigma, "M": M})
    phi = R.run(R.init(q, phi0, ux0, uy0), form, q, T)["h"].sum(0)
    return 0.5 * ((phi - target) ** 2).sum()


@pytest.mark.parametrize("form", ["stf2", "cpf1", "csf2"])
def test_autograd_matches_finite_differences(form):
    base, phi0, ux0, uy0, target = setup(form)
    s = torch.tensor(base.sigma, requires_grad=True)
    m = torch.tensor(base.M, requires_grad=True)
    ph = phi0.clone().requires_grad_(True)
    loss(base, s, m, ph, ux0, uy0, target, form).backward()
    with torch.no_grad():
        hs, hm = 1e-6 * base.sigma, 1e-6 * base.M
        fs = (loss(base, base.sigma + hs, base.M, phi0, ux0, uy0, target, form)
              - loss(base, base.sigma - hs, base.M, phi0, ux0, uy0, target, form)) / (2 * hs)
        fm = (loss(base, base.sigma, base.M + hm, phi0, ux0, uy0, target, form)
              - loss(base, base.sigma, base.M - hm, phi0, ux0, uy0, target, form)) / (2 * hm)
        e = torch.zeros_like(phi0)
        e[2, 13] = 1.0   # a node next to the moving wall
        fp = (loss(base, base.sigma, base.M, phi0 + 1e-6 * e, ux0, uy0, target, form)
              - loss(base, base.sigma, base.M, phi0 - 1e-6 * e, ux0, uy0, target, form)) / 2e-6
    assert abs(float(s.grad) - float(fs)) <= 1e-6 * abs(float(fs))
    assert abs(float(m.grad) - float(fm)) <= 1e-6 * abs(float(fm))
    assert abs(float(ph.grad[2, 13]) - float(fp)) <= 1e-6 * abs(float(fp)) + 1e-12


def test_complex_step_sigma():
    form = "csf1"
    base, phi0, ux0, uy0, target = setup(form)
    s = torch.tensor(base.sigma, requires_grad=True)
    loss(base, s, base.M, phi0, ux0, uy0, target, form).backward()
    h = 1e-20 * base.sigma
    c = lambda a: a.to(torch.complex128)
    q = R.Params(**{**base.__dict__, "sigma": complex(base.sigma, h)})
    phi = R.run(R.init(q, c(phi0), c(ux0), c(uy0)), form, q, T)["h"].sum(0)
    L = 0.5 * ((phi - c(target)) ** 2).sum()
    cs = L.imag.item() / h
    assert abs(float(s.grad) - cs) <= 1e-10 * abs(cs)
