"""Pins of the oracle's per-node algebra against the moment conditions the
paper's scheme must satisfy (arXiv:2012.14729, Sec. III).

The equilibria and forcing terms of Eqs. (31)-(36) are built so that the
macroscopic relations of Eq. (37) and the recovered equations (38)-(40) hold.
These tests evaluate the oracle's functions on random node data and check the
moments against those relations -- a dropped term, a wrong sign or a wrong
index in any of the per-direction formulas breaks one of them.
"""
import math

import pytest
import torch

from oracle import lbm_ref as R

torch.set_default_dtype(torch.float64)
N = 200


@pytest.fixture
def nodes():
    g = torch.Generator().manual_seed(1234)
    r = lambda s=1.0: s * torch.randn(N, generator=g)
    return dict(P=r(1e-3), rho=1.0 + torch.rand(N, generator=g) * 9.0, ux=r(0.05), uy=r(0.05),
                phi=torch.rand(N, generator=g) * 2 - 1, mu=r(1e-3), fx=r(1e-4), fy=r(1e-4),
                grx=r(0.1), gry=r(0.1), eta=0.7, divq=r(1e-3), dqx=r(1e-4), dqy=r(1e-4), a_h=0.37)


def moments(vals):
    m0 = sum(vals)
    mx = sum(R.CX[i] * vals[i] for i in range(9))
    my = sum(R.CY[i] * vals[i] for i in range(9))
    mxx = sum(R.CX[i] ** 2 * vals[i] for i in range(9))
    mxy = sum(R.CX[i] * R.CY[i] * vals[i] for i in range(9))
    myy = sum(R.CY[i] ** 2 * vals[i] for i in range(9))
    return m0, mx, my, mxx, mxy, myy


def close(a, b, tol=1e-13):
    a = torch.as_tensor(a, dtype=torch.float64)
    b = torch.as_tensor(b, dtype=torch.float64) + 0 * a
    scale = max(1.0, float(b.abs().max()))
    assert float((a - b).abs().max()) <= tol * scale, float((a - b).abs().max())


def test_lattice_tables():
    """D2Q9 of Eq. (34): weights sum to 1, first moment 0, second moment cs^2 I,
    fourth moment cs^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)."""
    assert math.isclose(sum(R.WT), 1.0, abs_tol=1e-15)
    for a in (R.CX, R.CY):
        assert abs(sum(R.WT[i] * a[i] for i in range(9))) < 1e-15
    assert math.isclose(sum(R.WT[i] * R.CX[i] ** 2 for i in range(9)), R.CS2, abs_tol=1e-15)
    assert abs(sum(R.WT[i] * R.CX[i] * R.CY[i] for i in range(9))) < 1e-15
    assert math.isclose(sum(R.WT[i] * R.CX[i] ** 4 for i in range(9)), 3 * R.CS2 ** 2, abs_tol=1e-15)
    assert math.isclose(sum(R.WT[i] * R.CX[i] ** 2 * R.CY[i] ** 2 for i in range(9)), R.CS2 ** 2, abs_tol=1e-15)
    for i in range(9):
        j = R.OPP[i]
        assert (R.CX[j], R.CY[j]) == (-R.CX[i], -R.CY[i])


def test_modified_weights():
    """Sum wbar = sum wbar c = 0 and sum wbar c c = cs^2 I  (Sec. III, after Eq. 36)."""
    m0, mx, my, mxx, mxy, myy = moments(list(R.WBAR))
    assert abs(m0) < 1e-15 and abs(mx) < 1e-15 and abs(my) < 1e-15
    assert math.isclose(mxx, R.CS2, abs_tol=1e-15) and math.isclose(myy, R.CS2, abs_tol=1e-15)
    assert abs(mxy) < 1e-15


def test_feq_moments(nodes):
    """sum f^eq = P_sf, sum c f^eq = cs^2 rho u  (consistent with Eq. 37)."""
    n = nodes
    feq = [R.f_eq(i, n["P"], n["rho"], n["ux"], n["uy"]) for i in range(9)]
    m0, mx, my, mxx, mxy, myy = moments(feq)
    close(m0, n["P"])
    close(mx, R.CS2 * n["rho"] * n["ux"])
    close(my, R.CS2 * n["rho"] * n["uy"])
    # second moment: P I + cs^2 rho u u (pressure-based equilibrium)
    close(mxx, R.CS2 * n["P"] + R.CS2 * n["rho"] * n["ux"] ** 2)
    close(mxy, R.CS2 * n["rho"] * n["ux"] * n["uy"])


def test_heq_moments(nodes):
    """sum h^eq = phi, sum c h^eq = phi u, sum c c h^eq = cs^2 eta mu I  (Eq. 32)."""
    n = nodes
    heq = [R.h_eq(i, n["phi"], n["mu"], n["ux"], n["uy"], n["eta"]) for i in range(9)]
    m0, mx, my, mxx, mxy, myy = moments(heq)
    close(m0, n["phi"])
    close(mx, n["phi"] * n["ux"])
    close(my, n["phi"] * n["uy"])
    close(mxx, R.CS2 * n["eta"] * n["mu"])
    close(myy, R.CS2 * n["eta"] * n["mu"])
    close(mxy, 0.0)


def test_flow_forcing_moments(nodes):
    """sum F_i = cs^2 u.grad(rho) and sum c_i F_i = cs^2 (F_sf + F_g): the two
    relations the corrections of Eq. (37) (pressure and velocity) rely on."""
    n = nodes
    Fi = [R.force_f(i, n["ux"], n["uy"], n["fx"], n["fy"], n["grx"], n["gry"]) for i in range(9)]
    m0, mx, my, *_ = moments(Fi)
    close(m0, R.CS2 * (n["ux"] * n["grx"] + n["uy"] * n["gry"]))
    close(mx, R.CS2 * n["fx"])
    close(my, R.CS2 * n["fy"])


def test_literal_gamma_reading_fails_zeroth_moment(nodes):
    """Reading A1: with Gamma_i = w_i + s_i (as printed) the zeroth moment of
    F_i would not equal cs^2 u.grad(rho); the oracle uses w_i (1 + s_i)."""
    n = nodes
    vals = []
    for i in range(9):
        s = R.s_i(i, n["ux"], n["uy"])
        gam = R.WT[i] + s
        vals.append((R.CX[i] - n["ux"]) * (gam * n["fx"] + s * R.CS2 * n["grx"])
                    + (R.CY[i] - n["uy"]) * (gam * n["fy"] + s * R.CS2 * n["gry"]))
    m0 = sum(vals)
    target = R.CS2 * (n["ux"] * n["grx"] + n["uy"] * n["gry"])
    assert float((m0 - target).abs().max()) > 1e-6


def test_ch_forcing_moments(nodes):
    """sum H_i = 0 (phi conserved) and sum c_i H_i = d_t(phi u)  (Eq. 36)."""
    n = nodes
    Hi = [R.force_h(i, n["a_h"], n["divq"], n["dqx"], n["dqy"]) for i in range(9)]
    m0, mx, my, mxx, mxy, myy = moments(Hi)
    close(m0, 0.0)
    close(mx, n["dqx"])
    close(my, n["dqy"])
    # second moment carries the div(phi u) correction: sum c c H = cs^2 A_H div(phi u) I
    close(mxx, R.CS2 * n["a_h"] * n["divq"])


def test_liang_special_case():
    """tau_h = 1/2 + sqrt(3)/6 makes tau_2 vanish, so the first term of Eq. (36)
    drops out (Sec. III, after Eq. 36)."""
    p = R.Params(nx=8, ny=8, tau_h=0.5 + math.sqrt(3) / 6)
    assert abs(R.constants(p).a_h) < 1e-14


def test_transport_coefficients():
    """mu = rho cs^2 (tau_f - 1/2) and M = cs^2 eta (tau_h - 1/2) (after Eq. 40)."""
    p = R.Params(nx=8, ny=8, rho1=7.0, rho2=2.0, nu1=0.05, nu2=0.3, M=0.02, tau_h=0.9)
    c = R.constants(p)
    for phi in (-1.0, -0.3, 0.4, 1.0):
        phi_t = torch.tensor(phi)
        rho = R.density(phi_t, p)
        mu = R.viscosity(phi_t, c)
        close(rho * R.CS2 * (R.tau_f(phi_t, p, c) - 0.5), mu)
    close(R.CS2 * c.eta * (p.tau_h - 0.5), p.M)
    close(R.density(torch.tensor(1.0), p), p.rho1)
    close(R.density(torch.tensor(-1.0), p), p.rho2)


def test_surface_tension_and_dirac_quadratures():
    """sigma = kappa int |phi'|^2 dr = (4/3) sqrt(2 beta kappa) for the tanh
    profile of Eq. (4) with beta, kappa from Eq. (6); Dirac normalisations of
    CSF-1 (alpha = 3W/8 on |grad phi|^2) and CSF-2 (alpha = 1/2 on |grad phi|)
    integrate to one (Appendix B)."""
    sigma, W = 0.37, 4.5
    p = R.Params(nx=8, ny=8, sigma=sigma, W=W)
    c = R.constants(p)
    r = torch.linspace(-40 * W, 40 * W, 400001)
    dr = float(r[1] - r[0])
    phi = torch.tanh(math.sqrt(2 * c.beta / c.kappa) * r)
    assert math.isclose(math.sqrt(c.kappa / (2 * c.beta)), W / 2, rel_tol=1e-14)
    dphi = (1 - phi ** 2) * math.sqrt(2 * c.beta / c.kappa)
    f0 = c.beta * (1 - phi ** 2) ** 2
    s_energy = float(torch.trapezoid(f0 + 0.5 * c.kappa * dphi ** 2, dx=dr))
    s_grad = float(torch.trapezoid(c.kappa * dphi ** 2, dx=dr))
    assert math.isclose(s_energy, sigma, rel_tol=1e-8)
    assert math.isclose(s_grad, sigma, rel_tol=1e-8)
    assert math.isclose(4.0 / 3.0 * math.sqrt(2 * c.beta * c.kappa), sigma, rel_tol=1e-14)
    assert math.isclose(float(torch.trapezoid(3 * W / 8 * dphi ** 2, dx=dr)), 1.0, rel_tol=1e-8)
    assert math.isclose(float(torch.trapezoid(0.5 * dphi, dx=dr)), 1.0, rel_tol=1e-8)
