"""Pins of the oracle's hydrodynamic pressure p_h = P_sf - D_form
(arXiv:2012.14729, Sec. II.B, Eqs. 17-21 and 26).

At a planar interface in mechanical equilibrium the hydrodynamic pressure is
uniform, while the generalised pressure P_sf of a form with gradient terms
(STF-1, PF-1, PF-2) varies across the interface by about the size of those
terms.  Subtracting the form's D must therefore flatten the profile; a wrong
sign or a dropped factor in D makes it as uneven as P_sf or worse.  For the
chemical-potential forms D nearly vanishes at equilibrium, because
f0 = (kappa/2)|grad phi|^2 and mu_phi = 0 on the equilibrium profile (Eq. 27
and the text before it).  STF-2 and the CSF forms carry no gradient term:
there p_h is P_sf itself.
"""
import pytest
import torch

from oracle import lbm_ref as R

torch.set_default_dtype(torch.float64)

NX, NY, STEPS = 32, 4, 200


def slab_params():
    return R.Params(nx=NX, ny=NY, rho1=2.0, rho2=1.0, nu1=0.1, nu2=0.1, sigma=0.01, W=4.0, M=0.1, tau_h=0.8)


def slab_phi():
    """fluid 1 between x = 8 and x = 24 (two planar interfaces, periodic x)."""
    x = torch.arange(NX, dtype=torch.float64)
    row = -torch.tanh(2.0 * (x - 8.0) / 4.0) * torch.tanh(2.0 * (x - 24.0) / 4.0)
    return row.view(1, NX).expand(NY, NX).clone()


_cache = {}


def relaxed(form):
    if form not in _cache:
        p = slab_params()
        _cache[form] = (R.run(R.init(p, slab_phi()), form, p, STEPS), p)
    return _cache[form]


def spread(a):
    return float(a.max() - a.min())


@pytest.mark.parametrize("form,ratio", [("stf1", 0.4), ("pf1", 0.1), ("pf2", 0.4)])
def test_hydro_pressure_is_flat_across_planar_interface(form, ratio):
    st, p = relaxed(form)
    assert float(R.moments(st, form, p)["ux"].abs().max()) < 1e-4   # close to mechanical equilibrium
    P = R.moments(st, form, p)["P"]
    ph = R.hydro_pressure(st, form, p)
    assert spread(P) > 1e-3                   # the form's gradient terms show in P_sf
    assert spread(ph) < ratio * spread(P), (spread(ph), spread(P))


@pytest.mark.parametrize("form", ["cpf1", "cpf2"])
def test_chemical_potential_form_offset_vanishes_at_equilibrium(form):
    st, p = relaxed(form)
    c = R.constants(p)
    m = R.macroscopic(st["f"], st["h"], st["J"], st["rho0"], form, p, c)
    d = R.pressure_offset(m, form, c)
    half_grad_energy = 0.5 * c.kappa * (m["gx"] ** 2 + m["gy"] ** 2)
    # each of f0 and (kappa/2)|grad phi|^2 reaches ~1.6e-3 here; their sum or a
    # sign slip would leave D of that size
    assert float(half_grad_energy.max()) > 1e-3
    assert float(d.abs().max()) < 0.2 * float(half_grad_energy.max())


@pytest.mark.parametrize("form", ["stf2", "csf1", "csf2"])
def test_no_gradient_term_forms_report_psf(form):
    p = R.Params(nx=24, ny=20, rho1=5.0, rho2=1.0, sigma=0.01, W=4.0)
    yy, xx = torch.meshgrid(torch.arange(20.0), torch.arange(24.0), indexing="ij")
    phi0 = torch.tanh(2.0 * (6.0 - torch.sqrt((xx - 11.5) ** 2 + (yy - 9.5) ** 2)) / 4.0)
    st = R.run(R.init(p, phi0), form, p, 3)
    assert torch.equal(R.hydro_pressure(st, form, p), R.moments(st, form, p)["P"])


def test_offsets_match_their_definitions_on_random_fields():
    """D_form written out from Eq. (21) and reading A23 on random node values."""
    g = torch.Generator().manual_seed(7)
    m = {k: torch.randn(50, generator=g) * s for k, s in
         (("phi", 0.7), ("mu", 1e-3), ("gx", 0.2), ("gy", 0.2), ("lap", 0.05))}
    p = R.Params(nx=8, ny=8, sigma=0.02, W=3.0)
    c = R.constants(p)
    beta, kappa = 3 * 0.02 / (4 * 3.0), 3 * 3.0 * 0.02 / 8
    phi, g2 = m["phi"], m["gx"] ** 2 + m["gy"] ** 2
    f0 = beta * (phi ** 2 - 1) ** 2
    want = {
        "stf1": -kappa * g2,
        "stf2": 0 * g2,
        "cpf1": f0 - phi * m["mu"] - kappa * g2 / 2,
        "cpf2": f0 - kappa * g2 / 2,
        "pf1": -kappa * g2 / 2,
        "pf2": kappa * phi * m["lap"] - kappa * g2 / 2,
        "csf1": 0 * g2,
        "csf2": 0 * g2,
    }
    for form, w in want.items():
        assert torch.allclose(R.pressure_offset(m, form, c), w, rtol=1e-12, atol=1e-18), form


def test_cpf1_hydro_pressure_obeys_laplace_law():
    """Stationary droplet (Sec. V.A), CPF-1.  P_sf differs from p_h by
    -phi mu_phi, and mu_phi settles at a nonzero constant for a curved
    interface, so the jump of P_sf across the interface misses sigma / R by
    2 mu_phi (about 4 % here) while that of p_h meets it.  Flipping the sign
    of the phi mu_phi term moves p_h's jump 9 % off."""
    import math
    n, r = 32, 8.0
    p = R.Params(nx=n, ny=n, rho1=10.0, rho2=1.0, nu1=1 / 6, nu2=1 / 6, sigma=0.01, W=4.0, M=0.1)
    yy, xx = torch.meshgrid(torch.arange(float(n)), torch.arange(float(n)), indexing="ij")
    phi0 = torch.tanh(2.0 * (r - torch.sqrt((xx - n / 2) ** 2 + (yy - n / 2) ** 2)) / 4.0)
    st = R.run(R.init(p, phi0), "cpf1", p, 600)
    m = R.moments(st, "cpf1", p)
    ph = R.hydro_pressure(st, "cpf1", p)
    r_num = math.sqrt(float(((1.0 + m["phi"]) / 2.0).sum()) / math.pi)
    jump = lambda a: float(a[n // 2, n // 2] - a[0, 0]) * r_num
    assert abs(jump(m["P"]) - p.sigma) / p.sigma > 0.03
    assert abs(jump(ph) - p.sigma) / p.sigma < 0.015, jump(ph)
