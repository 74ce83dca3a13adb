"""Physical and dimensionless parameters -> lattice parameters (host side).

The governing equations are made dimensionless (Sec. II.A, after Eq. 10)
with a reference velocity U_c, length L_c, time L_c / U_c, density
rho_c = rho_1 and viscosity mu_c = mu_1, which leaves five groups:

    Re = rho_c U_c L_c / mu_c        Pe = U_c L_c / (4 M beta)
    We = rho_c L_c U_c^2 / sigma     Fr = U_c / sqrt(g L_c)
    Cn = W / L_c

with beta = 3 sigma / (4 W) (Eq. 6).  A lattice realisation picks L_c in
nodes, U_c in lattice velocity (keep it well below the lattice sound speed
1/sqrt(3)) and rho_1; every lattice parameter then follows.  The rising
bubble benchmark (Sec. V.D) states its flow by Re, Eo = rho_1 U_g^2 L / sigma
and Mo = Eo^3 / Re^4 with U_g = sqrt(2 R g), L = 2 R; the sheared drop
(Sec. V.E) by Re = E rho R^2 / mu and Ca = mu E R / sigma with E = 2 U / H.

Everything here is plain arithmetic on Python floats: it builds the
parameter dictionaries that Simulation and Batch take, and runs nothing on
the GPU.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional


@dataclass
class Groups:
    """The dimensionless groups of Sec. II.A plus the two property ratios."""
    Re: float
    We: float
    Pe: float
    Cn: float
    Fr: Optional[float] = None       # None: no gravity
    rho_ratio: float = 1.0           # rho_2 / rho_1
    mu_ratio: float = 1.0            # mu_2 / mu_1


def lattice_params(groups: Groups, L_c: float, U_c: float, rho1: float = 1.0, tau_h: float = 0.8,
                   gravity_axis: str = "y", **extra) -> dict:
    """Lattice parameters realising `groups` with reference length L_c (nodes)
    and velocity U_c (lattice units).  Gravity, if any, points along -axis.
    `extra` entries (nx, ny, walls, wall speeds, rho0, eps_n) are passed
    through unchanged.  Returns the keyword dictionary of lbm_params."""
    if L_c <= 0 or U_c <= 0 or rho1 <= 0:
        raise ValueError("L_c, U_c and rho1 must be positive")
    if U_c >= 1.0 / math.sqrt(3.0):
        raise ValueError("U_c must stay below the lattice sound speed 1/sqrt(3)")
    g = groups
    W = g.Cn * L_c
    sigma = rho1 * L_c * U_c * U_c / g.We
    mu1 = rho1 * U_c * L_c / g.Re
    rho2 = rho1 * g.rho_ratio
    mu2 = mu1 * g.mu_ratio
    beta = 3.0 * sigma / (4.0 * W)
    M = U_c * L_c / (4.0 * beta * g.Pe)
    grav = 0.0 if g.Fr is None else U_c * U_c / (g.Fr * g.Fr * L_c)
    out = dict(rho1=rho1, rho2=rho2, nu1=mu1 / rho1, nu2=mu2 / rho2, sigma=sigma, W=W, M=M, tau_h=tau_h,
               gx=-grav if gravity_axis == "x" else 0.0, gy=-grav if gravity_axis == "y" else 0.0)
    out.update(extra)
    return out


def groups_of(params: dict, L_c: float, U_c: float) -> Groups:
    """The groups a lattice parameter dictionary realises at (L_c, U_c)."""
    rho1, rho2 = params["rho1"], params["rho2"]
    mu1, mu2 = rho1 * params["nu1"], rho2 * params["nu2"]
    sigma, W, M = params["sigma"], params["W"], params["M"]
    beta = 3.0 * sigma / (4.0 * W)
    grav = math.hypot(params.get("gx", 0.0), params.get("gy", 0.0))
    return Groups(Re=rho1 * U_c * L_c / mu1, We=rho1 * L_c * U_c * U_c / sigma, Pe=U_c * L_c / (4.0 * M * beta),
                  Cn=W / L_c, Fr=None if grav == 0.0 else U_c / math.sqrt(grav * L_c),
                  rho_ratio=rho2 / rho1, mu_ratio=mu2 / mu1)


def tau_f(nu: float) -> float:
    """Relaxation time of a fluid of kinematic viscosity nu (nu = cs^2 (tau - 1/2))."""
    return 0.5 + 3.0 * nu


def rising_bubble_params(R: float, Eo: float, Mo: float, U_g: float = 0.01, rho1: float = 1.0,
                         rho_ratio: float = 1e-3, mu_ratio: float = 1e-2, W: float = 4.0, M: float = 0.1,
                         tau_h: float = 0.8, **extra) -> dict:
    """Lattice parameters of a bubble of radius R (nodes) rising under gravity
    (Sec. V.D): Re = (Eo^3 / Mo)^(1/4), g = U_g^2 / (2 R), L = 2 R,
    sigma = rho_1 U_g^2 L / Eo, mu_1 = rho_1 U_g L / Re."""
    L = 2.0 * R
    Re = (Eo ** 3 / Mo) ** 0.25
    g = U_g * U_g / (2.0 * R)
    sigma = rho1 * U_g * U_g * L / Eo
    mu1 = rho1 * U_g * L / Re
    rho2, mu2 = rho1 * rho_ratio, mu1 * mu_ratio
    out = dict(rho1=rho1, rho2=rho2, nu1=mu1 / rho1, nu2=mu2 / rho2, sigma=sigma, W=W, M=M, tau_h=tau_h,
               gx=0.0, gy=-g)
    out.update(extra)
    return out


def shear_drop_params(R: float, H: float, Re: float, Ca: float, nu: float = 0.1, W: float = 4.0,
                      M: Optional[float] = 0.1, tau_h: float = 0.8, rho_ratio: float = 1.0, Pe: Optional[float] = None,
                      **extra) -> dict:
    """Lattice parameters of a drop of radius R in a channel of height H
    (nodes) sheared by walls at +-U (Sec. V.E): the drop (fluid 1) has
    density rho_ratio, the surrounding fluid density 1, both kinematic
    viscosity nu (so the viscosity ratio is rho_ratio too); E = Re nu / R^2
    (Re = E rho_d R^2 / mu_d), U = E H / 2, sigma = mu_s E R / Ca with the
    surrounding fluid's viscosity, the one small-deformation theory puts in
    Ca.  M = None takes the mobility from Pe (default 1/Cn) with L_c = R and
    U_c = E R: M = E R^2 / (4 beta Pe), Cn = W / R.  The wall speeds go to
    u_wall_lo = -U, u_wall_hi = +U (walls in y)."""
    E = Re * nu / (R * R)
    U = E * H / 2.0
    sigma = nu * E * R / Ca
    if M is None:
        beta = 3.0 * sigma / (4.0 * W)
        M = E * R * R / (4.0 * beta * ((R / W) if Pe is None else Pe))
    out = dict(wall_y=1, u_wall_lo=-U, u_wall_hi=U, rho1=rho_ratio, rho2=1.0, nu1=nu, nu2=nu, sigma=sigma, W=W,
               M=M, tau_h=tau_h)
    out.update(extra)
    return out


def taylor_deformation(Ca: float, viscosity_ratio: float = 1.0) -> float:
    """Small-deformation theory of a sheared drop (Sec. V.E, Eq. 52):
    D = Ca (19 lambda + 16) / (16 lambda + 16)."""
    lam = viscosity_ratio
    return Ca * (19.0 * lam + 16.0) / (16.0 * lam + 16.0)
