"""Seeded synthetic inputs for the benchmark configurations.

Shared by the tests, bench.py and smoke(): this module builds initial fields
(phi0, u0) and parameter sets only.  It holds none of the lattice Boltzmann
arithmetic and imports neither the oracle nor the HIP library.

Initial conditions follow the paper's benchmark set-ups (arXiv:2012.14729,
Sec. V): a tanh droplet (Sec. V.A, Eq. 45), two droplets about to merge
(Sec. V.B, Eq. 46), a bubble in a channel (Sec. V.D set-up) and a drop in
simple shear (Sec. V.E set-up).  All quantities are in lattice units.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

FORM_NAMES = ("stf1", "stf2", "cpf1", "cpf2", "pf1", "pf2", "csf1", "csf2")


@dataclass
class ParamSet:
    """Field-for-field copy of the C struct lbm_params."""
    nx: int
    ny: int
    wall_x: int = 0
    wall_y: int = 0
    u_wall_lo: float = 0.0
    u_wall_hi: float = 0.0
    rho1: float = 1.0
    rho2: float = 1.0
    nu1: float = 0.1
    nu2: float = 0.1
    sigma: float = 0.01
    W: float = 4.0
    M: float = 0.1
    tau_h: float = 0.8
    gx: float = 0.0
    gy: float = 0.0
    rho0: float = float("nan")
    eps_n: float = 1e-6

    def as_dict(self):
        return asdict(self)


def _grid(nx, ny):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y


def droplet(nx, ny, R, W, xc=None, yc=None, inside=1.0):
    """phi = tanh(2 (R - r) / W) about (xc, yc) (Eq. 45); inside=-1 gives a bubble of fluid 2."""
    x, y = _grid(nx, ny)
    xc = nx / 2 if xc is None else xc
    yc = ny / 2 if yc is None else yc
    r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
    return inside * np.tanh(2.0 * (R - r) / W)


def two_droplets(nx, ny, R1, R2, d, W):
    """phi = 1 + tanh(2(R1 - r1)/W) + tanh(2(R2 - r2)/W), centres at
    (nx/2 - R1 - d/2, ny/2) and (nx/2 + R2 + d/2, ny/2)  (Eq. 46)."""
    x, y = _grid(nx, ny)
    x1, x2 = nx / 2 - R1 - d / 2, nx / 2 + R2 + d / 2
    r1 = np.sqrt((x - x1) ** 2 + (y - ny / 2) ** 2)
    r2 = np.sqrt((x - x2) ** 2 + (y - ny / 2) ** 2)
    return 1.0 + np.tanh(2.0 * (R1 - r1) / W) + np.tanh(2.0 * (R2 - r2) / W)


# ----------------------------------------------------------------------------
# Benchmark configurations (lattice units)
# ----------------------------------------------------------------------------
def config_droplet64():
    """64x64 periodic stationary droplet, R = 16, W = 4, rho ratio 10,
    nu1 = nu2 = 0.1 (tau_f = 0.8), sigma = 0.01, tau_h = 0.8, M = 0.1."""
    p = ParamSet(nx=64, ny=64, rho1=10.0, rho2=1.0, nu1=0.1, nu2=0.1, sigma=0.01, W=4.0, M=0.1, tau_h=0.8)
    return p, droplet(64, 64, 16.0, 4.0), None, None


def config_droplet_large(n=2048, R=None, W=5.0):
    """n x n periodic stationary droplet with density ratio 1000 and dynamic
    viscosity ratio 100: rho1 = 1000, rho2 = 1, nu1 = 1/30, nu2 = 1/3,
    sigma = 1e-3, M = 0.1, tau_h = 0.8.  R = n/8 unless given."""
    R = n / 8 if R is None else R
    p = ParamSet(nx=n, ny=n, rho1=1000.0, rho2=1.0, nu1=1.0 / 30.0, nu2=1.0 / 3.0, sigma=1e-3, W=W, M=0.1, tau_h=0.8)
    return p, droplet(n, n, R, W), None, None


def config_bubble(nx=1024, ny=4096, R=128.0, yc=512.0):
    """Bubble (fluid 2, phi = -1) rising in a channel with no-slip walls at
    x = -1/2 and nx - 1/2, periodic in y.  rho1 = 1, rho2 = 1e-3, mu1/mu2 = 100,
    Eo = 10 and Mo = 1e-3 with U_g = sqrt(2 R g) = 0.01."""
    Ug = 0.01
    g = Ug * Ug / (2 * R)
    rho1, rho2 = 1.0, 1e-3
    Eo, Mo = 10.0, 1e-3
    sigma = rho1 * g * (2 * R) ** 2 / Eo
    Re = (Eo ** 3 / Mo) ** 0.25
    mu1 = rho1 * Ug * (2 * R) / Re
    mu2 = mu1 / 100.0
    p = ParamSet(nx=nx, ny=ny, wall_x=1, rho1=rho1, rho2=rho2, nu1=mu1 / rho1, nu2=mu2 / rho2,
                 sigma=sigma, W=4.0, M=0.1, tau_h=0.8, gx=0.0, gy=-g)
    return p, droplet(nx, ny, R, 4.0, xc=nx / 2, yc=yc, inside=-1.0), None, None


def config_shear(nx=512, ny=256, R=64.0, Re=1.0, Ca=0.2, nu=0.1, W=4.0):
    """Drop in simple shear: walls at y = -1/2 (-U) and ny - 1/2 (+U), periodic
    x, rho1 = rho2 = 1, E = 2U/ny with Re = E R^2 / nu and Ca = mu E R / sigma.
    u0 is the Couette profile."""
    E = Re * nu / (R * R)
    U = E * ny / 2.0
    sigma = nu * E * R / Ca
    p = ParamSet(nx=nx, ny=ny, wall_y=1, u_wall_lo=-U, u_wall_hi=U, rho1=1.0, rho2=1.0, nu1=nu, nu2=nu,
                 sigma=sigma, W=W, M=0.1, tau_h=0.8)
    x, y = _grid(nx, ny)
    ux0 = U * (2.0 * (y + 0.5) / ny - 1.0)
    return p, droplet(nx, ny, R, W), ux0, np.zeros_like(ux0)


def batch_instances(count=512, seed=14729, sides=tuple(range(32, 513, 16))):
    """Independent two-droplet instances of uneven size and force form.

    Draws per instance, in this order, from numpy default_rng(seed): side s,
    R1, R2 ~ U[6, s/5], gap d ~ U[1, 4], density ratio in {1, 10, 100},
    log10 sigma ~ U[-4, -2], force form index ~ U{0..7}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        s = int(rng.choice(sides))
        R1 = float(rng.uniform(6.0, s / 5.0))
        R2 = float(rng.uniform(6.0, s / 5.0))
        d = float(rng.uniform(1.0, 4.0))
        ratio = float(rng.choice([1.0, 10.0, 100.0]))
        sigma = float(10.0 ** rng.uniform(-4.0, -2.0))
        form = int(rng.integers(0, 8))
        p = ParamSet(nx=s, ny=s, rho1=ratio, rho2=1.0, nu1=0.1, nu2=0.1, sigma=sigma, W=4.0, M=0.1, tau_h=0.8)
        out.append((p, form, two_droplets(s, s, R1, R2, d, 4.0)))
    return out
