"""Physics benchmarks of Sec. V run on the GPU path.

Rising bubble (Sec. V.D, Table V): a bubble of radius 0.25 at (0.5, 0.5)
in a 1 x 2 box, free-slip side walls, no-slip top and bottom, density ratio
10, viscosity ratio 10, Re = 35, Eo = 10 (Table IV); y_c, v_c and the
circularity C are followed to t = 3 (in the benchmark's units: lengths in
box widths, times in seconds with U_g = sqrt(2 R g) = 0.7).

    python -m paper_2012_14729_amd.benchmarks bubble [--res 240] [--forms ...]

Capillary wave (Sec. V.C, Table III): the amplitude of a small standing
wave against the analytic solution of Eqs. (44)-(46), error E2 of Eq. (47).

    python -m paper_2012_14729_amd.benchmarks capillary [--H 80] [--rho-ratio 0.1]

Sheared drop (Sec. V.E): a drop of radius R at the centre of a 2H x H
channel whose walls move at +-U, equal densities and viscosities, Re = 0.1;
run until the Taylor deformation D settles and compare it with the
small-deformation theory (Eq. 52) and with Table VI.

    python -m paper_2012_14729_amd.benchmarks taylor [--forms stf1,...] [--ca 0.1,0.2] [--M 3.0]

prints one line per (form, Ca) with D, its change over the last sample
interval, and the theory.
"""
from __future__ import annotations

import argparse
import math
import time
from typing import Optional

import numpy as np
import torch

from . import Simulation
from .diagnostics import bubble_metrics, taylor_deformation, wave_amplitude
from .theory import capillary_error, capillary_frequency, capillary_wave as capillary_theory
from .units import Groups, lattice_params, shear_drop_params, taylor_deformation as taylor_theory


def capillary_params(H: int, rho_ratio: float = 1.0, U_c: float = 0.0125, W: float = 4.0,
                     M: Optional[float] = None, Pe: Optional[float] = None, tau_h: float = 1.5,
                     Re: Optional[float] = None) -> dict:
    """Lattice parameters of the capillary wave (see capillary_wave)."""
    if Re is None:
        Re = 50.0 * math.sqrt(min(rho_ratio, 1.0))
    Cn = W / H
    g = Groups(Re=Re, We=1.0, Pe=(1.0 / Cn) if Pe is None else Pe, Cn=Cn, rho_ratio=rho_ratio, mu_ratio=rho_ratio)
    p = lattice_params(g, L_c=float(H), U_c=U_c, tau_h=tau_h, nx=H, ny=3 * H, wall_y=1)
    if M is not None:
        p["M"] = M
    return p


def bubble_params(res: int, U_g: float = 0.05, W: float = 4.0, M: Optional[float] = None,
                  Pe: Optional[float] = None, tau_h: float = 4.0) -> dict:
    """Lattice parameters of the rising bubble (see rising_bubble)."""
    L = 0.5 * res                      # L_c = 2 R, R = res / 4
    Cn = W / L
    g = Groups(Re=35.0, We=10.0, Pe=(1.0 / Cn) if Pe is None else Pe, Cn=Cn, Fr=1.0, rho_ratio=0.1, mu_ratio=0.1)
    p = lattice_params(g, L_c=L, U_c=U_g, tau_h=tau_h, nx=res, ny=2 * res, wall_x=2, wall_y=1)
    if M is not None:
        p["M"] = M
    return p


def shear_drop(form: str, Ca: float, R: float = 20.0, H: float = 160.0, nu: float = 1.0 / 6.0, Re: float = 0.1,
               W: float = 4.0, M: Optional[float] = None, shear_times: float = 3.0, samples: int = 6,
               rho_ratio: float = 1.0, tau_h: float = 0.8, Pe: Optional[float] = None):
    """Run the sheared drop for `shear_times` / E steps; returns a dict with
    the history [(step, D)], the last D, L, B and the drop area.  The run
    starts from the circular drop in the Couette profile."""
    nx, ny = int(round(2 * H)), int(round(H))
    p = shear_drop_params(R=R, H=H, Re=Re, Ca=Ca, nu=nu, W=W, M=M, tau_h=tau_h, rho_ratio=rho_ratio, Pe=Pe,
                          nx=nx, ny=ny)
    E = Re * nu / (R * R)
    U = p["u_wall_hi"]
    x = np.arange(nx, dtype=np.float64)[None, :].repeat(ny, 0)
    y = np.arange(ny, dtype=np.float64)[:, None].repeat(nx, 1)
    r = np.sqrt((x - nx / 2 + 0.5) ** 2 + (y - ny / 2 + 0.5) ** 2)
    phi0 = np.tanh(2.0 * (R - r) / W).astype(np.float32)
    ux0 = (U * (2.0 * (y + 0.5) / ny - 1.0)).astype(np.float32)
    sim = Simulation(p, phi0, ux0, np.zeros_like(ux0))
    total = int(math.ceil(shear_times / E / samples)) * samples
    chunk = total // samples
    hist = []
    t0 = time.time()
    for k in range(samples):
        sim.step(chunk, form)
        d, L, B, area = taylor_deformation(sim.moments(form)["phi"])
        hist.append(((k + 1) * chunk, d))
    torch.cuda.synchronize()
    return dict(form=form, Ca=Ca, history=hist, D=hist[-1][1], L=L, B=B, area=area, steps=total,
                shear_time=total * E, seconds=time.time() - t0, diverged=sim.status(),
                theory=taylor_theory(Ca, rho_ratio), nodes=nx * ny, M=p["M"])


def rising_bubble(form: str, res: int = 240, U_g: float = 0.05, W: float = 4.0,
                  M: Optional[float] = None, Pe: Optional[float] = None, tau_h: float = 4.0, t_end: float = 3.0,
                  samples: int = 60):
    """The bubble of Sec. V.D on a res x 2 res lattice.  Returns the history
    [(t, y_c, v_c, C)] in the benchmark's units (y in box widths, v in m/s,
    t in s) and its extrema y_max, v_max, C_min.

    The groups follow Table IV with L_c = 2R, U_c = U_g = sqrt(2 R g):
    Re = 35, We = Eo = 10, Fr = 1, density and viscosity ratios 10; the
    lattice parameters come from units.lattice_params.  The interface is
    W = 4 nodes and the mobility follows from Pe = 1/Cn (the rules stated at
    the opening of Sec. V) unless M or Pe is given.  The paper does not give
    U_g or tau_h: U_g = 0.05 (tau_f = 1.0 at res 240) and tau_h = 4.0 by
    default.  At Pe = 1/Cn the mobility is large (M = 8.9 at res 240, 17.8
    at res 120), and the order-parameter scheme needs a large tau_h: with
    tau_h = 2.5 every form diverges within t = 0.05; with 4.0 every form but
    CPF-1 and PF-2 runs to t = 3."""
    nx, ny = res, 2 * res
    R = 0.25 * res
    p = bubble_params(res, U_g=U_g, W=W, M=M, Pe=Pe, tau_h=tau_h)
    x = np.arange(nx, dtype=np.float64)[None, :].repeat(ny, 0) + 0.5
    y = np.arange(ny, dtype=np.float64)[:, None].repeat(nx, 1) + 0.5
    r = np.sqrt((x - 0.5 * res) ** 2 + (y - 0.5 * res) ** 2)
    phi0 = np.tanh(2.0 * (r - R) / W).astype(np.float32)         # fluid 2 (phi = -1) inside
    sim = Simulation(p, phi0)
    L_lat, L_phys, Ug_phys = 2.0 * R, 0.5, 0.7
    dt = (L_phys / Ug_phys) / (L_lat / U_g)                        # seconds per step
    total = int(round(t_end / dt))
    chunk = max(1, total // samples)
    hist = []
    n = 0
    t0 = time.time()
    while n < total:
        k = min(chunk, total - n)
        sim.step(k, form)
        n += k
        m = sim.moments(form)
        if not bool(torch.isfinite(m["phi"]).all()):
            break                                                   # diverged: report up to here
        yc, vc, C = bubble_metrics(m["phi"], m["uy"])
        hist.append((n * dt, yc / res, vc / U_g * Ug_phys, C))
    torch.cuda.synchronize()
    return dict(form=form, res=res, M=p["M"], W=W, tau_h=tau_h, history=hist,
                y_max=max((h[1] for h in hist), default=float("nan")),
                v_max=max((h[2] for h in hist), default=float("nan")),
                C_min=min((h[3] for h in hist), default=float("nan")), steps=n, t_reached=n * dt,
                seconds=time.time() - t0, nodes=nx * ny, diverged=sim.status())


def capillary_wave(form: str, H: int = 80, rho_ratio: float = 1.0, h0: float = 0.01, U_c: float = 0.0125,
                   W: float = 4.0, M: Optional[float] = None, Pe: Optional[float] = None, tau_h: float = 1.5,
                   Re: Optional[float] = None, samples: int = 200):
    """The capillary wave of Sec. V.C: an H x 3H box, periodic in x, no-slip
    walls top and bottom, fluid 1 (density 1) below the interface
    y = 1.5 H + h0 H cos(k x), fluid 2 (density rho_ratio) above, equal
    kinematic viscosity, Re = U_c H / nu and We = rho_1 H U_c^2 / sigma = 1
    (U_c = sqrt(sigma / (rho_1 H))); the lattice parameters come from
    units.lattice_params with L_c = H, and the mobility from Pe = 1/Cn
    (the rule stated at the opening of Sec. V) unless M or Pe is given.
    Re defaults to 50 sqrt(rho_ratio) (rho_ratio <= 1): the paper's
    parameters give Re = 50 at equal densities, and its density-ratio-10
    runs keep H, nu, sigma and the light fluid's density while the lower
    fluid becomes ten times heavier, so U_c, taken from the heavy fluid,
    drops by sqrt(10).  tau_h (not given) is 1.5: at Pe = 1/Cn (M = 5.3 at
    H = 80) every form diverges within 150 steps with tau_h = 0.8, 1.0 or
    1.25.  Runs to t = 25 / w0 and returns the normalised amplitude history
    h(t)/h0 against theory (Eqs. 44-46) and the time-averaged error E2
    (Eq. 47).  h0 (a fraction of H) is not given in the paper: 0.01 H by
    default."""
    if not (0.0 < h0 < 0.5):
        raise ValueError("h0 (the initial amplitude as a fraction of H) must lie in (0, 0.5)")
    nx, ny = H, 3 * H
    p = capillary_params(H, rho_ratio=rho_ratio, U_c=U_c, W=W, M=M, Pe=Pe, tau_h=tau_h, Re=Re)
    nu, sigma = p["nu1"], p["sigma"]
    k = 2.0 * math.pi / H
    amp = h0 * H
    x = np.arange(nx, dtype=np.float64)[None, :].repeat(ny, 0) + 0.5
    y = np.arange(ny, dtype=np.float64)[:, None].repeat(nx, 1) + 0.5
    level = 1.5 * H
    phi0 = np.tanh(2.0 * (level + amp * np.cos(k * x) - y) / W).astype(np.float32)
    sim = Simulation(p, phi0)
    w0 = capillary_frequency(k, 1.0, rho_ratio, sigma)
    total = int(math.ceil(25.0 / w0))
    # normalise by the amplitude measured on the initial field, so that the
    # interpolation of the diffuse profile does not bias h(t)/h0
    a0 = wave_amplitude(sim.moments(form)["phi"], level)
    hist = [(0.0, 1.0)]
    n = 0
    t0 = time.time()
    for s_ in range(samples):
        m_ = int(round(total * (s_ + 1) / samples)) - n
        sim.step(m_, form)
        n += m_
        phi = sim.moments(form)["phi"]
        if not bool(torch.isfinite(phi).all()):
            break
        hist.append((n, wave_amplitude(phi, level) / a0))
    torch.cuda.synchronize()
    t = np.array([h[0] for h in hist])
    hn = np.array([h[1] for h in hist])
    done = n >= total and len(hist) == samples + 1
    e2 = capillary_error(t, hn, nu, k, 1.0, rho_ratio, sigma) if done else float("nan")
    return dict(form=form, H=H, rho_ratio=rho_ratio, M=p["M"], tau_h=tau_h, t=t, h=hn,
                theory=capillary_theory(t, nu, k, 1.0, rho_ratio, sigma),
                E2=e2, h0_measured=a0 / amp, steps=n, seconds=time.time() - t0, nodes=nx * ny,
                diverged=sim.status())


def _main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["taylor", "bubble", "capillary"])
    ap.add_argument("--H", type=int, default=80)
    ap.add_argument("--rho-ratio", type=float, default=1.0)
    ap.add_argument("--Uc", type=float, default=0.0125)
    ap.add_argument("--res", type=int, default=240)
    ap.add_argument("--W", type=float, default=4.0)
    ap.add_argument("--tau-h", type=float, default=None, help="default 1.5 capillary, 4.0 bubble")
    ap.add_argument("--Pe", type=float, default=None, help="Peclet number (default 1/Cn; ignored with --M)")
    ap.add_argument("--forms", default="stf1,stf2,cpf1,cpf2,pf1,pf2,csf1,csf2")
    ap.add_argument("--ca", default="0.1,0.2,0.3,0.4")
    ap.add_argument("--R", type=float, default=20.0)
    ap.add_argument("--shear-times", type=float, default=4.0)
    ap.add_argument("--M", type=float, default=None, help="mobility (default: from Pe; 0.1 taylor)")
    a = ap.parse_args()
    if a.which == "capillary":
        for form in a.forms.split(","):
            r = capillary_wave(form, H=a.H, rho_ratio=a.rho_ratio, U_c=a.Uc, M=a.M, Pe=a.Pe,
                               tau_h=1.5 if a.tau_h is None else a.tau_h)
            print(f"capillary form={form} H={a.H} rho2/rho1={a.rho_ratio:g} Uc={a.Uc:g} M={r['M']:.4g} "
                  f"tau_h={r['tau_h']:g} E2={r['E2']:.4f} "
                  f"h(0)/h0={r['h0_measured']:.4f} steps={r['steps']} "
                  f"MLUPS={r['nodes'] * r['steps'] / r['seconds'] / 1e6:.0f} diverged={r['diverged']}", flush=True)
        return
    if a.which == "bubble":
        for form in a.forms.split(","):
            r = rising_bubble(form, res=a.res, W=a.W, M=a.M, Pe=a.Pe, tau_h=4.0 if a.tau_h is None else a.tau_h)
            print(f"bubble form={form} res={a.res} W={r['W']:g} M={r['M']:.4g} tau_h={r['tau_h']:g} "
                  f"y_max={r['y_max']:.4f} v_max={r['v_max']:.4f} "
                  f"C_min={r['C_min']:.4f} steps={r['steps']} t={r['t_reached']:.2f} "
                  f"MLUPS={r['nodes'] * r['steps'] / r['seconds'] / 1e6:.0f} diverged={r['diverged']}", flush=True)
        return
    for Ca in [float(v) for v in a.ca.split(",")]:
        for form in a.forms.split(","):
            r = shear_drop(form, Ca, R=a.R, H=8 * a.R, M=a.M, shear_times=a.shear_times, rho_ratio=a.rho_ratio,
                           tau_h=0.8 if a.tau_h is None else a.tau_h)
            h = r["history"]
            print(f"taylor form={form} Ca={Ca} R={a.R:g} rho_d/rho_s={a.rho_ratio:g} M={r['M']:.4g} D={r['D']:.4f} dD_last={h[-1][1] - h[-2][1]:+.4f} "
                  f"theory={r['theory']:.4f} steps={r['steps']} tE={r['shear_time']:.2f} area={r['area']:.0f} "
                  f"MLUPS={r['nodes'] * r['steps'] / r['seconds'] / 1e6:.0f} diverged={r['diverged']}", flush=True)


if __name__ == "__main__":
    _main()
