"""Physics benchmarks of Sec. V run on the GPU path.

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

import numpy as np
import torch

from . import Simulation
from .diagnostics import taylor_deformation
from .units import shear_drop_params, taylor_deformation as taylor_theory


def shear_drop(form: str, Ca: float, R: float = 20.0, H: float = 160.0, nu: float = 1.0 / 6.0, Re: float = 0.1,
               W: float = 4.0, M: float = 0.1, shear_times: float = 3.0, samples: int = 6):
    """Run the sheared drop for `shear_times` / E steps; returns a dict with
    the history [(step, D)], the last D, L, B and the drop area.  The run
    starts from the circular drop in the Couette profile."""
    nx, ny = int(round(2 * H)), int(round(H))
    p = shear_drop_params(R=R, H=H, Re=Re, Ca=Ca, nu=nu, W=W, M=M, nx=nx, ny=ny)
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
                theory=taylor_theory(Ca, 1.0), nodes=nx * ny)


def _main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["taylor"])
    ap.add_argument("--forms", default="stf1,stf2,cpf1,cpf2,pf1,pf2,csf1,csf2")
    ap.add_argument("--ca", default="0.1,0.2,0.3,0.4")
    ap.add_argument("--R", type=float, default=20.0)
    ap.add_argument("--shear-times", type=float, default=4.0)
    ap.add_argument("--M", type=float, default=0.1)
    a = ap.parse_args()
    for Ca in [float(v) for v in a.ca.split(",")]:
        for form in a.forms.split(","):
            r = shear_drop(form, Ca, R=a.R, H=8 * a.R, M=a.M, shear_times=a.shear_times)
            h = r["history"]
            print(f"taylor form={form} Ca={Ca} R={a.R:g} M={a.M:g} D={r['D']:.4f} dD_last={h[-1][1] - h[-2][1]:+.4f} "
                  f"theory={r['theory']:.4f} steps={r['steps']} tE={r['shear_time']:.2f} area={r['area']:.0f} "
                  f"MLUPS={r['nodes'] * r['steps'] / r['seconds'] / 1e6:.0f} diverged={r['diverged']}", flush=True)


if __name__ == "__main__":
    _main()
