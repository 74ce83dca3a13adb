"""Shape diagnostics of the order-parameter field (Sec. V benchmarks).

These read the phi moment that lbm_moments writes (a float32 [ny, nx] tensor,
on the GPU or the CPU) and reduce it with plain torch operations; they are
post-processing of results, not part of the time step.
"""
from __future__ import annotations

import torch


def interface_points(phi: torch.Tensor):
    """Points of the phi = 0 contour: zero crossings between neighbouring
    nodes along x and along y, placed by linear interpolation.  Returns
    (x, y) float64 tensors in node coordinates."""
    phi = phi.double()
    ny, nx = phi.shape
    y = torch.arange(ny, dtype=torch.float64, device=phi.device).view(ny, 1)
    x = torch.arange(nx, dtype=torch.float64, device=phi.device).view(1, nx)
    a, b = phi[:, :-1], phi[:, 1:]
    cx = (a > 0) != (b > 0)
    xs = (x[:, :-1] + a / (a - b))[cx]
    ys = y.expand(ny, nx - 1)[cx]
    a2, b2 = phi[:-1, :], phi[1:, :]
    cy = (a2 > 0) != (b2 > 0)
    xs2 = x.expand(ny - 1, nx)[cy]
    ys2 = (y[:-1, :] + a2 / (a2 - b2))[cy]
    return torch.cat([xs, xs2]), torch.cat([ys, ys2])


def taylor_deformation(phi: torch.Tensor):
    """Taylor deformation D = (L - B) / (L + B) of a single drop of fluid 1
    (phi > 0) that does not touch the domain edge (Sec. V.E): L and B are
    twice the largest and smallest distance from the drop's centroid to the
    phi = 0 contour.  Returns (D, L, B, area of phi > 0 in nodes)."""
    phi = phi.double()
    ny, nx = phi.shape
    w = (phi > 0).double()
    area = w.sum()
    if float(area) == 0.0:
        raise ValueError("no phi > 0 region")
    y = torch.arange(ny, dtype=torch.float64, device=phi.device).view(ny, 1)
    x = torch.arange(nx, dtype=torch.float64, device=phi.device).view(1, nx)
    cx, cy = (w * x).sum() / area, (w * y).sum() / area
    px, py = interface_points(phi)
    r = torch.sqrt((px - cx) ** 2 + (py - cy) ** 2)
    L, B = 2.0 * float(r.max()), 2.0 * float(r.min())
    return (L - B) / (L + B), L, B, float(area)
