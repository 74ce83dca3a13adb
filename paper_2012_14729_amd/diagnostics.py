"""Shape diagnostics of the order-parameter field (Sec. V benchmarks).

These read the phi moment that lbm_moments writes (a float32 [ny, nx] tensor,
on the GPU or the CPU) and reduce it with plain torch operations; they are
post-processing of results, not part of the time step.
"""
from __future__ import annotations

import math

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


def contour_length(phi: torch.Tensor) -> float:
    """Length of the phi = 0 contour (marching squares on the node grid, no
    wrap): each cell with two sign changes on its edges adds the segment
    between the two linear-interpolated crossings; a saddle cell (four
    crossings) adds the two segments that pair each crossing with its
    neighbour counter-clockwise from the bottom edge."""
    p = phi.double()
    a, b = p[:-1, :-1], p[:-1, 1:]     # (x, y), (x + 1, y)
    c, d = p[1:, 1:], p[1:, :-1]       # (x + 1, y + 1), (x, y + 1)

    def cut(u, v):
        return (u > 0) != (v > 0), u / (u - v)

    # crossing points in cell-local coordinates on the edges bottom, right, top, left
    cb, tb = cut(a, b)
    cr, tr = cut(b, c)
    ct, tt = cut(d, c)
    cl, tl = cut(a, d)
    pts = [(tb, torch.zeros_like(tb)), (torch.ones_like(tr), tr), (tt, torch.ones_like(tt)), (torch.zeros_like(tl), tl)]
    flags = [cb, cr, ct, cl]
    n = cb.int() + cr.int() + ct.int() + cl.int()
    total = torch.zeros((), dtype=torch.float64, device=p.device)
    # two crossings: the segment between them
    two = n == 2
    first = torch.zeros_like(two)
    x0 = torch.zeros_like(tb); y0 = torch.zeros_like(tb); x1 = torch.zeros_like(tb); y1 = torch.zeros_like(tb)
    for f, (px, py) in zip(flags, pts):
        take0 = f & ~first
        take1 = f & first
        x0 = torch.where(take0, px, x0); y0 = torch.where(take0, py, y0)
        x1 = torch.where(take1, px, x1); y1 = torch.where(take1, py, y1)
        first = first | f
    seg = torch.sqrt((x1 - x0) ** 2 + (y1 - y0) ** 2)
    total = total + seg[two].sum()
    four = n == 4
    if bool(four.any()):
        (bx, by), (rx, ry), (tx, ty), (lx, ly) = pts
        s1 = torch.sqrt((rx - bx) ** 2 + (ry - by) ** 2) + torch.sqrt((lx - tx) ** 2 + (ly - ty) ** 2)
        total = total + s1[four].sum()
    return float(total)


def bubble_metrics(phi: torch.Tensor, uy: torch.Tensor):
    """Rising-bubble quantities of Sec. V.D for a bubble of fluid 2 (phi < 0),
    in node units: centre of mass y_c = sum (1 - phi) y / sum (1 - phi), rise
    velocity v_c = sum (1 - phi) u_y / sum (1 - phi), and circularity
    C = 2 sqrt(pi A) / P_b (A = area of phi < 0, P_b = length of the phi = 0
    contour).  Node (x, y) sits at y + 1/2 from the lower wall."""
    phi = phi.double()
    if not bool(torch.isfinite(phi).all()):
        raise ValueError("phi holds non-finite values (the run diverged)")
    ny, nx = phi.shape
    w = 1.0 - phi
    y = torch.arange(ny, dtype=torch.float64, device=phi.device).view(ny, 1) + 0.5
    sw = w.sum()
    yc = float((w * y).sum() / sw)
    vc = float((w * uy.double()).sum() / sw)
    area = float((phi < 0).double().sum())
    perim = contour_length(phi)
    if perim == 0.0:
        raise ValueError("no phi = 0 contour")
    return yc, vc, 2.0 * math.sqrt(math.pi * area) / perim


def interface_heights(phi: torch.Tensor):
    """Height of the phi = 0 level in every column (fluid 1, phi > 0, below):
    the first downward crossing from the bottom, linearly interpolated, in
    distance from the lower wall (node j sits at j + 1/2).  Columns with no
    crossing give NaN."""
    p = phi.double()
    ny, nx = p.shape
    a, b = p[:-1, :], p[1:, :]
    cross = (a > 0) & (b <= 0)
    j = torch.argmax(cross.int(), dim=0)                 # first crossing per column
    has = cross.any(dim=0)
    cols = torch.arange(nx, device=p.device)
    pa, pb = a[j, cols], b[j, cols]
    y = j.double() + 0.5 + pa / (pa - pb)
    return torch.where(has, y, torch.full_like(y, float("nan")))


def wave_amplitude(phi: torch.Tensor, mean_level: float) -> float:
    """Amplitude of the first Fourier mode of the interface heights about
    mean_level, for a wave cos(2 pi (i + 1/2) / nx) along x."""
    y = interface_heights(phi) - mean_level
    nx = y.numel()
    x = (torch.arange(nx, dtype=torch.float64, device=y.device) + 0.5) * (2.0 * math.pi / nx)
    return float(2.0 / nx * (y * torch.cos(x)).sum())
