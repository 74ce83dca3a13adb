"""CPU checks of the shape diagnostics on analytic fields."""
import math

import torch

from paper_2012_14729_amd import diagnostics as Dg


def ellipse_phi(a, b, theta, nx=320, ny=160, W=4.0, xc=160.3, yc=80.2):
    y = torch.arange(ny, dtype=torch.float64).view(ny, 1)
    x = torch.arange(nx, dtype=torch.float64).view(1, nx)
    X, Y = x - xc, y - yc
    u = X * math.cos(theta) + Y * math.sin(theta)
    v = -X * math.sin(theta) + Y * math.cos(theta)
    # signed distance approximated by the scaled radius, fine for the contour
    r = torch.sqrt((u / a) ** 2 + (v / b) ** 2)
    return torch.tanh(2.0 * (1.0 - r) * math.sqrt(a * b) / W)


def test_circle_has_no_deformation():
    d, L, B, area = Dg.taylor_deformation(ellipse_phi(20.0, 20.0, 0.0))
    assert d < 0.01
    assert abs(L / 2 - 20.0) < 0.6 and abs(B / 2 - 20.0) < 0.6
    assert abs(area - math.pi * 400) / (math.pi * 400) < 0.02


def test_ellipse_deformation_at_any_angle():
    for a, b, th in ((26.0, 16.0, 35.0), (30.0, 14.0, -20.0), (22.0, 19.0, 80.0)):
        d, L, B, _ = Dg.taylor_deformation(ellipse_phi(a, b, math.radians(th)))
        exact = (a - b) / (a + b)
        assert abs(d - exact) < 0.01, (a, b, th, d, exact)
        assert abs(L - 2 * a) < 1.5 and abs(B - 2 * b) < 1.5


def test_interface_points_lie_on_the_contour():
    phi = ellipse_phi(25.0, 15.0, 0.3)
    px, py = Dg.interface_points(phi)
    assert px.numel() > 100
    # bilinear value of phi at the crossing points is ~0
    x0, y0 = px.floor().long(), py.floor().long()
    fx, fy = px - x0, py - y0
    v = (phi[y0, x0] * (1 - fx) * (1 - fy) + phi[y0, x0 + 1] * fx * (1 - fy)
         + phi[y0 + 1, x0] * (1 - fx) * fy + phi[y0 + 1, x0 + 1] * fx * fy)
    assert float(v.abs().max()) < 0.05


def test_contour_length_of_circle_and_ellipse():
    ny, nx = 200, 160
    y = torch.arange(ny, dtype=torch.float64).view(ny, 1)
    x = torch.arange(nx, dtype=torch.float64).view(1, nx)
    r = torch.sqrt((x - 80.3) ** 2 + (y - 100.6) ** 2)
    assert abs(Dg.contour_length(torch.tanh(2 * (r - 30.0) / 4)) - 2 * math.pi * 30.0) < 0.05
    a, b = 40.0, 20.0
    rr = torch.sqrt(((x - 80.3) / a) ** 2 + ((y - 100.6) / b) ** 2)
    h = ((a - b) / (a + b)) ** 2
    ramanujan = math.pi * (a + b) * (1 + 3 * h / (10 + math.sqrt(4 - 3 * h)))
    assert abs(Dg.contour_length(torch.tanh(2 * (rr - 1) * math.sqrt(a * b) / 4)) - ramanujan) < 0.05


def test_bubble_metrics_of_a_round_bubble():
    ny, nx = 240, 120
    y = torch.arange(ny, dtype=torch.float64).view(ny, 1)
    x = torch.arange(nx, dtype=torch.float64).view(1, nx)
    r = torch.sqrt((x - 59.5) ** 2 + (y - 70.25) ** 2)
    phi = torch.tanh(2 * (r - 30.0) / 5.0)          # fluid 2 inside
    uy = torch.where(phi < 0, torch.full_like(phi, 0.01), torch.zeros_like(phi))
    yc, vc, C = Dg.bubble_metrics(phi, uy)
    assert abs(yc - 70.75) < 1e-6                    # node centres at y + 1/2
    assert abs(vc - 0.01) < 2e-3 and abs(C - 1.0) < 0.005
