"""Pins of the oracle's free-slip (specular) half-way walls.

A free-slip wall is a plane of mirror symmetry: a lattice of width n with
free-slip walls at x = -1/2 and n - 1/2 must evolve exactly like the left
half of a periodic lattice of width 2n whose initial fields are mirrored
about x = n - 1/2 (phi even, u_x odd).  That single comparison exercises the
specular streaming, the even extension of phi, the mirrored ghost velocity
and every force stencil near the wall; with no-slip walls on the other axis
it also fixes the corner rule (a link into a corner bounces back).  A
gravity-driven single-phase column between free-slip walls feels no wall
friction: its velocity is g (n + 1/2) everywhere after n steps (Eq. 37's
half-force shift)."""
import pytest
import torch

from oracle import lbm_ref as R

torch.set_default_dtype(torch.float64)


def _drop(nx, ny, xc, yc, r, W=3.0):
    yy, xx = torch.meshgrid(torch.arange(float(ny)), torch.arange(float(nx)), indexing="ij")
    return torch.tanh(2.0 * (r - torch.sqrt((xx - xc) ** 2 + (yy - yc) ** 2)) / W)


def _mirror_run(form, axis, other_wall, steps=12):
    n, m = 14, 12                               # half width along `axis`, other side
    base = dict(rho1=5.0, rho2=1.0, nu1=0.1, nu2=0.15, sigma=0.01, W=3.0, M=0.1, gx=2e-6, gy=-3e-6, rho0=2.0)
    if axis == "x":
        half = _drop(n, m, 4.3, 5.6, 3.5)
        full = torch.cat([half, half.flip(1)], dim=1)
        ph = R.Params(nx=n, ny=m, wall_x=2, wall_y=other_wall, **base)
        pf = R.Params(nx=2 * n, ny=m, wall_x=0, wall_y=other_wall, **base)
        # gravity along x would break the mirror symmetry: keep it along the wall
        ph.gx = pf.gx = 0.0
    else:
        half = _drop(m, n, 5.6, 4.3, 3.5)
        full = torch.cat([half, half.flip(0)], dim=0)
        ph = R.Params(nx=m, ny=n, wall_x=other_wall, wall_y=2, **base)
        pf = R.Params(nx=m, ny=2 * n, wall_x=other_wall, wall_y=0, **base)
        ph.gy = pf.gy = 0.0
    a = R.moments(R.run(R.init(ph, half), form, ph, steps), form, ph)
    b = R.moments(R.run(R.init(pf, full), form, pf, steps), form, pf)
    for k in ("phi", "rho", "ux", "uy", "P"):
        bk = b[k][:, :n] if axis == "x" else b[k][:n, :]
        scale = max(float(bk.abs().max()), 1e-30)
        assert float((a[k] - bk).abs().max()) <= 1e-11 * scale + 1e-300, (form, axis, k)
    # the mirrored lattice really is symmetric (the comparison is not vacuous)
    un = b["ux"] if axis == "x" else b["uy"]
    assert float(un.abs().max()) > 1e-7


@pytest.mark.parametrize("form", R.FORMS)
def test_free_slip_x_wall_is_a_mirror_plane(form):
    _mirror_run(form, "x", 0)


@pytest.mark.parametrize("form", ["stf2", "cpf1", "csf1"])
def test_free_slip_y_wall_is_a_mirror_plane(form):
    _mirror_run(form, "y", 0)


@pytest.mark.parametrize("form", ["stf1", "pf2"])
def test_free_slip_meets_no_slip_at_corners(form):
    _mirror_run(form, "x", 1)
    _mirror_run(form, "y", 1)


def test_column_between_free_slip_walls_accelerates_uniformly():
    g, n = 1e-6, 40
    p = R.Params(nx=10, ny=8, wall_x=2, rho1=1.0, rho2=1.0, gx=0.0, gy=g, rho0=0.0)
    st = R.run(R.init(p, torch.ones(8, 10)), "stf2", p, n)
    m = R.moments(st, "stf2", p)
    assert float((m["uy"] - g * (n + 0.5)).abs().max()) < 1e-15
    assert float(m["ux"].abs().max()) < 1e-18
    # the same column between no-slip walls is slowed at the walls
    q = R.Params(nx=10, ny=8, wall_x=1, rho1=1.0, rho2=1.0, gx=0.0, gy=g, rho0=0.0)
    mq = R.moments(R.run(R.init(q, torch.ones(8, 10)), "stf2", q, n), "stf2", q)
    assert float(mq["uy"][:, 0].mean()) < 0.9 * g * (n + 0.5)


def test_free_slip_box_conserves_order_parameter():
    """phi = sum h_i, and the mass rho(phi) with it, is conserved: specular
    reflection and the corner bounce-back only move populations."""
    p = R.Params(nx=16, ny=12, wall_x=2, wall_y=2, rho1=3.0, rho2=1.0, sigma=0.01, W=3.0, gy=-1e-5)
    st0 = R.init(p, _drop(16, 12, 5.2, 6.7, 4.0))
    st = R.run(st0, "csf2", p, 25)
    assert abs(float(st["h"].sum() - st0["h"].sum())) < 1e-11
    assert float((st["h"].sum(0) - st0["h"].sum(0)).abs().max()) > 1e-6   # the drop did move


def test_free_slip_walls_refuse_wall_speeds():
    p = R.Params(nx=8, ny=8, wall_x=2, u_wall_hi=0.01)
    with pytest.raises(ValueError):
        R.init(p, torch.zeros(8, 8))
