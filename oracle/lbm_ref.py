"""Vectorised CPU reference of the phase-field LBM time step (oracle).

TEST INFRASTRUCTURE ONLY -- imported by tests/, __graft_entry__.smoke() and
bench.py's cpu_baseline leg; never by the HIP library.

Follows Zhang, Liang & Guo, arXiv:2012.14729:
  Sec. II.A  -- mixture density/viscosity (Eqs. 9-10), chemical potential
                (Eq. 2 with f0 = beta (1 - phi^2)^2), beta and kappa (Eq. 6);
  Sec. II.B  -- the eight interfacial forces (Eqs. 17, 18, 20, 24, 25);
  Sec. III   -- the two lattice Boltzmann equations (Eqs. 29-30), equilibria
                (Eqs. 31-33), D2Q9 lattice (Eq. 34), forcing terms (Eqs. 35-36),
                macroscopic moments (Eq. 37), transport coefficients (after
                Eq. 40), isotropic difference stencils (Eqs. 41-42);
  Sec. IV    -- half-way bounce-back with moving walls (Eq. 43) and the
                order-parameter wall condition (Eq. 44);
  Sec. V.D   -- free-slip side walls of the rising-bubble test (reading A24);
  Sec. V     -- explicit-Euler time derivative and the modified weights
                (opening paragraph of Sec. V).

Lattice units throughout: dx = dt = c = 1, cs^2 = 1/3.  Fields are torch
tensors indexed [y, x] (x fastest).  Populations are [9, ny, nx].

State convention: the state at time n holds the pre-collision populations
f_i(x, n), h_i(x, n) plus J = (phi u) of the previous step.  One call to
``step`` performs the collision of Eqs. (29)-(30) at time n and the streaming
to time n+1 (with bounce-back at walls).

The readings taken where the paper is silent or garbled are listed next to
the code that uses them (labels A1..A23 as in the design notes):
  A1  forcing term of Eq. (35): Gamma_i = w_i (1 + s_i) and the pressure
      gradient term is w_i s_i grad(cs^2 rho);
  A3  the factor 3 in Eq. (36) is 1/cs^2;
  A4  d_t(phi u) = (phi u)^n - (phi u)^(n-1); before the first step
      (phi u)^(-1) = phi0 u0;
  A5  div(phi u) by the isotropic stencil of Eq. (41) on the node field phi u
      of the current step;
  A6  tau_f(x) = 1/2 + mu(phi)/(cs^2 rho(phi)), mu linear in phi;
  A8  n = grad(phi)/sqrt(|grad(phi)|^2 + eps^2); CSF-1 is taken as
      -kappa |grad(phi)|^2 n div(n) (the delta-function form of Eq. 24 with the
      regularised normal);
  A9  at a half-way wall phi is extended by even reflection (ghost -1-k holds
      node k), which gives n_w.grad(phi) = n_w.grad(mu) = 0; the ghost velocity
      is 2 u_w - u(mirror node);
  A10 rho(x_w), phi(x_w) in Eq. (43) are taken at the fluid node x_f;
  A11 initial populations: f = f^eq(P=0, u0, rho(phi0)),
      h = h^eq(phi0, mu(phi0), u0);
  A12 rho0 (background density of F_g): if not given, the mean of rho(phi0)
      over the domain, fixed for the run;
  A18 second-level derivatives apply the same stencil twice;
  A23 the hydrodynamic pressure of STF-1 is P_sf + kappa |grad(phi)|^2 (the
      sign printed after Eq. 17 contradicts Eqs. 19, 21 and 26);
  A24 a free-slip wall (named, not specified, in Sec. V.D) is a half-way
      plane of mirror symmetry: links crossing it reflect specularly, phi is
      extended evenly, the ghost velocity mirrors (normal component negated,
      tangential copied); a link into a corner bounces back.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import torch

# ----------------------------------------------------------------------------
# D2Q9 lattice: Sec. III, Eq. (34) and the weights given right after it.
# ----------------------------------------------------------------------------
CX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
CY = (0, 0, 1, 0, -1, 1, 1, -1, -1)
WT = (4.0 / 9.0,) + (1.0 / 9.0,) * 4 + (1.0 / 36.0,) * 4
CS2 = 1.0 / 3.0
# opposite direction: c_opp = -c
OPP = tuple(next(j for j in range(9) if CX[j] == -CX[i] and CY[j] == -CY[i]) for i in range(9))
# modified weights of the CH forcing (Sec. V opening paragraph): wbar_0 = w_0 - 1
WBAR = (WT[0] - 1.0,) + WT[1:]

FORMS = ("stf1", "stf2", "cpf1", "cpf2", "pf1", "pf2", "csf1", "csf2")


@dataclass
class Params:
    """Problem statement in lattice units (mirrors the C struct lbm_params)."""
    nx: int
    ny: int
    wall_x: int = 0          # half-way walls at x = -1/2 and x = nx - 1/2: 1 no-slip, 2 free-slip
    wall_y: int = 0          # half-way walls at y = -1/2 and y = ny - 1/2: 1 no-slip, 2 free-slip
    u_wall_lo: float = 0.0   # tangential speed of the low wall of the walled axis
    u_wall_hi: float = 0.0   # tangential speed of the high wall
    rho1: float = 1.0        # fluid 1 (phi = +1)
    rho2: float = 1.0        # fluid 2 (phi = -1)
    nu1: float = 0.1
    nu2: float = 0.1
    sigma: object = 0.01     # float or 0-d tensor (for derivatives)
    W: float = 4.0
    M: object = 0.1          # float or 0-d tensor (for derivatives)
    tau_h: float = 0.8
    gx: float = 0.0
    gy: float = 0.0
    rho0: Optional[float] = None   # None/NaN -> mean of rho(phi0)  (A12)
    eps_n: float = 1e-6


@dataclass
class Const:
    beta: object
    kappa: object
    eta: object
    a_h: float
    mu1: float
    mu2: float


def constants(p: Params) -> Const:
    """Derived coefficients.

    beta = 3 sigma / (4 W), kappa = 3 W sigma / 8           (Sec. II.A, Eq. 6)
    M = cs^2 eta (tau_h - 1/2)  =>  eta                      (Sec. III, after Eq. 40)
    tau_2 = tau_h^2 - tau_h + 1/6, tau_1 = tau_h - 1/2,
    A_H = 3 tau_2 / (tau_h tau_1)                            (Sec. III, after Eq. 36)
    mu_k = rho_k nu_k (dynamic viscosity of each fluid).
    """
    beta = 3.0 * p.sigma / (4.0 * p.W)
    kappa = 3.0 * p.W * p.sigma / 8.0
    eta = p.M / (CS2 * (p.tau_h - 0.5))
    tau2 = p.tau_h * p.tau_h - p.tau_h + 1.0 / 6.0
    tau1 = p.tau_h - 0.5
    a_h = 3.0 * tau2 / (p.tau_h * tau1)
    return Const(beta, kappa, eta, a_h, p.rho1 * p.nu1, p.rho2 * p.nu2)


# ----------------------------------------------------------------------------
# Ghost extension (Sec. IV; readings A9).
# ----------------------------------------------------------------------------
def _ext_axis(a: torch.Tensor, k: int, dim: int, wall: bool) -> torch.Tensor:
    n = a.shape[dim]
    if wall:
        # ghost index -1-m holds node m; ghost n+m holds node n-1-m
        lo = a.narrow(dim, 0, k).flip(dim)
        hi = a.narrow(dim, n - k, k).flip(dim)
    else:
        lo = a.narrow(dim, n - k, k)
        hi = a.narrow(dim, 0, k)
    return torch.cat([lo, a, hi], dim=dim)


def extend_scalar(a: torch.Tensor, k: int, p: Params) -> torch.Tensor:
    """[ny, nx] -> [ny+2k, nx+2k]: periodic wrap or even reflection at walls."""
    a = _ext_axis(a, k, 1, bool(p.wall_x))
    return _ext_axis(a, k, 0, bool(p.wall_y))


def _wall_velocity(p: Params):
    """Velocity vectors (lo, hi) of the walls: a y-wall moves along x, an
    x-wall moves along y."""
    if p.wall_y:
        return (p.u_wall_lo, 0.0), (p.u_wall_hi, 0.0)
    if p.wall_x:
        return (0.0, p.u_wall_lo), (0.0, p.u_wall_hi)
    return (0.0, 0.0), (0.0, 0.0)


def extend_velocity(ux: torch.Tensor, uy: torch.Tensor, p: Params):
    """Extend u by one ghost layer: periodic wrap; u_ghost = 2 u_w - u_mirror
    at a no-slip half-way wall (reading A9); at a free-slip wall (a plane of
    mirror symmetry) the normal component changes sign and the tangential
    one is copied.  x is extended first, then y (corners compose both)."""
    (lox, loy), (hix, hiy) = _wall_velocity(p)

    def ext(a, dim, wall, lo_w, hi_w, sign):
        n = a.shape[dim]
        if wall == 2:
            lo = sign * a.narrow(dim, 0, 1)
            hi = sign * a.narrow(dim, n - 1, 1)
        elif wall:
            lo = 2.0 * lo_w - a.narrow(dim, 0, 1)
            hi = 2.0 * hi_w - a.narrow(dim, n - 1, 1)
        else:
            lo = a.narrow(dim, n - 1, 1)
            hi = a.narrow(dim, 0, 1)
        return torch.cat([lo, a, hi], dim=dim)

    ux = ext(ux, 1, p.wall_x, lox, hix, -1.0)
    uy = ext(uy, 1, p.wall_x, loy, hiy, 1.0)
    ux = ext(ux, 0, p.wall_y, lox, hix, 1.0)
    uy = ext(uy, 0, p.wall_y, loy, hiy, -1.0)
    return ux, uy


# ----------------------------------------------------------------------------
# Isotropic central differences, Sec. III, Eqs. (41)-(42).  Each takes a field
# extended by one layer and returns values on the inner region.
# ----------------------------------------------------------------------------
def _nb(e: torch.Tensor, i: int) -> torch.Tensor:
    """Value at x + c_i for every inner node of an extended field."""
    ny, nx = e.shape[0] - 2, e.shape[1] - 2
    return e[1 + CY[i]: 1 + CY[i] + ny, 1 + CX[i]: 1 + CX[i] + nx]


def grad(e: torch.Tensor):
    """grad Psi = (1/cs^2) sum_{i=1..8} w_i c_i Psi(x + c_i)   (Eq. 41)."""
    gx = sum(WT[i] * CX[i] * _nb(e, i) for i in range(1, 9) if CX[i] != 0) / CS2
    gy = sum(WT[i] * CY[i] * _nb(e, i) for i in range(1, 9) if CY[i] != 0) / CS2
    return gx, gy


def lap(e: torch.Tensor):
    """lap Psi = (2/cs^2) sum_{i=1..8} w_i [Psi(x + c_i) - Psi(x)]   (Eq. 42)."""
    c = _nb(e, 0)
    return (2.0 / CS2) * sum(WT[i] * (_nb(e, i) - c) for i in range(1, 9))


def div(ex: torch.Tensor, ey: torch.Tensor):
    """div V = (1/cs^2) sum_i w_i c_i . V(x + c_i)  (Eq. 41 contracted)."""
    return sum(WT[i] * (CX[i] * _nb(ex, i) + CY[i] * _nb(ey, i)) for i in range(1, 9)) / CS2


def _inner(e: torch.Tensor) -> torch.Tensor:
    return e[1:-1, 1:-1]


# ----------------------------------------------------------------------------
# Chemical potential (Sec. II.A, Eq. 2; f0 = beta (1 - phi^2)^2 below Eq. 3)
# ----------------------------------------------------------------------------
def chemical_potential(phi, lap_phi, c: Const):
    """mu_phi = d f0/d phi - kappa lap(phi) = 4 beta phi (phi^2 - 1) - kappa lap(phi)."""
    return 4.0 * c.beta * phi * (phi * phi - 1.0) - c.kappa * lap_phi


# ----------------------------------------------------------------------------
# Interfacial forces, Sec. II.B.  phie2 is phi extended by two layers; the
# force is returned on the interior nodes.
# ----------------------------------------------------------------------------
def interfacial_force(phie2: torch.Tensor, form: str, p: Params, c: Const):
    gx1, gy1 = grad(phie2)                 # on the 1-layer ring + interior
    l1 = lap(phie2)
    phi1 = _inner(phie2)
    mu1 = chemical_potential(phi1, l1, c)
    gx, gy = _inner(gx1), _inner(gy1)      # interior
    if form == "stf1":                     # Eq. (17): F = -div( kappa grad(phi) (x) grad(phi) )
        txx, txy, tyy = c.kappa * gx1 * gx1, c.kappa * gx1 * gy1, c.kappa * gy1 * gy1
        return -div(txx, txy), -div(txy, tyy)
    if form == "stf2":                     # Eq. (18): F = div( kappa (|grad phi|^2 I - grad phi (x) grad phi) )
        g2 = gx1 * gx1 + gy1 * gy1
        txx, txy, tyy = c.kappa * (g2 - gx1 * gx1), -c.kappa * gx1 * gy1, c.kappa * (g2 - gy1 * gy1)
        return div(txx, txy), div(txy, tyy)
    if form == "cpf1":                     # Eq. (20): F = -phi grad(mu)
        mx, my = grad(mu1)
        phi = _inner(phi1)
        return -phi * mx, -phi * my
    if form == "cpf2":                     # Eq. (20): F = mu grad(phi)
        mu = _inner(mu1)
        return mu * gx, mu * gy
    if form == "pf1":                      # Eq. (20): F = -kappa grad(phi) lap(phi)
        lp = _inner(l1)
        return -c.kappa * gx * lp, -c.kappa * gy * lp
    if form == "pf2":                      # Eq. (20): F = kappa phi grad(lap phi)
        lx, ly = grad(l1)
        phi = _inner(phi1)
        return c.kappa * phi * lx, c.kappa * phi * ly
    if form in ("csf1", "csf2"):           # Eqs. (24)-(25) with the regularised normal (A8)
        inv = 1.0 / torch.sqrt(gx1 * gx1 + gy1 * gy1 + p.eps_n * p.eps_n)
        nx1, ny1 = gx1 * inv, gy1 * inv
        divn = div(nx1, ny1)
        if form == "csf1":                 # -kappa |grad phi|^2 n div(n)
            g2 = gx * gx + gy * gy
            return -c.kappa * g2 * _inner(nx1) * divn, -c.kappa * g2 * _inner(ny1) * divn
        return -0.5 * p.sigma * gx * divn, -0.5 * p.sigma * gy * divn
    raise ValueError(f"unknown force form {form!r}")


# ----------------------------------------------------------------------------
# Mixture properties (Sec. II.A, Eqs. 9-10) and local relaxation time (A6)
# ----------------------------------------------------------------------------
def density(phi, p: Params):
    return p.rho1 * (1.0 + phi) / 2.0 + p.rho2 * (1.0 - phi) / 2.0


def viscosity(phi, c: Const):
    return c.mu1 * (1.0 + phi) / 2.0 + c.mu2 * (1.0 - phi) / 2.0


def tau_f(phi, p: Params, c: Const):
    """mu = rho cs^2 (tau_f - 1/2)  (Sec. III, after Eq. 40)."""
    return 0.5 + viscosity(phi, c) / (CS2 * density(phi, p))


# ----------------------------------------------------------------------------
# Equilibria and source terms, Sec. III
# ----------------------------------------------------------------------------
def s_i(i: int, ux, uy):
    """s_i(u) = c_i.u / cs^2 + uu:(c_i c_i - cs^2 I) / (2 cs^4)   (Eq. 33)."""
    cu = CX[i] * ux + CY[i] * uy
    return cu / CS2 + (cu * cu - CS2 * (ux * ux + uy * uy)) / (2.0 * CS2 * CS2)


def f_eq(i, P, rho, ux, uy):
    """f_i^eq = w_i [P + cs^2 rho s_i(u)]   (Eq. 31)."""
    return WT[i] * (P + CS2 * rho * s_i(i, ux, uy))


def h_eq(i, phi, mu, ux, uy, eta):
    """h_0^eq = phi + (w_0 - 1) eta mu;  h_i^eq = w_i eta mu + w_i phi c_i.u / cs^2   (Eq. 32)."""
    if i == 0:
        return phi + (WT[0] - 1.0) * eta * mu
    return WT[i] * eta * mu + WT[i] * phi * (CX[i] * ux + CY[i] * uy) / CS2


def force_f(i, ux, uy, fx, fy, grx, gry):
    """F_i = (c_i - u) . [Gamma_i F + w_i s_i grad(cs^2 rho)],  Gamma_i = w_i (1 + s_i)
    (Eq. 35 under reading A1)."""
    s = s_i(i, ux, uy)
    gam = WT[i] * (1.0 + s)
    return ((CX[i] - ux) * (gam * fx + WT[i] * s * CS2 * grx)
            + (CY[i] - uy) * (gam * fy + WT[i] * s * CS2 * gry))


def force_h(i, a_h, divq, dqx, dqy):
    """H_i = wbar_i A_H div(u phi) + w_i c_i . d_t(phi u) / cs^2   (Eq. 36, A3)."""
    return WBAR[i] * a_h * divq + WT[i] * (CX[i] * dqx + CY[i] * dqy) / CS2


# ----------------------------------------------------------------------------
# Macroscopic fields of a pre-collision state (Eq. 37) plus everything the
# collision needs.
# ----------------------------------------------------------------------------
def macroscopic(f, h, J, rho0, form: str, p: Params, c: Const):
    phi = h.sum(0)                                       # Eq. (37), phi = sum h_i
    phie2 = extend_scalar(phi, 2, p)
    fsx, fsy = interfacial_force(phie2, form, p, c)
    phie1 = _inner(phie2)
    gx, gy = grad(phie1)
    lp = lap(phie1)
    mu = chemical_potential(phi, lp, c)
    rho = density(phi, p)
    grx, gry = grad(density(phie1, p))                  # grad rho by Eq. (41)
    fx = fsx + (rho - rho0) * p.gx                       # F_g = (rho - rho0) g  (Eq. 8)
    fy = fsy + (rho - rho0) * p.gy
    jx = sum(CX[i] * f[i] for i in range(9) if CX[i] != 0)
    jy = sum(CY[i] * f[i] for i in range(9) if CY[i] != 0)
    ux = (jx + 0.5 * CS2 * fx) / (CS2 * rho)             # Eq. (37)
    uy = (jy + 0.5 * CS2 * fy) / (CS2 * rho)
    P = f.sum(0) + 0.5 * CS2 * (ux * grx + uy * gry)     # Eq. (37)
    return dict(phi=phi, rho=rho, ux=ux, uy=uy, P=P, mu=mu, fx=fx, fy=fy,
                grx=grx, gry=gry, gx=gx, gy=gy, lap=lp)


def moments(state, form: str, p: Params):
    """phi, rho, u_x, u_y, P_sf of a state (what lbm_moments returns)."""
    c = constants(p)
    m = macroscopic(state["f"], state["h"], state["J"], state["rho0"], form, p, c)
    return {k: m[k] for k in ("phi", "rho", "ux", "uy", "P")}


# ----------------------------------------------------------------------------
# Streaming with half-way bounce-back (Eqs. 29-30 left-hand sides; Eq. 43)
# ----------------------------------------------------------------------------
def _mirror(i: int, axis: str) -> int:
    """Direction with the x (or y) component of c_i reversed."""
    cx, cy = (-CX[i], CY[i]) if axis == "x" else (CX[i], -CY[i])
    return next(j for j in range(9) if CX[j] == cx and CY[j] == cy)


def _stream(post, wall_value, p: Params):
    """post: [9, ny, nx] post-collision populations.  wall_value(i, u_w, src_mask)
    returns the moving-wall correction subtracted when direction i leaves the
    domain.  Returns the populations at the next time step.

    A link that crosses a no-slip wall bounces back to its own node (Eq. 43).
    A link that crosses only a free-slip wall is reflected specularly: the
    normal component of c_i reverses and the population lands on the node
    beside its origin, shifted along the wall by the tangential component.
    A link into a corner (both axes at once) bounces back."""
    ny, nx = p.ny, p.nx
    new = torch.zeros_like(post)
    ys = torch.arange(ny).view(ny, 1).expand(ny, nx)
    xs = torch.arange(nx).view(1, nx).expand(ny, nx)
    (lox, loy), (hix, hiy) = _wall_velocity(p)
    for i in range(9):
        dx, dy = xs + CX[i], ys + CY[i]
        out_x = (dx < 0) | (dx >= nx) if p.wall_x else torch.zeros_like(dx, dtype=torch.bool)
        out_y = (dy < 0) | (dy >= ny) if p.wall_y else torch.zeros_like(dy, dtype=torch.bool)
        dx, dy = dx % nx, dy % ny
        inside = ~(out_x | out_y)
        new[i][dy[inside], dx[inside]] = post[i][inside]
        slip_x = out_x & ~out_y if p.wall_x == 2 else torch.zeros_like(out_x)
        slip_y = out_y & ~out_x if p.wall_y == 2 else torch.zeros_like(out_y)
        if bool(slip_x.any()):           # lands on (x, y + c_iy)
            new[_mirror(i, "x")][dy[slip_x], xs[slip_x]] = post[i][slip_x]
        if bool(slip_y.any()):           # lands on (x + c_ix, y)
            new[_mirror(i, "y")][ys[slip_y], dx[slip_y]] = post[i][slip_y]
        out = ~(inside | slip_x | slip_y)
        if bool(out.any()):
            # wall velocity of the wall the link crosses (low or high side)
            uwx = torch.zeros((ny, nx), dtype=torch.float64)
            uwy = torch.zeros((ny, nx), dtype=torch.float64)
            if p.wall_y:
                lo_y, hi_y = (ys + CY[i] < 0), (ys + CY[i] >= ny)
                uwx = torch.where(lo_y, torch.full_like(uwx, lox), uwx)
                uwx = torch.where(hi_y, torch.full_like(uwx, hix), uwx)
            if p.wall_x:
                lo_x, hi_x = (xs + CX[i] < 0), (xs + CX[i] >= nx)
                uwy = torch.where(lo_x, torch.full_like(uwy, loy), uwy)
                uwy = torch.where(hi_x, torch.full_like(uwy, hiy), uwy)
            cu_w = (CX[i] * uwx + CY[i] * uwy).to(post.dtype) if not post.is_complex() else \
                (CX[i] * uwx + CY[i] * uwy).to(post.dtype)
            j = OPP[i]
            corr = wall_value(i, cu_w)
            new[j][out] = post[i][out] - corr[out]
    return new


# ----------------------------------------------------------------------------
# Initialisation (reading A11) and one time step
# ----------------------------------------------------------------------------
def resolve_rho0(phi0, p: Params):
    """Background density of F_g (A12): given value, or mean of rho(phi0)."""
    if p.rho0 is not None and not (isinstance(p.rho0, float) and math.isnan(p.rho0)):
        return float(p.rho0)
    return float(density(phi0.detach().real if phi0.is_complex() else phi0.detach(), p).mean())


def init(p: Params, phi0: torch.Tensor, ux0=None, uy0=None):
    """Initial state from phi0 (and optional u0): P0 = 0,
    f_i = f_i^eq(0, rho(phi0), u0), h_i = h_i^eq(phi0, mu(phi0), u0), J = phi0 u0."""
    c = constants(p)
    if (p.wall_x == 2 or p.wall_y == 2) and (p.u_wall_lo != 0.0 or p.u_wall_hi != 0.0):
        raise ValueError("free-slip walls do not move, and moving walls need exactly one walled axis")
    zeros = torch.zeros_like(phi0)
    ux0 = zeros if ux0 is None else ux0.to(phi0.dtype)
    uy0 = zeros if uy0 is None else uy0.to(phi0.dtype)
    mu0 = chemical_potential(phi0, lap(extend_scalar(phi0, 1, p)), c)
    rho = density(phi0, p)
    f = torch.stack([f_eq(i, zeros, rho, ux0, uy0) for i in range(9)])
    h = torch.stack([h_eq(i, phi0, mu0, ux0, uy0, c.eta) for i in range(9)])
    J = torch.stack([phi0 * ux0, phi0 * uy0])
    return dict(f=f, h=h, J=J, rho0=resolve_rho0(phi0, p), t=0)


def step(state, form: str, p: Params):
    """One time step n -> n+1 (Eqs. 29-30 with Eqs. 31-37 and 43)."""
    c = constants(p)
    f, h, J = state["f"], state["h"], state["J"]
    m = macroscopic(f, h, J, state["rho0"], form, p, c)
    phi, rho, ux, uy = m["phi"], m["rho"], m["ux"], m["uy"]
    # div(phi u) on the current node field (A5) and the explicit-Euler d_t(phi u) (A4)
    qx, qy = phi * ux, phi * uy
    uxe, uye = extend_velocity(ux, uy, p)
    phie1 = extend_scalar(phi, 1, p)
    divq = div(phie1 * uxe, phie1 * uye)
    dqx, dqy = qx - J[0], qy - J[1]
    tf = tau_f(phi, p, c)
    th = p.tau_h
    fpost, hpost = [], []
    for i in range(9):
        feq = f_eq(i, m["P"], rho, ux, uy)
        Fi = force_f(i, ux, uy, m["fx"], m["fy"], m["grx"], m["gry"])
        fpost.append(f[i] - (f[i] - feq) / tf + (1.0 - 0.5 / tf) * Fi)        # Eq. (29)
        heq = h_eq(i, phi, m["mu"], ux, uy, c.eta)
        Hi = force_h(i, c.a_h, divq, dqx, dqy)
        hpost.append(h[i] - (h[i] - heq) / th + (1.0 - 0.5 / th) * Hi)        # Eq. (30)
    fpost, hpost = torch.stack(fpost), torch.stack(hpost)
    # Eq. (43): f_opp(i)(x_f) = f_i^+(x_f) - 2 w_i rho(x_f) c_i.u_w ;
    #           h_opp(i)(x_f) = h_i^+(x_f) - 2 w_i phi(x_f) c_i.u_w / cs^2   (A10)
    fnew = _stream(fpost, lambda i, cu: 2.0 * WT[i] * rho * cu, p)
    hnew = _stream(hpost, lambda i, cu: 2.0 * WT[i] * phi * cu / CS2, p)
    return dict(f=fnew, h=hnew, J=torch.stack([qx, qy]), rho0=state["rho0"], t=state["t"] + 1)


# ----------------------------------------------------------------------------
# Hydrodynamic pressure (Sec. II.B).  Each force form moves different gradient
# terms into the generalised pressure P_sf of the momentum equation, so
# p_h = P_sf - D_form:
#   STF-1  D = -kappa |grad phi|^2        (reading A23: from Eq. 19, see below)
#   STF-2  D = 0                          (text after Eq. 18)
#   CPF-1  D = f0 - phi mu_phi - (kappa/2) |grad phi|^2      (Eq. 21)
#   CPF-2  D = f0 - (kappa/2) |grad phi|^2                   (Eq. 21)
#   PF-1   D = -(kappa/2) |grad phi|^2                       (Eq. 21)
#   PF-2   D = kappa phi lap(phi) - (kappa/2) |grad phi|^2   (Eq. 21)
#   CSF-1, CSF-2  D = 0 (the CSF force holds no gradient term; Sec. II.B after
#                  Eq. 26, the pressure of the CSF model is p_h)
# with f0 = beta (1 - phi^2)^2.  A23: the text after Eq. (17) prints
# P_stf-1 = p_h + kappa |grad phi|^2, but Eq. (19) gives
# F_stf-1 = F_pf-1 - grad(kappa |grad phi|^2 / 2), so with Eq. (21)'s
# P_pf-1 = p_h - (kappa/2)|grad phi|^2 the consistent value is
# P_stf-1 = p_h - kappa |grad phi|^2 (the same follows from Eq. 26 against
# STF-2).  Derivatives are the isotropic stencils of Eqs. (41)-(42).
# ----------------------------------------------------------------------------
def pressure_offset(m, form: str, c: Const):
    """D_form of a macroscopic() result m (fields phi, mu, gx, gy, lap)."""
    phi = m["phi"]
    g2 = m["gx"] * m["gx"] + m["gy"] * m["gy"]
    f0 = c.beta * (1.0 - phi * phi) ** 2
    if form == "stf1":
        return -c.kappa * g2
    if form in ("stf2", "csf1", "csf2"):
        return torch.zeros_like(phi)
    if form == "cpf1":
        return f0 - phi * m["mu"] - 0.5 * c.kappa * g2
    if form == "cpf2":
        return f0 - 0.5 * c.kappa * g2
    if form == "pf1":
        return -0.5 * c.kappa * g2
    if form == "pf2":
        return c.kappa * phi * m["lap"] - 0.5 * c.kappa * g2
    raise ValueError(f"unknown force form {form!r}")


def hydro_pressure(state, form: str, p: Params):
    """p_h = P_sf - D_form of a state (what lbm_hydro_pressure returns)."""
    c = constants(p)
    m = macroscopic(state["f"], state["h"], state["J"], state["rho0"], form, p, c)
    return m["P"] - pressure_offset(m, form, c)


def run(state, form: str, p: Params, nsteps: int):
    for _ in range(nsteps):
        state = step(state, form, p)
    return state


# ----------------------------------------------------------------------------
# Diagnostics used by the tests and the benchmark configurations
# ----------------------------------------------------------------------------
def laplace_sigma(mom, p: Params):
    """sigma_num = R_num (p_in - p_out)  (Sec. V.A, Laplace law); R_num from the
    area of fluid 1, p_in at the centre node, p_out at the corner node."""
    area = ((1.0 + mom["phi"]) / 2.0).sum()
    r_num = torch.sqrt(area / math.pi)
    p_in = mom["P"][p.ny // 2, p.nx // 2]
    p_out = mom["P"][0, 0]
    return float(r_num * (p_in - p_out)), float(r_num)
