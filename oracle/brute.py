"""Brute-force per-cell reference of one phase-field LBM step (oracle).

TEST INFRASTRUCTURE ONLY -- imported by tests/ to pin the vectorised oracle.

Written independently of ``lbm_ref``: plain Python floats, nested loops over
cells and directions, and neighbour lookup through an index map (wrap on a
periodic axis, mirror about the half-way wall otherwise) instead of padded
arrays.  Same equations (arXiv:2012.14729, Sec. II-IV) and the same readings
(A1, A3-A6, A8-A12, A18).  Intended for grids of about 8x8.
"""
from __future__ import annotations

import math

C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W = [4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36]
CS2 = 1 / 3


def _opp(i):
    cx, cy = C[i]
    return C.index((-cx, -cy))


class Brute:
    def __init__(self, nx, ny, wall_x=0, wall_y=0, u_lo=0.0, u_hi=0.0, rho1=1.0, rho2=1.0,
                 nu1=0.1, nu2=0.1, sigma=0.01, Wd=4.0, M=0.1, tau_h=0.8, gx=0.0, gy=0.0,
                 rho0=None, eps=1e-6):
        self.nx, self.ny = nx, ny
        self.wx, self.wy = wall_x, wall_y
        self.u_lo, self.u_hi = u_lo, u_hi
        self.rho1, self.rho2 = rho1, rho2
        self.mu1, self.mu2 = rho1 * nu1, rho2 * nu2
        self.sigma = sigma
        self.beta = 0.75 * sigma / Wd
        self.kappa = 0.375 * Wd * sigma
        self.eta = M / (CS2 * (tau_h - 0.5))
        self.tau_h = tau_h
        t2 = tau_h ** 2 - tau_h + 1 / 6
        self.ah = 3 * t2 / (tau_h * (tau_h - 0.5))
        self.gx, self.gy = gx, gy
        self.rho0 = rho0
        self.eps = eps

    # -- neighbour index map ------------------------------------------------
    def _map(self, k, n, wall):
        if 0 <= k < n:
            return k
        if not wall:
            return k % n
        return -1 - k if k < 0 else 2 * n - 1 - k

    def at(self, fld, x, y):
        return fld[self._map(y, self.ny, self.wy)][self._map(x, self.nx, self.wx)]

    def wall_u(self, side):
        """side: 'lo' or 'hi' -> wall velocity vector."""
        u = self.u_lo if side == "lo" else self.u_hi
        if self.wy:
            return (u, 0.0)
        if self.wx:
            return (0.0, u)
        return (0.0, 0.0)

    def vel_at(self, ux, uy, x, y):
        """Velocity with the ghost rule u_g = 2 u_w - u_mirror for one layer."""
        vx, vy = self.at(ux, x, y), self.at(uy, x, y)
        for coord, n, wall in ((x, self.nx, self.wx), (y, self.ny, self.wy)):
            if wall and (coord < 0 or coord >= n):
                w = self.wall_u("lo" if coord < 0 else "hi")
                vx, vy = 2 * w[0] - vx, 2 * w[1] - vy
        return vx, vy

    # -- point-wise stencils on a callable field g(x, y) ----------------------
    @staticmethod
    def grad_pt(g, x, y):
        sx = sy = 0.0
        for i in range(1, 9):
            v = g(x + C[i][0], y + C[i][1])
            sx += W[i] * C[i][0] * v
            sy += W[i] * C[i][1] * v
        return sx / CS2, sy / CS2

    @staticmethod
    def lap_pt(g, x, y):
        c = g(x, y)
        s = 0.0
        for i in range(1, 9):
            s += W[i] * (g(x + C[i][0], y + C[i][1]) - c)
        return 2 * s / CS2

    @staticmethod
    def div_pt(gx, gy, x, y):
        s = 0.0
        for i in range(1, 9):
            s += W[i] * (C[i][0] * gx(x + C[i][0], y + C[i][1]) + C[i][1] * gy(x + C[i][0], y + C[i][1]))
        return s / CS2

    # -- physics ---------------------------------------------------------------
    def rho_of(self, phi):
        return self.rho1 * (1 + phi) / 2 + self.rho2 * (1 - phi) / 2

    def mu_of(self, phi):
        return self.mu1 * (1 + phi) / 2 + self.mu2 * (1 - phi) / 2

    def force(self, phi, form, x, y):
        P = lambda a, b: self.at(phi, a, b)
        G = lambda a, b: self.grad_pt(P, a, b)
        L = lambda a, b: self.lap_pt(P, a, b)
        MU = lambda a, b: 4 * self.beta * P(a, b) * (P(a, b) ** 2 - 1) - self.kappa * L(a, b)
        k = self.kappa
        if form in ("stf1", "stf2"):
            def T(a, b):
                gx, gy = G(a, b)
                if form == "stf1":
                    return -k * gx * gx, -k * gx * gy, -k * gy * gy
                g2 = gx * gx + gy * gy
                return k * (g2 - gx * gx), -k * gx * gy, k * (g2 - gy * gy)
            fx = self.div_pt(lambda a, b: T(a, b)[0], lambda a, b: T(a, b)[1], x, y)
            fy = self.div_pt(lambda a, b: T(a, b)[1], lambda a, b: T(a, b)[2], x, y)
            return fx, fy
        if form == "cpf1":
            mx, my = self.grad_pt(MU, x, y)
            return -P(x, y) * mx, -P(x, y) * my
        if form == "cpf2":
            gx, gy = G(x, y)
            return MU(x, y) * gx, MU(x, y) * gy
        if form == "pf1":
            gx, gy = G(x, y)
            return -k * gx * L(x, y), -k * gy * L(x, y)
        if form == "pf2":
            lx, ly = self.grad_pt(L, x, y)
            return k * P(x, y) * lx, k * P(x, y) * ly
        if form in ("csf1", "csf2"):
            def N(a, b):
                gx, gy = G(a, b)
                r = math.sqrt(gx * gx + gy * gy + self.eps ** 2)
                return gx / r, gy / r
            dn = self.div_pt(lambda a, b: N(a, b)[0], lambda a, b: N(a, b)[1], x, y)
            gx, gy = G(x, y)
            if form == "csf1":
                nx_, ny_ = N(x, y)
                g2 = gx * gx + gy * gy
                return -k * g2 * nx_ * dn, -k * g2 * ny_ * dn
            return -0.5 * self.sigma * gx * dn, -0.5 * self.sigma * gy * dn
        raise ValueError(form)

    def init(self, phi0, ux0=None, uy0=None):
        nx, ny = self.nx, self.ny
        ux0 = ux0 or [[0.0] * nx for _ in range(ny)]
        uy0 = uy0 or [[0.0] * nx for _ in range(ny)]
        if self.rho0 is None:
            self.rho0 = sum(self.rho_of(phi0[y][x]) for y in range(ny) for x in range(nx)) / (nx * ny)
        f = [[[0.0] * nx for _ in range(ny)] for _ in range(9)]
        h = [[[0.0] * nx for _ in range(ny)] for _ in range(9)]
        J = [[[0.0] * nx for _ in range(ny)] for _ in range(2)]
        P = lambda a, b: self.at(phi0, a, b)
        for y in range(ny):
            for x in range(nx):
                ph = phi0[y][x]
                mu = 4 * self.beta * ph * (ph * ph - 1) - self.kappa * self.lap_pt(P, x, y)
                ux, uy = ux0[y][x], uy0[y][x]
                rho = self.rho_of(ph)
                for i in range(9):
                    cu = C[i][0] * ux + C[i][1] * uy
                    s = cu / CS2 + (cu * cu - CS2 * (ux * ux + uy * uy)) / (2 * CS2 * CS2)
                    f[i][y][x] = W[i] * CS2 * rho * s
                    if i == 0:
                        h[i][y][x] = ph + (W[0] - 1) * self.eta * mu
                    else:
                        h[i][y][x] = W[i] * self.eta * mu + W[i] * ph * cu / CS2
                J[0][y][x] = ph * ux
                J[1][y][x] = ph * uy
        return f, h, J

    def moments(self, f, h, form):
        nx, ny = self.nx, self.ny
        phi = [[sum(h[i][y][x] for i in range(9)) for x in range(nx)] for y in range(ny)]
        out = {k: [[0.0] * nx for _ in range(ny)] for k in ("phi", "rho", "ux", "uy", "P", "mu", "fx", "fy", "grx", "gry")}
        R = lambda a, b: self.rho_of(self.at(phi, a, b))
        Pf = lambda a, b: self.at(phi, a, b)
        for y in range(ny):
            for x in range(nx):
                ph = phi[y][x]
                rho = self.rho_of(ph)
                fx, fy = self.force(phi, form, x, y)
                fx += (rho - self.rho0) * self.gx
                fy += (rho - self.rho0) * self.gy
                jx = sum(C[i][0] * f[i][y][x] for i in range(9))
                jy = sum(C[i][1] * f[i][y][x] for i in range(9))
                ux = (jx + 0.5 * CS2 * fx) / (CS2 * rho)
                uy = (jy + 0.5 * CS2 * fy) / (CS2 * rho)
                grx, gry = self.grad_pt(R, x, y)
                out["phi"][y][x] = ph
                out["rho"][y][x] = rho
                out["ux"][y][x] = ux
                out["uy"][y][x] = uy
                out["P"][y][x] = sum(f[i][y][x] for i in range(9)) + 0.5 * CS2 * (ux * grx + uy * gry)
                out["mu"][y][x] = 4 * self.beta * ph * (ph * ph - 1) - self.kappa * self.lap_pt(Pf, x, y)
                out["fx"][y][x], out["fy"][y][x] = fx, fy
                out["grx"][y][x], out["gry"][y][x] = grx, gry
        return out

    def step(self, f, h, J, form):
        nx, ny = self.nx, self.ny
        m = self.moments(f, h, form)
        phi, ux, uy = m["phi"], m["ux"], m["uy"]
        Qx = lambda a, b: self.at(phi, a, b) * self.vel_at(ux, uy, a, b)[0]
        Qy = lambda a, b: self.at(phi, a, b) * self.vel_at(ux, uy, a, b)[1]
        fn = [[[0.0] * nx for _ in range(ny)] for _ in range(9)]
        hn = [[[0.0] * nx for _ in range(ny)] for _ in range(9)]
        Jn = [[[0.0] * nx for _ in range(ny)] for _ in range(2)]
        th = self.tau_h
        for y in range(ny):
            for x in range(nx):
                ph, rho = phi[y][x], m["rho"][y][x]
                vx, vy = ux[y][x], uy[y][x]
                tf = 0.5 + self.mu_of(ph) / (CS2 * rho)
                dq = self.div_pt(Qx, Qy, x, y)
                qx, qy = ph * vx, ph * vy
                dtx, dty = qx - J[0][y][x], qy - J[1][y][x]
                Jn[0][y][x], Jn[1][y][x] = qx, qy
                for i in range(9):
                    cx, cy = C[i]
                    cu = cx * vx + cy * vy
                    s = cu / CS2 + (cu * cu - CS2 * (vx * vx + vy * vy)) / (2 * CS2 * CS2)
                    feq = W[i] * (m["P"][y][x] + CS2 * rho * s)
                    gam = W[i] * (1 + s)
                    Fi = ((cx - vx) * (gam * m["fx"][y][x] + W[i] * s * CS2 * m["grx"][y][x])
                          + (cy - vy) * (gam * m["fy"][y][x] + W[i] * s * CS2 * m["gry"][y][x]))
                    fp = f[i][y][x] - (f[i][y][x] - feq) / tf + (1 - 0.5 / tf) * Fi
                    if i == 0:
                        heq = ph + (W[0] - 1) * self.eta * m["mu"][y][x]
                    else:
                        heq = W[i] * self.eta * m["mu"][y][x] + W[i] * ph * cu / CS2
                    wb = W[0] - 1 if i == 0 else W[i]
                    Hi = wb * self.ah * dq + W[i] * (cx * dtx + cy * dty) / CS2
                    hp = h[i][y][x] - (h[i][y][x] - heq) / th + (1 - 0.5 / th) * Hi
                    # streaming / bounce-back
                    tx, ty = x + cx, y + cy
                    crossed = None
                    if self.wx and not (0 <= tx < nx):
                        crossed = "lo" if tx < 0 else "hi"
                    if self.wy and not (0 <= ty < ny):
                        crossed = "lo" if ty < 0 else "hi"
                    if crossed is None:
                        fn[i][ty % ny][tx % nx] = fp
                        hn[i][ty % ny][tx % nx] = hp
                    else:
                        uw = self.wall_u(crossed)
                        cuw = cx * uw[0] + cy * uw[1]
                        o = _opp(i)
                        fn[o][y][x] = fp - 2 * W[i] * rho * cuw
                        hn[o][y][x] = hp - 2 * W[i] * ph * cuw / CS2
        return fn, hn, Jn
