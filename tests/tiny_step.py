"""A second, independent FP64 implementation of the coupled time step, for
tiny lattices only: plain per-node Python loops written from the paper's
equations (Sec. 2A-2C) and the readings recorded in the design notes, with
no code shared with the C oracle (no D2Q9 tables, no MRT matrix, no EOS
routine of its own).  The test ``test_oracle_tiny.py`` runs both on a few
steps of 7x5 lattices with every boundary kind and compares every stored
value; this pins the oracle's indexing and boundary rules where no closed
form exists (corners, inlet temperature, outlets, heater sums).

TEST INFRASTRUCTURE ONLY.
"""
from __future__ import annotations

import math

import numpy as np

# D2Q9, App. A ordering: rest, +x, +y, -x, -y, (+,+), (-,+), (-,-), (+,-)
VEL = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
WT = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4


def opposite(i):
    cx, cy = VEL[i]
    return VEL.index((-cx, -cy))


def mrt_rows():
    """Lallemand-Luo moment basis, built from its definitions: density,
    energy e = -4 + 3|c|^2, energy square eps = 4 - 21/2 |c|^2 + 9/2 |c|^4,
    momenta, heat fluxes q = (-5 + 3|c|^2) c, stresses cx^2 - cy^2, cx cy."""
    M = np.zeros((9, 9))
    for i, (cx, cy) in enumerate(VEL):
        c2 = cx * cx + cy * cy
        M[0, i] = 1
        M[1, i] = -4 + 3 * c2
        M[2, i] = 4 - 10.5 * c2 + 4.5 * c2 * c2
        M[3, i] = cx
        M[4, i] = (-5 + 3 * c2) * cx
        M[5, i] = cy
        M[6, i] = (-5 + 3 * c2) * cy
        M[7, i] = cx * cx - cy * cy
        M[8, i] = cx * cy
    return M


def equilibrium(rho, ux, uy):
    out = np.zeros(9)
    for i, (cx, cy) in enumerate(VEL):
        cu = cx * ux + cy * uy
        out[i] = WT[i] * rho * (1 + cu / (1 / 3) + cu * cu / (2 / 9) - (ux * ux + uy * uy) / (2 / 3))
    return out


class PR:
    """Peng-Robinson EOS (Eq. 12) with alpha(T) read as
    [1 + kappa (1 - sqrt(T/Tc))]^2 and Tc from b = 0.0778 R Tc / pc and
    a = 0.45724 R^2 Tc^2 / pc."""

    def __init__(self, a, b, R, omega):
        self.a, self.b, self.R = a, b, R
        self.kappa = 0.37464 + 1.54226 * omega - 0.26992 * omega ** 2
        pc_over_Tc = 0.0778 * R / b                   # from b
        self.Tc = a * pc_over_Tc / (0.45724 * R * R)  # from a = 0.45724 R^2 Tc / (pc / Tc)

    def alpha(self, T):
        return (1 + self.kappa * (1 - math.sqrt(T / self.Tc))) ** 2

    def p(self, rho, T):
        a, b, R = self.a, self.b, self.R
        return rho * R * T / (1 - b * rho) - a * self.alpha(T) * rho ** 2 / (1 + 2 * b * rho - (b * rho) ** 2)

    def dp_dT(self, rho, T):
        # analytic derivative of alpha: d/dT [1 + k(1 - sqrt(T/Tc))]^2
        a, b, R = self.a, self.b, self.R
        s = math.sqrt(T / self.Tc)
        dalpha = 2 * (1 + self.kappa * (1 - s)) * (-self.kappa) * 0.5 / math.sqrt(T * self.Tc)
        return rho * R / (1 - b * rho) - a * dalpha * rho ** 2 / (1 + 2 * b * rho - (b * rho) ** 2)


class TinyLBM:
    """State: post-collision f*, g* [9][ny][nx], outlet memory for directions
    3, 6, 7 at x = nx - 1, and the lagged mean density."""

    def __init__(self, P, Tw_s, rw_s, Tw_n, rw_n, heater, rho0, T0):
        self.P = P
        self.nx, self.ny = P.nx, P.ny
        self.eos = PR(P.a, P.b, P.R, P.omega)
        self.Tw = {-1: np.asarray(Tw_s, float), 1: np.asarray(Tw_n, float)}
        self.psiw = {}
        for side, rw in ((-1, rw_s), (1, rw_n)):
            self.psiw[side] = np.array([self.psi(r, t) for r, t in zip(np.asarray(rw, float), self.Tw[side])])
        self.heater = np.asarray(heater, int)
        self.fs = np.array([WT[i] * rho0 for i in range(9)])
        self.gs = np.array([WT[i] * T0 for i in range(9)])
        self.fold = {i: self.fs[i, :, self.nx - 1].copy() for i in (3, 6, 7)}
        self.rbar = float(np.mean(rho0))
        M = mrt_rows()
        s_nu, s_e, s_eps, s_q = P.rates()
        S = np.diag([0, s_e, s_eps, 0, s_q, 0, s_q, s_nu, s_nu])
        self.Coll = np.linalg.inv(M) @ S @ M

    def psi(self, rho, T):
        q = 2 * (self.eos.p(rho, T) - rho / 3) / (self.P.c0 * self.P.g)
        return math.sqrt(q) if q > 0 else 0.0

    # ---- geometry
    def solid(self, y):
        return self.P.bc_y == 1 and (y < 0 or y >= self.ny)

    def wall_col(self, x):
        return x % self.nx if self.P.bc_x == 0 else min(max(x, 0), self.nx - 1)

    def side(self, y):
        return -1 if y < 0 else 1

    # ---- one step
    def streamed(self):
        P, nx, ny = self.P, self.nx, self.ny
        f = np.zeros((9, ny, nx))
        g = np.zeros((9, ny, nx))
        for y in range(ny):
            for x in range(nx):
                for i, (cx, cy) in enumerate(VEL):
                    xs, ys = x - cx, y - cy
                    if self.solid(ys):
                        o = opposite(i)
                        Tw = self.Tw[self.side(ys)][self.wall_col(xs)]
                        f[i, y, x] = self.fs[o, y, x]
                        g[i, y, x] = -self.gs[o, y, x] + 2 * WT[i] * Tw
                        continue
                    ys %= ny
                    if P.bc_x == 0:
                        xs %= nx
                    elif not 0 <= xs < nx:
                        continue  # ghost column, set below
                    f[i, y, x] = self.fs[i, ys, xs]
                    g[i, y, x] = self.gs[i, ys, xs]
        if P.bc_x == 0:
            return f, g
        u = P.u_in
        for y in range(ny):
            # inlet x = 0: unknowns are the right-moving populations whose
            # source is the ghost column (not a wall cell)
            fn = f[:, y, 0]
            rin = (fn[0] + fn[2] + fn[4] + 2 * (fn[3] + fn[6] + fn[7])) / (1 - u)
            d24 = fn[2] - fn[4]
            new = {1: fn[3] + 2 / 3 * rin * u, 5: fn[7] - d24 / 2 + rin * u / 6, 8: fn[6] + d24 / 2 + rin * u / 6}
            for i in (1, 5, 8):
                if not self.solid(y - VEL[i][1]):
                    f[i, y, 0] = new[i]
                    geq_even = WT[i] * P.T_in * (1 + 4.5 * u * u - 1.5 * u * u)
                    g[i, y, 0] = -self.gs[opposite(i), y, 0] + 2 * geq_even
        X = nx - 1
        if P.bc_x == 2:
            for y in range(ny):
                near_wall = self.solid(y - 1) or self.solid(y + 1)
                if near_wall:
                    for i in (3, 6, 7):
                        if not self.solid(y - VEL[i][1]):
                            f[i, y, X] = f[i, y, X - 1]
                            g[i, y, X] = g[i, y, X - 1]
                    continue
                fn = f[:, y, X]
                ro = P.rho_out
                uo = -1 + (fn[0] + fn[2] + fn[4] + 2 * (fn[1] + fn[5] + fn[8])) / ro
                d24 = fn[2] - fn[4]
                f[3, y, X] = fn[1] - 2 / 3 * ro * uo
                f[6, y, X] = fn[8] - d24 / 2 - ro * uo / 6
                f[7, y, X] = fn[5] + d24 / 2 - ro * uo / 6
                for i in (3, 6, 7):
                    g[i, y, X] = g[i, y, X - 1]
            return f, g
        U = P.u_in if P.U_out is None else P.U_out
        newfold = {}
        for i in (3, 6, 7):
            newfold[i] = np.zeros(ny)
            for y in range(ny):
                if not self.solid(y - VEL[i][1]):
                    f[i, y, X] = (self.fold[i][y] + U * f[i, y, X - 1]) / (1 + U)
                    g[i, y, X] = g[i, y, X - 1]
                newfold[i][y] = f[i, y, X]
        self._newfold = newfold
        return f, g

    def evaluate(self):
        P, nx, ny = self.P, self.nx, self.ny
        f, g = self.streamed()
        rho = f.sum(axis=0)
        jx = sum(VEL[i][0] * f[i] for i in range(9))
        jy = sum(VEL[i][1] * f[i] for i in range(9))
        T = np.full((ny, nx), P.T_iso) if P.isothermal else g.sum(axis=0)
        p = np.vectorize(self.eos.p)(rho, T)
        psi = np.vectorize(self.psi)(rho, T)
        dpdT = np.vectorize(self.eos.dp_dT)(rho, T)
        g1, g2 = 2 * P.g, P.g / 2
        G_wet = P.neutral_G_wet if P.G_wet is None else P.G_wet
        Fx = np.zeros((ny, nx))
        Fy = np.zeros((ny, nx))
        for y in range(ny):
            for x in range(nx):
                sx = sy = 0.0
                for i in range(1, 9):
                    cx, cy = VEL[i]
                    G = g1 if abs(cx) + abs(cy) == 1 else g2
                    x1, y1 = x + cx, y + cy
                    if self.solid(y1):
                        pw = self.psiw[self.side(y1)][self.wall_col(x1)]
                        sx += -G_wet * psi[y, x] * WT[i] * pw * cx
                        sy += -G_wet * psi[y, x] * WT[i] * pw * cy
                        continue
                    y1 %= ny
                    x1 = x1 % nx if P.bc_x == 0 else min(max(x1, 0), nx - 1)
                    q = psi[y1, x1]
                    sx += -P.beta * psi[y, x] * G * q * cx - (1 - P.beta) / 2 * G * q * q * cx
                    sy += -P.beta * psi[y, x] * G * q * cy - (1 - P.beta) / 2 * G * q * q * cy
                if P.single_phase:
                    sx = sy = 0.0
                Fx[y, x] = sx + (rho[y, x] - self.rbar) * P.ga_x + P.fb_x
                Fy[y, x] = sy + (rho[y, x] - self.rbar) * P.ga_y + P.fb_y
        ux, uy = jx / rho, jy / rho
        uax, uay = ux + Fx / (2 * rho), uy + Fy / (2 * rho)
        phi = np.zeros((ny, nx))
        for y in range(ny):
            for x in range(nx):
                if P.bc_x == 0:
                    xe, xw = (x + 1) % nx, (x - 1) % nx
                else:
                    xe, xw = min(x + 1, nx - 1), max(x - 1, 0)
                dux = (uax[y, xe] - uax[y, xw]) / 2
                # ghost of a wall cell: the wall node's own u_y for the
                # advective part, its mirror for the compression part
                nb = {}
                for dy in (1, -1):
                    if self.solid(y + dy):
                        nb[dy] = (uay[y, x], -uay[y, x])
                    else:
                        v = uay[(y + dy) % ny, x]
                        nb[dy] = (v, v)
                div_adv = dux + (nb[1][0] - nb[-1][0]) / 2
                div_mass = dux + (nb[1][1] - nb[-1][1]) / 2
                phi[y, x] = T[y, x] * div_adv - T[y, x] * dpdT[y, x] / (rho[y, x] * P.c_v) * div_mass
        return dict(f=f, g=g, rho=rho, ux=ux, uy=uy, T=T, p=p, psi=psi, Fx=Fx, Fy=Fy, uax=uax, uay=uay,
                    phi=phi)

    def step(self):
        P = self.P
        s = self.evaluate()
        ny, nx = self.ny, self.nx
        for y in range(ny):
            for x in range(nx):
                rho = s["rho"][y, x]
                ux, uy = s["ux"][y, x], s["uy"][y, x]
                dux, duy = s["Fx"][y, x] / rho, s["Fy"][y, x] / rho
                fv = s["f"][:, y, x]
                e0 = equilibrium(rho, ux, uy)
                self.fs[:, y, x] = fv - self.Coll @ (fv - e0) + (equilibrium(rho, ux + dux, uy + duy) - e0)
                if not P.isothermal:
                    gv = s["g"][:, y, x]
                    ge = equilibrium(s["T"][y, x], s["uax"][y, x], s["uay"][y, x])
                    self.gs[:, y, x] = gv - (gv - ge) / P.tau_g + np.array(WT) * s["phi"][y, x]
        if P.bc_x == 1:
            self.fold = self._newfold
        self.rbar = float(s["rho"].mean())

    def diag(self):
        s = self.evaluate()
        P = self.P
        q = 0.0
        if P.bc_y == 1:
            q = sum(2 * (self.Tw[-1][x] - s["T"][0, x]) for x in range(self.nx) if self.heater[x])
        return dict(mass=s["rho"].sum(), energy=s["T"].sum(), heater_q=q,
                    vapor_cells=float((s["rho"] < P.rho_mid).sum()),
                    p_in=s["p"][self.ny // 2, 0], p_out=s["p"][self.ny // 2, self.nx - 1])
