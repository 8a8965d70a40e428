"""Pins of the oracle's constant-pressure exit (Sec. 2C: non-equilibrium
bounce-back at a fixed outlet density rho_out, zero temperature gradient).

* Definition: after streaming and boundary conditions, every outlet node off
  the walls holds exactly density rho_out and zero transverse momentum,
  whatever the state (mass and y-momentum of the Zou-He completion).
* Closed form: a single-phase channel fed at the inlet with u_in and held at
  rho_out at the exit reaches the Hagen-Poiseuille state: constant mass flux
  along x, and a pressure gradient dp/dx = -12 mu U / H^2 (c_s^2 = 1/3,
  mu = rho nu, H = ny between halfway bounce-back walls)."""
import numpy as np
import pytest


def _ts(O):
    return 0.86 * O.crit_temperature()


def test_outlet_node_density_and_transverse_momentum(oracle_mod):
    O = oracle_mod
    Ts = _ts(O)
    rl, rv, _ = O.maxwell(Ts)
    for bcy, rows in ((O.BCY_PERIODIC, slice(0, 12)), (O.BCY_WALLS, slice(1, 11))):
        for rho_out in (rl, 0.93 * rl):
            P = O.Params(nx=20, ny=12, bc_x=O.BCX_CHANNEL_P, bc_y=bcy, rho_out=rho_out, T_in=0.95 * Ts,
                         T_iso=Ts, rho_mid=0.5 * (rl + rv), u_in=0.01)
            o = O.Oracle(P)
            if bcy == O.BCY_WALLS:
                o.set_wall(0, Ts, 3.8)
                o.set_wall(1, Ts, 3.8)
            o.init(rho_u=rl, T_u=Ts, noise=0.05, seed=3)
            for _ in range(3):
                o.step(1)
                f, _g = o.streamed()
                col = f[:, rows, -1]
                rho = col.sum(axis=0)
                jy = (O.CY[:, None] * col).sum(axis=0)
                assert np.abs(rho - rho_out).max() < 1e-13 * rho_out
                assert np.abs(jy).max() < 1e-13 * rho_out
                # the outflow is not trivial: x-momentum differs from zero
                jx = (O.CX[:, None] * col).sum(axis=0)
                assert np.abs(jx).max() > 1e-5


def test_hagen_poiseuille_with_pressure_outlet(oracle_mod):
    O = oracle_mod
    Ts = _ts(O)
    nx, ny, u_in, rho_out = 96, 16, 0.01, 1.0
    P = O.Params(nx=nx, ny=ny, bc_x=O.BCX_CHANNEL_P, bc_y=O.BCY_WALLS, isothermal=1, single_phase=1,
                 T_iso=Ts, T_in=Ts, ga_y=0.0, u_in=u_in, rho_out=rho_out)
    o = O.Oracle(P)
    o.set_wall(0, Ts, 1.0)
    o.set_wall(1, Ts, 1.0)
    o.init(rho_u=1.0, T_u=Ts)
    o.step(15000)
    F = o.fields()
    rho, ux = F["rho"], F["ux"]
    # Mass flux through each column.  A weakly damped odd-even (checkerboard)
    # acoustic mode between the two open ends (relative amplitude ~5e-4 here,
    # decaying by ~1.3 % per 1000 steps) cancels in averages of neighbouring
    # columns.
    q = (rho * ux).sum(axis=0)
    q2 = 0.5 * (q[:-1] + q[1:])
    assert np.abs(q2[5:] - q2[5:].mean()).max() < 5e-5 * q2.mean()
    # the inlet imposes u_in on the rows away from the walls
    assert np.abs(ux[1:-1, 0] - u_in).max() < 1e-12
    # fully developed pressure drop between x = 30 and x = 70
    x0, x1 = 30, 70
    p0, p1 = rho[:, x0 - 1:x0 + 1].mean() / 3.0, rho[:, x1 - 1:x1 + 1].mean() / 3.0
    rbar = rho[:, x0:x1 + 1].mean()
    U = q2.mean() / (rbar * ny)
    nu = (P.tau_f - 0.5) / 3.0
    dpdx_theory = -12.0 * rbar * nu * U / ny**2
    assert (p1 - p0) / (x1 - x0) == pytest.approx(dpdx_theory, rel=0.01)
    # the exit holds rho_out on the rows away from the walls
    assert np.abs(rho[1:-1, -1] - rho_out).max() < 1e-12
