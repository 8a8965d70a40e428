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


def test_pressure_exit_corners_take_zero_gradient(oracle_mod):
    """Outlet nodes next to a wall: the populations from the ghost column
    equal those at x = nx-2 (zero gradient), the wall's own ones stay."""
    O = oracle_mod
    Ts = _ts(O)
    rl, rv, _ = O.maxwell(Ts)
    P = O.Params(nx=20, ny=12, bc_x=O.BCX_CHANNEL_P, bc_y=O.BCY_WALLS, rho_out=rl, T_in=0.95 * Ts,
                 T_iso=Ts, rho_mid=0.5 * (rl + rv), u_in=0.01)
    o = O.Oracle(P)
    o.set_wall(0, Ts, 3.8)
    o.set_wall(1, Ts, 3.8)
    o.init(rho_u=rl, T_u=Ts, noise=0.05, seed=5)
    o.step(2)
    f, g = o.streamed()
    for y, ghost in ((0, (3, 7)), (P.ny - 1, (3, 6))):
        for i in ghost:
            assert f[i, y, -1] == f[i, y, -2] and g[i, y, -1] == g[i, y, -2]


def test_pressure_exit_channel_stays_bounded(oracle_mod):
    """Regression for the corner rule: the multiphase channel of the paper's
    cross-section (40 rows, Re_in = 0.96, T_in = 0.9 Tc, exit at rho_l),
    40 x 250, 20000 steps.  With the Zou-He completion also applied next to
    the walls, the corner velocity grows from ~0.05 and the run fails near
    step 16500."""
    O = oracle_mod
    Tc = O.crit_temperature()
    Tin = 0.9 * Tc
    rl, rv, _ = O.maxwell(Tin)
    nx, ny = 250, 40
    P = O.Params(nx=nx, ny=ny, bc_x=O.BCX_CHANNEL_P, bc_y=O.BCY_WALLS, rho_out=rl, u_in=0.96 / 6.0 / ny,
                 T_in=Tin, T_iso=Tin, rho_mid=0.5 * (rl + rv))
    o = O.Oracle(P)
    rw = rv + 0.6 * (rl - rv)
    o.set_wall(0, np.full(nx, Tin), np.full(nx, rw))
    o.set_wall(1, np.full(nx, Tin), np.full(nx, rw))
    o.init(rho_u=rl, T_u=Tin, noise=1e-3, seed=11)
    o.step(20000)
    F = o.fields()
    assert np.isfinite(F["rho"]).all() and np.isfinite(F["T"]).all()
    assert max(np.abs(F["ux"]).max(), np.abs(F["uy"]).max()) < 0.08
    assert F["T"].min() > 0.85 * Tc
