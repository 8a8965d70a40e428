"""Pins of the buoyancy force of Eq. 14 (Sec. 2A): its sign and magnitude
through the momentum it puts into a uniform bulk, and the time level of the
domain-average density it uses."""
import numpy as np
import pytest


def _slab(O, ga_x, ga_y, nx=4, ny=48, relax=3000):
    """Flat liquid slab in vapour (periodic box, isothermal at 0.86 Tc),
    relaxed without gravity, then copied into two oracles, one with g_a and
    one without, that share the state and its lagged mean."""
    Ts = 0.86 * O.crit_temperature()
    rl, rv, _ = O.maxwell(Ts)
    base = dict(nx=nx, ny=ny, bc_x=O.BCX_PERIODIC, bc_y=O.BCY_PERIODIC, isothermal=1, T_iso=Ts, T_in=Ts)
    o = O.Oracle(O.Params(ga_x=0.0, ga_y=0.0, **base))
    y = np.arange(ny)
    prof = rv + (rl - rv) * 0.5 * (np.tanh((y - ny / 4) / 2) - np.tanh((y - 3 * ny / 4) / 2))
    o.init(rho0=np.tile(prof[:, None], (1, nx)), T_u=Ts)
    o.step(relax)
    fs, gs = o.state()
    out = []
    for gx, gy in ((ga_x, ga_y), (0.0, 0.0)):
        q = O.Oracle(O.Params(ga_x=gx, ga_y=gy, **base))
        q.init(rho_u=1.0, T_u=Ts)
        q.set_state(fs, gs)
        q.set_rbar(o.rbar())
        out.append(q)
    return out, rl, rv


def _momentum(o):
    f, _ = o.streamed()
    from oracle.oracle import CX, CY
    return np.tensordot(CX, f, axes=1), np.tensordot(CY, f, axes=1)


def test_buoyancy_pushes_bulk_momentum(oracle_mod):
    """Newton's law on the collision invariant: one step adds F to the
    momentum of every node, and in a uniform bulk streaming moves as much
    momentum in as out, so the difference the buoyancy makes to the bulk
    momentum after one step is Eq. 14's force density g_a (rho - rho_avg)
    itself: pointing along g_a in the liquid (denser than the mean), against
    it in the vapour.  In the closed box rho_avg is the conserved mass over
    the node count, whatever its time level."""
    O = oracle_mod
    gx, gy = 3e-6, -1e-5
    (og, o0), rl, rv = _slab(O, gx, gy)
    rho = og.fields()["rho"]
    rbar = rho.mean()
    for o in (og, o0):
        o.step(1)
    jx_g, jy_g = _momentum(og)
    jx_0, jy_0 = _momentum(o0)
    ny = rho.shape[0]
    # liquid bulk (flat to 1e-7), and the middle of the vapour layer, whose
    # wide interfaces leave it uniform to about 1e-3 only
    for rows, sign, tol in ((slice(ny // 2 - 2, ny // 2 + 3), 1.0, 2e-6), (slice(0, 2), -1.0, 2e-3)):
        d = rho[rows] - rbar
        assert np.all(np.sign(d) == sign)
        assert np.allclose(jy_g[rows] - jy_0[rows], d * gy, rtol=tol, atol=0)
        assert np.allclose(jx_g[rows] - jx_0[rows], d * gx, rtol=tol, atol=0)
    # the force sums to zero over the closed box (Eq. 14 with the domain mean)
    assert abs((jy_g - jy_0).sum()) < 1e-12 * np.abs(jy_g - jy_0).max() * rho.size


def test_buoyancy_uses_previous_state_mean(oracle_mod):
    """rho_avg of Eq. 14 is the mean density of the whole domain at the
    previous time level (the explicit level of the step): checked on an open
    channel whose mass changes from step to step, against the mean of the
    previous state's density read out before the step; at the first step
    that is the mean initial density.  The same-state mean and the mean two
    steps back both miss by far more than the tolerance."""
    O = oracle_mod
    Ts = 0.86 * O.crit_temperature()
    P = O.Params(nx=12, ny=6, bc_x=O.BCX_CHANNEL, bc_y=O.BCY_WALLS, single_phase=1, isothermal=1, T_iso=Ts,
                 T_in=Ts, u_in=0.05, ga_x=2e-3, ga_y=-1e-3)
    o = O.Oracle(P)
    o.set_wall(0, Ts, 1.0)
    o.set_wall(1, Ts, 1.0)
    rng = np.random.default_rng(3)
    rho0 = 1.0 + 0.01 * rng.uniform(-1, 1, (P.ny, P.nx))
    o.init(rho0=rho0, T_u=Ts)
    means = [rho0.mean()]
    for n in range(6):
        F = o.fields(extra=True)
        rho = F["rho"]
        for comp, ga in (("Fx", P.ga_x), ("Fy", P.ga_y)):
            expect = (rho - means[-1]) * ga
            tol = 1e-13 * np.abs(expect).max()
            assert np.abs(F[comp] - expect).max() <= tol
            assert np.abs(F[comp] - (rho - rho.mean()) * ga).max() > 1e3 * tol
            if len(means) > 1:
                assert np.abs(F[comp] - (rho - means[-2]) * ga).max() > 1e3 * tol
        means.append(rho.mean())
        o.step(1)
