"""The oracle against a second, independent implementation of the step
(tests/tiny_step.py: per-node Python loops from the equations of Sec. 2A-2C)
on 7x5 lattices, 5 steps, every boundary kind: stored distributions, outlet
memory, fields, forces, source and diagnostics agree to 1e-12.  This pins
the parts with no closed form: corner rules, inlet temperature, both
outlets, the wall closure of div u, the heater and pressure read-outs."""
import numpy as np
import pytest

from tiny_step import TinyLBM

CASES = {
    "periodic": dict(bc_x=0, bc_y=0),
    "walls": dict(bc_x=0, bc_y=1),
    "channel_convective": dict(bc_x=1, bc_y=1),
    "channel_pressure": dict(bc_x=2, bc_y=1),
    "channel_periodic_y": dict(bc_x=1, bc_y=0),
    "channel_isothermal": dict(bc_x=1, bc_y=1, isothermal=1),
    "channel_single_phase": dict(bc_x=1, bc_y=1, single_phase=1),
    "walls_G_wet": dict(bc_x=0, bc_y=1, G_wet=-25.0),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_matches_independent_step(oracle_mod, name):
    O = oracle_mod
    nx, ny, steps = 7, 5, 5
    rng = np.random.default_rng(abs(hash(name)) % 2**32)
    Tc = O.crit_temperature()
    Ts = 0.86 * Tc
    rl, rv, _ = O.maxwell(Ts)
    P = O.Params(nx=nx, ny=ny, T_in=0.95 * Ts, T_iso=Ts, u_in=0.03, rho_mid=0.5 * (rl + rv), rho_out=rl,
                 ga_x=2e-4, ga_y=-3e-4, fb_x=1e-5, fb_y=-2e-5, tau_f=0.8, tau_g=0.7, c_v=5.0,
                 s_e=1.1, s_eps=1.3, s_q=1.4, **CASES[name])
    # a two-phase random start: liquid with a vapour pocket, noisy temperature
    rho0 = rl * (1 + 0.02 * rng.uniform(-1, 1, (ny, nx)))
    rho0[1:3, 2:4] = rv * (1 + 0.05 * rng.uniform(-1, 1, (2, 2)))
    T0 = Ts * (1 + 0.05 * rng.uniform(-1, 1, (ny, nx)))
    Tw_s = Ts * (1 + 0.1 * rng.uniform(0, 1, nx))
    Tw_n = Ts * (1 + 0.1 * rng.uniform(-1, 0, nx))
    rw_s = rng.uniform(1.0, 6.0, nx)
    rw_n = rng.uniform(1.0, 6.0, nx)
    heater = (rng.uniform(0, 1, nx) < 0.5).astype(np.int32)
    o = O.Oracle(P)
    o.set_wall(0, Tw_s, rw_s, heater)
    o.set_wall(1, Tw_n, rw_n)
    o.init(rho0=rho0, T0=T0)
    t = TinyLBM(P, Tw_s, rw_s, Tw_n, rw_n, heater, rho0, T0)
    for _ in range(steps):
        o.step(1)
        t.step()
    fs, gs = o.state()
    assert np.allclose(fs, t.fs, rtol=0, atol=1e-12 * np.abs(t.fs).max())
    if not P.isothermal:
        assert np.allclose(gs, t.gs, rtol=0, atol=1e-12 * np.abs(t.gs).max())
    assert o.rbar() == pytest.approx(t.rbar, rel=1e-13)
    F = o.fields(extra=True)
    s = t.evaluate()
    for k, kt in (("rho", "rho"), ("ux", "uax"), ("uy", "uay"), ("T", "T"), ("p", "p"), ("psi", "psi"),
                  ("Fx", "Fx"), ("Fy", "Fy"), ("phi", "phi")):
        scale = max(np.abs(s[kt]).max(), 1e-30)
        assert np.abs(F[k] - s[kt]).max() <= 1e-12 * scale, k
    d, dt = o.diag(), t.diag()
    for k in dt:
        assert d[k] == pytest.approx(dt[k], rel=1e-12, abs=1e-14), k
    # the run moved: forces, source and the ends are exercised
    assert np.abs(s["Fx"]).max() > 1e-4 and np.abs(s["phi"]).max() > 1e-8 or P.isothermal
