"""Pins of the oracle's local operators: the equilibrium (Eq. 3), the MRT
collision with exact-difference forcing (Eqs. 2, 5) and the thermal
collision with its source (Eqs. 16-18)."""
import numpy as np
import pytest

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def _random_state(rng):
    rho = rng.uniform(0.3, 7.0)
    u = rng.uniform(-0.05, 0.05, 2)
    f = np.array([0.0] * 9)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    cu = CX * u[0] + CY * u[1]
    f = w * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u @ u))
    f *= 1 + rng.uniform(-0.05, 0.05, 9)  # off equilibrium
    return f


def test_equilibrium_moments(oracle_mod):
    """Eq. 3 reproduces rho, rho u and the Euler momentum flux rho(uu + I/3)."""
    O = oracle_mod
    rng = np.random.default_rng(0)
    for _ in range(20):
        rho = rng.uniform(0.1, 8)
        ux, uy = rng.uniform(-0.1, 0.1, 2)
        e = O.feq(rho, ux, uy)
        assert e.sum() == pytest.approx(rho, rel=1e-14)
        assert (e * CX).sum() == pytest.approx(rho * ux, abs=1e-14 * rho)
        assert (e * CY).sum() == pytest.approx(rho * uy, abs=1e-14 * rho)
        assert (e * CX * CX).sum() == pytest.approx(rho * (ux * ux + 1 / 3), rel=1e-13)
        assert (e * CX * CY).sum() == pytest.approx(rho * ux * uy, abs=1e-13 * rho)


def test_mrt_basis_orthogonal(oracle_mod):
    M = oracle_mod.mrt_matrix()
    G = M @ M.T
    assert np.allclose(G, np.diag(np.diag(G)), atol=0)
    assert np.allclose(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])
    # rows 0, 3, 5 are the conserved moments rho, jx, jy
    assert np.array_equal(M[3], CX) and np.array_equal(M[5], CY)


def test_collision_invariants(oracle_mod):
    """Sum f* = rho, sum f* c = rho u + F (EDM adds F dt to the momentum),
    sum g* = T + phi, for any pre-collision state (P4)."""
    O = oracle_mod
    P = O.Params(tau_f=0.8, s_e=1.3, s_eps=0.9, s_q=1.1)
    rng = np.random.default_rng(1)
    for _ in range(50):
        f = _random_state(rng)
        F = rng.uniform(-1e-2, 1e-2, 2)
        out = O.collide_f_node(P, f, F[0], F[1])
        rho = f.sum()
        assert out.sum() == pytest.approx(rho, rel=1e-14)
        assert (out * CX).sum() == pytest.approx((f * CX).sum() + F[0], abs=1e-14 * rho)
        assert (out * CY).sum() == pytest.approx((f * CY).sum() + F[1], abs=1e-14 * rho)
        g = _random_state(rng) * 0.01
        phi = rng.uniform(-1e-4, 1e-4)
        ua = rng.uniform(-0.05, 0.05, 2)
        go = O.collide_g_node(P, g, ua[0], ua[1], phi)
        assert go.sum() == pytest.approx(g.sum() + phi, rel=1e-13)


def test_mrt_reduces_to_bgk(oracle_mod):
    """With every rate equal to 1/tau the MRT operator is the BGK operator of
    Eq. 2:  f* = f - (f - f^eq)/tau + [f^eq(u + du) - f^eq(u)]  (P5)."""
    O = oracle_mod
    rng = np.random.default_rng(2)
    for tau in (0.55, 0.8, 1.0, 1.7):
        s = 1.0 / tau
        P = O.Params(tau_f=tau, s_e=s, s_eps=s, s_q=s)
        for _ in range(10):
            f = _random_state(rng)
            F = rng.uniform(-1e-2, 1e-2, 2)
            rho = f.sum()
            ux, uy = (f * CX).sum() / rho, (f * CY).sum() / rho
            e0 = O.feq(rho, ux, uy)
            e1 = O.feq(rho, ux + F[0] / rho, uy + F[1] / rho)
            bgk = f - (f - e0) / tau + (e1 - e0)
            assert np.allclose(O.collide_f_node(P, f, F[0], F[1]), bgk, rtol=0, atol=1e-14 * rho)


def test_thermal_collision_relaxes_to_equilibrium(oracle_mod):
    """tau_g = 1 and phi = 0: g* is g^eq(T, u_act) of Eq. 18 exactly."""
    O = oracle_mod
    P = O.Params(tau_g=1.0)
    rng = np.random.default_rng(3)
    g = _random_state(rng) * 0.01
    ua = (0.02, -0.01)
    assert np.allclose(O.collide_g_node(P, g, ua[0], ua[1], 0.0), O.feq(g.sum(), *ua), atol=1e-16)
