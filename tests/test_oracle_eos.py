"""Pins of the oracle's thermodynamics: Peng-Robinson EOS (Eq. 12), its
temperature derivative (Eq. 19), the critical point implied by the constants
a, b (Sec. 2A), and the Maxwell construction against the densities the paper
prints (Sec. 3E)."""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def test_critical_point_is_inflection(oracle_mod):
    """a = 0.45724 R^2Tc^2/pc, b = 0.0778 RTc/pc put the critical point of the
    PR EOS at Tc = 0.0778 a/(0.45724 b R) with dp/drho = d2p/drho2 = 0 and
    Z_c = pc/(rho_c R Tc) = 0.3074.  A wrong sign or a dropped term in the
    oracle's p(rho, T) breaks the double zero."""
    O = oracle_mod
    P = O.Params()
    Tc = P.Tc
    assert Tc == pytest.approx(0.0729220, abs=5e-8)
    p = lambda r: O.eos(P, r, Tc)[0]
    h = 1e-4
    d1 = lambda r: (p(r + h) - p(r - h)) / (2 * h)
    d2 = lambda r: (p(r + h) - 2 * p(r) + p(r - h)) / (h * h)
    from scipy.optimize import brentq
    rc = brentq(d2, 1.0, 5.0)
    pc = 0.0778 * P.R * Tc / P.b
    assert abs(d1(rc)) < 2e-3 * pc / rc
    assert p(rc) == pytest.approx(pc, rel=2e-3)
    assert pc / (rc * P.R * Tc) == pytest.approx(0.3074, rel=5e-3)
    # alpha(Tc) = 1 for any acentric factor: p at Tc does not depend on omega
    P2 = O.Params(omega=0.0)
    assert O.eos(P2, rc, Tc)[0] == pytest.approx(p(rc), rel=1e-14)


def test_dpdT_matches_finite_difference(oracle_mod):
    O = oracle_mod
    P = O.Params()
    Tc = P.Tc
    for rho in (0.3, 1.0, 2.657, 5.0, 6.5, 7.5):
        for tr in (0.7, 0.86, 0.95, 1.1):
            T = tr * Tc
            h = 1e-6 * T
            fd = (O.eos(P, rho, T + h)[0] - O.eos(P, rho, T - h)[0]) / (2 * h)
            an = O.eos(P, rho, T)[2]
            assert an == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_psi_defined_in_working_range(oracle_mod):
    """Eq. 11 needs p - rho/3 <= 0 (c0 g < 0); the oracle clamps and counts
    otherwise.  Up to 1.2 Tc that only happens far above liquid density."""
    O = oracle_mod
    P = O.Params()
    for tr in (0.6, 0.86, 1.0, 1.2):
        for rho in np.linspace(0.01, 8.0, 81):
            assert not O.eos(P, rho, tr * P.Tc)[3]
    assert O.eos(P, 9.5, 1.2 * P.Tc)[3]


def test_psi_identity_and_pressure(oracle_mod):
    """Eq. 11 inverted: c0 g psi^2 / 2 + c_s^2 rho = p for every state the
    oracle evaluates, and p itself equals the Peng-Robinson pressure of
    Eq. 12 written in molar volume by the separate numpy code of the Maxwell
    construction (pr_pressure_v), so a slip in either the EOS or the psi map
    (a constant, a sign, c0 against g) fails here."""
    O = oracle_mod
    for omega in (0.32, 0.344):
        P = O.Params(omega=omega)
        for tr in (0.6, 0.86, 0.9, 1.0, 1.2):
            T = tr * P.Tc
            for rho in (0.05, 0.38, 1.0, 2.657, 5.0, 6.5, 8.0):
                p, psi, _, clamped = O.eos(P, rho, T)
                assert not clamped
                assert P.c0 * P.g * psi ** 2 / 2 + rho / 3 == pytest.approx(p, rel=1e-13, abs=1e-16)
                assert p == pytest.approx(O.pr_pressure_v(1.0 / rho, T, omega=omega), rel=1e-12, abs=1e-16)


def _check_maxwell(O, T, omega):
    rl, rv, ps = O.maxwell(T, omega=omega)
    P = O.Params(omega=omega)
    # equal pressures, evaluated with the oracle library's own EOS
    assert O.eos(P, rl, T)[0] == pytest.approx(ps, rel=1e-9)
    assert O.eos(P, rv, T)[0] == pytest.approx(ps, rel=1e-9)
    # equal areas: int_{v_l}^{v_v} (p - p_s) dv = 0, by quadrature of the C EOS
    f = lambda v: O.eos(P, 1.0 / v, T)[0] - ps
    area, err = quad(f, 1.0 / rl, 1.0 / rv, limit=400, epsabs=1e-13)
    assert abs(area) < 1e-9 * ps * (1.0 / rv - 1.0 / rl)
    # stable branches: dp/drho > 0 at both coexisting densities
    h = 1e-6
    for r in (rl, rv):
        assert O.eos(P, r + h, T)[0] > O.eos(P, r - h, T)[0]
    return rl, rv, ps


def test_maxwell_against_printed_densities(oracle_mod):
    """Sec. 3E prints rho_l = 5.95, rho_v = 0.59 at 0.9 Tc for the PR EOS with
    the R134a acentric factor.  The Maxwell values with alpha read as
    [1 + kappa(1 - sqrt(T/Tc))]^2 land on both; reading sqrt(T/Tc^2)
    literally gives no coexistence at all at this temperature."""
    O = oracle_mod
    g = json.load(open(GOLDEN))["coexistence_0p9Tc_R134a"]
    Tc = O.crit_temperature(g["a"], g["b"], g["R"])
    rl, rv, _ = _check_maxwell(O, g["T_over_Tc"] * Tc, g["omega"])
    assert rv == pytest.approx(g["rho_v"], rel=5e-3)
    assert rl == pytest.approx(g["rho_l"], rel=1.5e-2)


@pytest.mark.parametrize("tr", [0.7, 0.8, 0.86, 0.9, 0.95])
def test_maxwell_construction(oracle_mod, tr):
    O = oracle_mod
    rl, rv, ps = _check_maxwell(O, tr * O.crit_temperature(), 0.344)
    assert rl > rv > 0


def test_maxwell_operating_point(oracle_mod):
    """The channel's saturation state (T_sat = 0.86 Tc, omega = 0.344)."""
    O = oracle_mod
    rl, rv, ps = O.maxwell(0.86 * O.crit_temperature(), omega=0.344)
    assert rl == pytest.approx(6.4989, abs=2e-4)
    assert rv == pytest.approx(0.3797, abs=2e-4)
    assert ps == pytest.approx(0.018491, abs=2e-6)
