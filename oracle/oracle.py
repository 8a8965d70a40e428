"""Python side of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this module; the product package never imports it, and
it imports nothing from the product package.

* ``build()`` compiles ``lbm_oracle.c`` (plain C, gcc, OpenMP over rows).
* ``Oracle`` wraps one simulation state of that library through ctypes.
* ``maxwell()`` is the equal-area (Maxwell) construction for the
  Peng-Robinson EOS of Eq. 12, written independently in numpy/scipy.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field, fields

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# D2Q9 ordering used throughout (rest, +x, +y, -x, -y, ++, -+, --, +-).
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def build(force: bool = True) -> str:
    """Compile the oracle shared library next to its source."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.oc_create.restype = C.c_void_p
        L.oc_create.argtypes = [C.c_void_p]
        L.oc_destroy.argtypes = [C.c_void_p]
        L.oc_set_wall.argtypes = [C.c_void_p, C.c_int, dp, dp, C.POINTER(C.c_int)]
        L.oc_splitmix64.restype = C.c_uint64
        L.oc_splitmix64.argtypes = [C.c_uint64]
        L.oc_noise.restype = C.c_double
        L.oc_noise.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_int]
        L.oc_init.argtypes = [C.c_void_p, dp, dp, C.c_double, C.c_double, C.c_double, C.c_uint64]
        L.oc_step.argtypes = [C.c_void_p, C.c_int64]
        L.oc_step_count.restype = C.c_int64
        L.oc_step_count.argtypes = [C.c_void_p]
        L.oc_fields.argtypes = [C.c_void_p] + [dp] * 9
        L.oc_diag.argtypes = [C.c_void_p, dp]
        L.oc_get_state.argtypes = [C.c_void_p, dp, dp]
        L.oc_set_state.argtypes = [C.c_void_p, dp, dp]
        L.oc_get_streamed.argtypes = [C.c_void_p, dp, dp]
        L.oc_get_rbar.restype = C.c_double
        L.oc_get_rbar.argtypes = [C.c_void_p]
        L.oc_set_rbar.argtypes = [C.c_void_p, C.c_double]
        L.oc_eos.restype = C.c_int
        L.oc_eos.argtypes = [C.c_void_p, C.c_double, C.c_double, dp]
        L.oc_Tc.restype = C.c_double
        L.oc_Tc.argtypes = [C.c_void_p]
        L.oc_feq.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.oc_collide_f_node.argtypes = [C.c_void_p, dp, C.c_double, C.c_double, dp]
        L.oc_collide_g_node.argtypes = [C.c_void_p, dp, C.c_double, C.c_double, C.c_double, dp]
        L.oc_mrt_matrix.argtypes = [dp]
        L.oc_set_threads.argtypes = [C.c_int]
        L.oc_max_threads.restype = C.c_int
        _lib = L
    return _lib


class _CParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "a", "b", "R", "omega", "beta", "c0", "g", "s_nu", "s_e", "s_eps", "s_q",
        "tau_g", "c_v", "ga_x", "ga_y", "fb_x", "fb_y", "u_in", "T_in", "U_out",
        "T_iso", "rho_mid", "rho_out", "G_wet")] + [(n, C.c_int32) for n in (
        "nx", "ny", "bc_x", "bc_y", "isothermal", "single_phase")]


BCX_PERIODIC, BCX_CHANNEL, BCX_CHANNEL_P = 0, 1, 2
BCY_PERIODIC, BCY_WALLS = 0, 1


def crit_temperature(a=2 / 49, b=2 / 21, R=1.0) -> float:
    """T_c from a = 0.45724 R^2 Tc^2/pc and b = 0.0778 R Tc/pc (Eq. 12)."""
    return 0.0778 * a / (0.45724 * b * R)


@dataclass
class Params:
    """Model parameters (lattice units).  Defaults: the flow-boiling channel
    with the design readings (tau_f = 1, tau_g = 0.6, c_v = 6, MRT rates with
    s_q fixing Lambda = 3/16, g_a = (0, -5e-5))."""
    nx: int = 200
    ny: int = 50
    a: float = 2 / 49
    b: float = 2 / 21
    R: float = 1.0
    omega: float = 0.344
    beta: float = 1.16
    c0: float = 6.0
    g: float = -1.0
    tau_f: float = 1.0
    s_e: float | None = None
    s_eps: float | None = None
    s_q: float | None = None
    tau_g: float = 0.6
    c_v: float = 6.0
    ga_x: float = 0.0
    ga_y: float = -5e-5
    fb_x: float = 0.0
    fb_y: float = 0.0
    u_in: float = 0.005
    T_in: float = 0.0
    U_out: float | None = None
    T_iso: float = 0.0
    rho_mid: float = 0.0
    rho_out: float = 0.0     # outlet density of BCX_CHANNEL_P
    G_wet: float | None = None  # adhesion strength of Eq. 15 (None: neutral_G_wet)
    bc_x: int = BCX_CHANNEL
    bc_y: int = BCY_WALLS
    isothermal: int = 0
    single_phase: int = 0

    def rates(self):
        s_nu = 1.0 / self.tau_f
        s_e = s_nu if self.s_e is None else self.s_e
        s_eps = s_nu if self.s_eps is None else self.s_eps
        s_q = 8.0 * (2.0 - s_nu) / (8.0 - s_nu) if self.s_q is None else self.s_q
        return s_nu, s_e, s_eps, s_q

    def to_c(self) -> _CParams:
        s_nu, s_e, s_eps, s_q = self.rates()
        c = _CParams()
        for f in _CParams._fields_:
            n = f[0]
            if n == "s_nu":
                c.s_nu = s_nu
            elif n == "s_e":
                c.s_e = s_e
            elif n == "s_eps":
                c.s_eps = s_eps
            elif n == "s_q":
                c.s_q = s_q
            elif n == "U_out":
                c.U_out = self.u_in if self.U_out is None else self.U_out
            elif n == "G_wet":
                c.G_wet = self.neutral_G_wet if self.G_wet is None else self.G_wet
            else:
                setattr(c, n, getattr(self, n))
        return c

    @property
    def Tc(self) -> float:
        return crit_temperature(self.a, self.b, self.R)

    @property
    def neutral_G_wet(self) -> float:
        """The G_wet of Eq. 15 (not printed in the paper) at which a wall whose
        false density equals the adjacent fluid density exerts no net force.
        Eq. 10 with g1 = 2g, g2 = g/2 is G_i = 18 g w_i on D2Q9, and a flat
        wall removes the solid neighbours from both sums of Eq. 9, whose
        missing pull is (1 + beta)/2 sum_solid G_i psi^2 c_i; Eq. 15 returns
        it when G_wet w_i = (1 + beta)/2 G_i, i.e. G_wet = 9 g (1 + beta)."""
        return 9.0 * self.g * (1.0 + self.beta)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def eos(P: Params, rho: float, T: float):
    """(p, psi, dp/dT, clamped) at one state point, from the oracle library."""
    out = np.zeros(3)
    c = P.to_c()
    clamped = lib().oc_eos(C.byref(c), float(rho), float(T), _dp(out))
    return out[0], out[1], out[2], bool(clamped)


def splitmix64(z: int) -> int:
    return int(lib().oc_splitmix64(C.c_uint64(z & 0xFFFFFFFFFFFFFFFF)))


class Oracle:
    """One FP64 simulation state.  Arrays are [ny, nx] row-major."""

    def __init__(self, P: Params):
        self.P = P
        self._c = P.to_c()
        self.h = lib().oc_create(C.byref(self._c))
        if not self.h:
            raise ValueError("invalid oracle parameters")
        self.nx, self.ny = P.nx, P.ny

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().oc_destroy(h)
            self.h = None

    def set_wall(self, side: int, T_wall, rho_w, heater=None):
        Tw = np.ascontiguousarray(np.broadcast_to(np.asarray(T_wall, float), (self.nx,)))
        rw = np.ascontiguousarray(np.broadcast_to(np.asarray(rho_w, float), (self.nx,)))
        hp = None
        if heater is not None:
            ha = np.ascontiguousarray(np.asarray(heater, dtype=np.int32))
            hp = ha.ctypes.data_as(C.POINTER(C.c_int))
        lib().oc_set_wall(self.h, int(side), _dp(Tw), _dp(rw), hp)

    def init(self, rho0=None, T0=None, rho_u=1.0, T_u=None, noise=0.0, seed=0):
        T_u = self.P.T_in if T_u is None else T_u
        r = None if rho0 is None else np.ascontiguousarray(np.broadcast_to(np.asarray(rho0, float), (self.ny, self.nx)))
        t = None if T0 is None else np.ascontiguousarray(np.broadcast_to(np.asarray(T0, float), (self.ny, self.nx)))
        lib().oc_init(self.h, None if r is None else _dp(r), None if t is None else _dp(t),
                      float(rho_u), float(T_u), float(noise), C.c_uint64(seed))

    def step(self, n: int = 1):
        lib().oc_step(self.h, int(n))

    @property
    def steps(self) -> int:
        return int(lib().oc_step_count(self.h))

    def fields(self, extra: bool = False) -> dict:
        shp = (self.ny, self.nx)
        names = ["rho", "ux", "uy", "T", "p", "psi", "Fx", "Fy", "phi"]
        arrs = {n: np.zeros(shp) for n in names}
        lib().oc_fields(self.h, *[_dp(arrs[n]) for n in names])
        if not extra:
            return {k: arrs[k] for k in ("rho", "ux", "uy", "T")}
        return arrs

    DIAG_NAMES = ("mass", "energy", "heater_q", "vapor_cells", "psi_clamped", "nonfinite", "p_in", "p_out")

    def diag(self) -> dict:
        out = np.zeros(len(self.DIAG_NAMES))
        lib().oc_diag(self.h, _dp(out))
        return dict(zip(self.DIAG_NAMES, out.tolist()))

    def state(self):
        fs = np.zeros((9, self.ny, self.nx))
        gs = np.zeros((9, self.ny, self.nx))
        lib().oc_get_state(self.h, _dp(fs), _dp(gs))
        return fs, gs

    def set_state(self, fs, gs):
        fs = np.ascontiguousarray(fs, dtype=float)
        gs = np.ascontiguousarray(gs, dtype=float)
        lib().oc_set_state(self.h, _dp(fs), _dp(gs))

    def streamed(self):
        f = np.zeros((9, self.ny, self.nx))
        g = np.zeros((9, self.ny, self.nx))
        lib().oc_get_streamed(self.h, _dp(f), _dp(g))
        return f, g

    def rbar(self) -> float:
        """Mean density the force of the next evaluation uses (Eq. 14): that
        of the previous state."""
        return float(lib().oc_get_rbar(self.h))

    def set_rbar(self, v: float):
        lib().oc_set_rbar(self.h, float(v))


def collide_f_node(P: Params, f, Fx, Fy):
    f = np.ascontiguousarray(f, float)
    out = np.zeros(9)
    c = P.to_c()
    lib().oc_collide_f_node(C.byref(c), _dp(f), float(Fx), float(Fy), _dp(out))
    return out


def collide_g_node(P: Params, g, uax, uay, phi):
    g = np.ascontiguousarray(g, float)
    out = np.zeros(9)
    c = P.to_c()
    lib().oc_collide_g_node(C.byref(c), _dp(g), float(uax), float(uay), float(phi), _dp(out))
    return out


def feq(rho, ux, uy):
    out = np.zeros(9)
    lib().oc_feq(float(rho), float(ux), float(uy), _dp(out))
    return out


def mrt_matrix():
    out = np.zeros(81)
    lib().oc_mrt_matrix(_dp(out))
    return out.reshape(9, 9)


# ---------------------------------------------------------------------------
# Maxwell equal-area construction for the Peng-Robinson EOS (Eq. 12), written
# in molar volume v = 1/rho:  p(v) = RT/(v-b) - a alpha/(v^2 + 2bv - b^2).

def _alpha(T, Tc, omega):
    kappa = 0.37464 + 1.54226 * omega - 0.26992 * omega ** 2
    return (1.0 + kappa * (1.0 - math.sqrt(T / Tc))) ** 2


def pr_pressure_v(v, T, a=2 / 49, b=2 / 21, R=1.0, omega=0.344):
    Tc = crit_temperature(a, b, R)
    al = _alpha(T, Tc, omega)
    return R * T / (v - b) - a * al / (v * v + 2 * b * v - b * b)


def pr_antiderivative_v(v, T, a=2 / 49, b=2 / 21, R=1.0, omega=0.344):
    """A primitive of p(v) dv:  RT ln(v-b) - a alpha/(2 sqrt2 b) ln((v+b-sqrt2 b)/(v+b+sqrt2 b))."""
    Tc = crit_temperature(a, b, R)
    al = _alpha(T, Tc, omega)
    r2 = math.sqrt(2.0)
    return R * T * math.log(v - b) - a * al / (2 * r2 * b) * math.log((v + b - r2 * b) / (v + b + r2 * b))


def maxwell(T, a=2 / 49, b=2 / 21, R=1.0, omega=0.344):
    """Coexisting (rho_l, rho_v, p_sat) at T < Tc by the equal-area rule."""
    from scipy.optimize import brentq

    Tc = crit_temperature(a, b, R)
    if not (0 < T < Tc):
        raise ValueError("T must lie below the critical temperature")
    p = lambda v: pr_pressure_v(v, T, a, b, R, omega)
    dp = lambda v: (p(v * (1 + 1e-7)) - p(v * (1 - 1e-7))) / (2e-7 * v)
    # Spinodals: extrema of p(v) on either side of the critical volume.
    vs = np.geomspace(b * 1.0001, 1e4 * b, 200001)
    ps = np.array([p(v) for v in vs[::50]])
    vv = vs[::50]
    d = np.diff(ps)
    idx = np.where(np.sign(d[1:]) != np.sign(d[:-1]))[0]
    if len(idx) < 2:
        raise ValueError("no van der Waals loop at this temperature")
    v_min = brentq(dp, vv[idx[0]], vv[idx[0] + 2])   # local minimum of p (liquid spinodal)
    v_max = brentq(dp, vv[idx[1]], vv[idx[1] + 2])   # local maximum of p (vapour spinodal)
    p_lo, p_hi = max(p(v_min), 1e-9 * p(v_max)), p(v_max)

    def roots(ps_):
        vl = brentq(lambda v: p(v) - ps_, b * (1 + 1e-12), v_min, xtol=1e-16)
        vhi = 2.0 * v_max
        while p(vhi) >= ps_:
            vhi *= 2.0
        vg = brentq(lambda v: p(v) - ps_, v_max, vhi, xtol=1e-15 * vhi)
        return vl, vg

    def area(ps_):
        vl, vg = roots(ps_)
        return (pr_antiderivative_v(vg, T, a, b, R, omega) - pr_antiderivative_v(vl, T, a, b, R, omega)) - ps_ * (vg - vl)

    eps = 1e-12 * (p_hi - p_lo)
    psat = brentq(area, p_lo + eps, p_hi - eps, xtol=1e-16, rtol=1e-15, maxiter=500)
    vl, vg = roots(psat)
    return 1.0 / vl, 1.0 / vg, psat


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's per-node loops; returns the count now in use."""
    lib().oc_set_threads(int(n))
    return int(lib().oc_max_threads())
