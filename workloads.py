"""Seeded synthetic inputs shared by the oracle side and the GPU side.

Only sizes, boundary maps, parameter values and seeds live here -- none of
the method's arithmetic.  The numeric constants are inputs:
  * TC: critical temperature of the Peng-Robinson constants a = 2/49,
    b = 2/21, R = 1 (pinned against the oracle's EOS in the CPU tests);
  * RHO_L, RHO_V: Maxwell coexistence densities at 0.86 Tc, omega = 0.344
    (pinned against the oracle's Maxwell construction); RHO_L_POOL,
    RHO_V_POOL the same at 0.9 Tc with omega = 0.32 (R134a), the state of
    the pool-boiling validation;
  * RHO_W_60: false wall density giving a ~60 degree contact angle at
    0.86 Tc (from the oracle's sessile-drop sweep, tests/golden/contact_angle_0p86Tc.json);
    wall_density_for_angle() reads that stored table backwards for any angle
    of its partial-wetting range.
The workloads follow the flow-boiling channel of Sec. 2C of the paper with
the sizes of the benchmark configurations (no dataset is involved).
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

CA_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "contact_angle_0p86Tc.json")

TC = 0.07292200407413424
TSAT_FRAC = 0.86
RHO_L = 6.4989457632878835
RHO_V = 0.3796789993997205
RHO_W_60 = 3.8
RHO_L_POOL = 5.881229445687165
RHO_V_POOL = 0.5901822861200811


@dataclass
class Channel:
    """Flow-boiling channel: walls S/N, velocity inlet W, convective outlet E,
    bottom heater centred in x, the same wettability on both walls."""
    nx: int = 200
    ny: int = 50
    u_in: float = 0.005
    superheat: float = 0.10     # heater at (1 + superheat) T_sat
    heater_len: int = 20
    rho_w: float = RHO_W_60
    seed: int = 1
    noise: float = 1e-3
    theta: float | None = None  # contact angle the wall density was chosen for (degrees)
    steps: int = 2000
    extra: dict = field(default_factory=dict)

    @property
    def T_sat(self):
        return TSAT_FRAC * TC

    @property
    def T_in(self):
        return 0.95 * self.T_sat

    @property
    def T_heater(self):
        return (1.0 + self.superheat) * self.T_sat

    def params(self) -> dict:
        """Parameter values common to both implementations."""
        p = dict(nx=self.nx, ny=self.ny, u_in=self.u_in, T_in=self.T_in, T_iso=self.T_sat,
                 rho_mid=0.5 * (RHO_L + RHO_V), ga_x=0.0, ga_y=-5e-5, tau_f=1.0, tau_g=0.6,
                 c_v=6.0, omega=0.344, bc_x=1, bc_y=1)
        p.update(self.extra)
        return p

    def heater(self) -> np.ndarray:
        h = np.zeros(self.nx, np.int32)
        c = self.nx // 2
        h[c - self.heater_len // 2: c - self.heater_len // 2 + self.heater_len] = 1
        return h

    def walls(self):
        """(T_south, rho_w_south, heater, T_north, rho_w_north), each [nx]."""
        h = self.heater()
        Ts = np.where(h == 1, self.T_heater, self.T_in)
        return Ts, np.full(self.nx, self.rho_w), h, np.full(self.nx, self.T_in), np.full(self.nx, self.rho_w)

    def init_args(self) -> dict:
        return dict(rho_u=RHO_L, T_u=self.T_sat, noise=self.noise, seed=self.seed)


def wall_density_for_angle(theta_deg: float) -> float:
    """False wall density whose sessile-drop contact angle at 0.86 Tc is
    theta_deg: piecewise-linear inverse of the stored calibration table over
    its partial-wetting rows (0 < theta < 180)."""
    tab = json.load(open(CA_TABLE))["table"]
    rows = [(t["theta_deg"], t["rho_w"]) for t in tab if t["theta_deg"] is not None and 0 < t["theta_deg"] < 180]
    th = np.array([r[0] for r in rows])[::-1]  # increasing angle
    rw = np.array([r[1] for r in rows])[::-1]
    if not th[0] <= theta_deg <= th[-1]:
        raise ValueError(f"contact angle {theta_deg} outside the calibrated range [{th[0]:.1f}, {th[-1]:.1f}]")
    return float(np.interp(theta_deg, th, rw))


def c1() -> Channel:
    """200x50 channel, 20-cell heater at 0.1 T_sat superheat, u_in = 0.005."""
    return Channel()


def c2(superheat: float = 0.10, u_in: float = 0.005) -> Channel:
    """1600x200 channel, 80-cell heater."""
    return Channel(nx=1600, ny=200, heater_len=80, superheat=superheat, u_in=u_in, steps=100000)


C2_SWEEP = [(s, u) for s in (0.05, 0.10, 0.15) for u in (0.002, 0.005, 0.01)]


def ensemble(n: int = 64, seed: int = 4, steps: int = 20000) -> list[Channel]:
    """Uneven channels: Lx in {400, 800, 1200, 1600}, Ly in {50, 100, 200},
    u_in ~ U[0.002, 0.01], superheat ~ U[0.05, 0.2], contact angle
    ~ U[30, 120] degrees turned into a wall density through the calibration
    table; heater 0.4 Ly cells, centred."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nx = int(rng.choice([400, 800, 1200, 1600]))
        ny = int(rng.choice([50, 100, 200]))
        c = Channel(nx=nx, ny=ny, u_in=float(rng.uniform(0.002, 0.01)),
                    superheat=float(rng.uniform(0.05, 0.2)), heater_len=int(0.4 * ny), seed=1000 + i,
                    steps=steps)
        c.theta = float(rng.uniform(30.0, 120.0))
        # below the smallest partial-wetting angle of the table (31.7
        # degrees; a film forms beyond it) the wall density of that angle
        c.rho_w = wall_density_for_angle(max(c.theta, MIN_PARTIAL_ANGLE))
        out.append(c)
    return out


def _partial_wetting_range():
    tab = json.load(open(CA_TABLE))["table"]
    th = [t["theta_deg"] for t in tab if t["theta_deg"] is not None and 0 < t["theta_deg"] < 180]
    return min(th), max(th)


MIN_PARTIAL_ANGLE, MAX_PARTIAL_ANGLE = _partial_wetting_range()


@dataclass
class Pool:
    """Pool-boiling box (Sec. 2D): saturated R134a at 0.9 Tc (omega 0.32),
    periodic sides, the bottom wall at T_sat with a heater of heater_len
    cells at its centre, a liquid pool of depth `depth` under a vapour layer
    (the free surface) capped by a non-wetting wall (false density rho_v),
    buoyancy g_a downwards.  The box is 4 times wider than tall."""
    nx: int = 512
    ny: int = 128
    depth: int = 112
    ga: float = 5e-5
    T_heater_over_Tc: float = 1.2
    heater_len: int = 11
    rho_w: float = 3.5          # false wall density of the bottom wall
    rho_w_heater: float = 1.2   # and of the heater cells
    tau_g: float = 0.6
    c_v: float = 6.0

    @property
    def T_sat(self):
        return 0.9 * TC

    def params(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, bc_x=0, bc_y=1, u_in=0.0, T_in=self.T_sat, T_iso=self.T_sat,
                    rho_mid=0.5 * (RHO_L_POOL + RHO_V_POOL), ga_x=0.0, ga_y=-self.ga, tau_f=1.0,
                    tau_g=self.tau_g, c_v=self.c_v, omega=0.32)

    def heater(self) -> np.ndarray:
        h = np.zeros(self.nx, np.int32)
        c = self.nx // 2 - self.heater_len // 2
        h[c: c + self.heater_len] = 1
        return h

    def walls(self):
        """(T_south, rho_w_south, heater, T_north, rho_w_north), each [nx]."""
        h = self.heater()
        Ts = np.where(h == 1, self.T_heater_over_Tc * TC, self.T_sat)
        rws = np.where(h == 1, self.rho_w_heater, self.rho_w)
        return Ts, rws, h, np.full(self.nx, self.T_sat), np.full(self.nx, RHO_V_POOL)

    def init_args(self) -> dict:
        y = np.arange(self.ny)[:, None] * np.ones((1, self.nx))
        rho0 = RHO_V_POOL + (RHO_L_POOL - RHO_V_POOL) * 0.5 * (1 - np.tanh((y - self.depth) / 2.0))
        return dict(rho0=rho0, T_u=self.T_sat)


def roofline_channel() -> Channel:
    """Synthetic 8192x1024 channel: FP32 A/B state of 1.2 GB, several times
    the 256 MB Infinity Cache, so the step streams from HBM."""
    return Channel(nx=8192, ny=1024, heater_len=410, steps=200)
