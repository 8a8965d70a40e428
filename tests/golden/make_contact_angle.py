"""Writes contact_angle_0p86Tc.json: the static contact angle of a sessile
drop on the bottom wall against the false wall density rho_w of the adhesion
force (Eq. 15), at 0.86 Tc, computed with the FP64 oracle only.

Protocol: 120x60 box, periodic in x, walls S/N (north wall at rho_v, i.e.
non-wetting), isothermal at 0.86 Tc, g_a = 0; a half-disc of saturated
liquid of radius 22 on the bottom wall, relaxed for 12000 steps.  The angle
is read from the drop height h (rho_mid crossing on the centre column) and
base width w (rho_mid crossings along the wall row): tan(theta/2) = 2h/w.
The wall density used by the flow-boiling channels for a ~60 degree angle
is read off this table.

    OMP_NUM_THREADS=8 python3 tests/golden/make_contact_angle.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "contact_angle_0p86Tc.json")
RHO_W = (2.5, 3.0, 3.4, 3.8, 4.2, 4.6, 5.2, 6.0)


def contact_angle(rw: float, nx=120, ny=60, R=22, steps=12000) -> dict:
    from oracle import oracle as O

    T = 0.86 * O.crit_temperature()
    rl, rv, _ = O.maxwell(T)
    P = O.Params(nx=nx, ny=ny, bc_x=O.BCX_PERIODIC, bc_y=O.BCY_WALLS, isothermal=1, T_iso=T, T_in=T,
                 ga_y=0.0, u_in=0.0, rho_mid=0.5 * (rl + rv))
    o = O.Oracle(P)
    o.set_wall(0, np.full(nx, T), np.full(nx, rw))
    o.set_wall(1, np.full(nx, T), np.full(nx, rv))
    y, x = np.mgrid[0:ny, 0:nx]
    r = np.sqrt((x - nx / 2 + 0.5) ** 2 + (y + 0.5) ** 2)
    o.init(rho0=rv + (rl - rv) * 0.5 * (1 - np.tanh((r - R) / 2.0)), T_u=T)
    o.step(steps)
    rho = o.fields()["rho"]
    mid = 0.5 * (rl + rv)
    col = rho[:, nx // 2]
    h = None
    for j in range(ny - 1):
        if col[j] >= mid > col[j + 1]:
            h = j + (col[j] - mid) / (col[j] - col[j + 1]) + 0.5
            break
    row = rho[0]
    liq = np.where(row >= mid)[0]
    if h is None or len(liq) == 0:
        return {"rho_w": rw, "theta_deg": None, "h": h, "w": 0.0}
    if len(liq) == nx:
        return {"rho_w": rw, "theta_deg": 0.0, "h": h, "w": float(nx)}
    i0, i1 = liq.min(), liq.max()
    a = i0 - (row[i0] - mid) / (row[i0] - row[i0 - 1])
    b = i1 + (row[i1] - mid) / (row[i1] - row[i1 + 1])
    w = b - a
    return {"rho_w": rw, "theta_deg": float(2 * np.degrees(np.arctan(2 * h / w))), "h": float(h), "w": float(w)}


def main():
    rows = []
    for rw in RHO_W:
        rows.append(contact_angle(rw))
        print(rows[-1], flush=True)
    doc = {"_comment": "Static contact angle vs false wall density (Eq. 15 adhesion), sessile drop, oracle only; "
                       "written by tests/golden/make_contact_angle.py",
           "T_over_Tc": 0.86, "omega": 0.344, "box": [120, 60], "drop_radius": 22, "steps": 12000,
           "table": rows}
    json.dump(doc, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main()
