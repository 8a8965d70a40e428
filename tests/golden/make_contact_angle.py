"""Writes contact_angle_0p86Tc.json: the static contact angle of a sessile
drop on the bottom wall against the false wall density rho_w of the adhesion
force (Eq. 15, with the default G_wet), at 0.86 Tc, computed with the FP64
oracle only.

Protocol: 160x60 box, periodic in x, walls S/N (north wall at rho_v, i.e.
non-wetting), isothermal at 0.86 Tc, g_a = 0; a half-disc of saturated
liquid of radius 22 on the bottom wall, relaxed for 12000 steps.  The angle
is read from the drop height h (rho_mid crossing on the centre column) and
base width w (rho_mid crossings along the wall row): tan(theta/2) = 2h/w.
The wall density used by the flow-boiling channels for a ~60 degree angle
is read off this table, and the batched ensemble draws contact angles in
[30, 120] degrees and inverts them through it.  One process per wall
density, one thread each:

    python3 tests/golden/make_contact_angle.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "contact_angle_0p86Tc.json")
RHO_W = (1.9, 2.0, 2.1, 2.2, 2.4, 2.6, 3.0, 3.4, 3.8, 4.2, 4.6, 4.66, 4.7, 4.72, 4.74, 4.8, 5.0, 5.4)


def contact_angle(rw: float, nx=160, ny=60, R=22, steps=12000) -> dict:
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
    if len(liq) == 0:
        # the drop has left the wall: no contact (180 degrees)
        return {"rho_w": rw, "theta_deg": 180.0, "h": None if h is None else float(h), "w": 0.0}
    if len(liq) == nx:
        # a liquid film over the whole wall: complete wetting
        return {"rho_w": rw, "theta_deg": 0.0, "h": None if h is None else float(h), "w": float(nx)}
    if h is None:
        return {"rho_w": rw, "theta_deg": None, "h": None, "w": 0.0}
    i0, i1 = liq.min(), liq.max()
    a = i0 - (row[i0] - mid) / (row[i0] - row[i0 - 1])
    b = i1 + (row[i1] - mid) / (row[i1] - row[i1 + 1])
    w = b - a
    return {"rho_w": rw, "theta_deg": float(2 * np.degrees(np.arctan(2 * h / w))), "h": float(h), "w": float(w)}


def main():
    from concurrent.futures import ProcessPoolExecutor

    os.environ["OMP_NUM_THREADS"] = "1"
    with ProcessPoolExecutor(max_workers=min(len(RHO_W), os.cpu_count() or 1)) as ex:
        rows = list(ex.map(contact_angle, RHO_W))
    for r in rows:
        print(r, flush=True)
    doc = {"_comment": "Static contact angle vs false wall density (Eq. 15 adhesion), sessile drop, oracle only; "
                       "written by tests/golden/make_contact_angle.py",
           "T_over_Tc": 0.86, "omega": 0.344, "box": [160, 60], "drop_radius": 22, "steps": 12000,
           "table": rows}
    json.dump(doc, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main()
