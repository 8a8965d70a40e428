"""Parameter sweeps of the flow-boiling channel as one batched ensemble
(Sec. 3B-3D of the paper: departure size and time against the inlet
Reynolds number, the wall superheat and the wettability).

Every run is one domain of a batch (one launch per step for all of them).
Every K steps the density fields are read back and the vapour (rho <
rho_mid) is labelled into 8-connected components.  Per run:

* onset: first sample with vapour on the heater;
* leave: first sample after onset at which no vapour component covers a
  heater cell (the bubble has slid or lifted off the heater); the size at
  that sample is the equivalent diameter D = 2 sqrt(A / pi) of the
  component(s) that covered the heater at the previous sample;
* lift: first sample at which such a component no longer touches the
  bottom wall row (departure into the stream), with its diameter;
* nonfinite: first sample with a non-finite density, if any.

    python3 paper_2009_05264_amd/sweeps.py --steps 18000
    python3 paper_2009_05264_amd/sweeps.py --c2 --steps 100000 --K 500
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


class Tracker:
    def __init__(self, heater: np.ndarray, rho_mid: float):
        self.hx = np.where(heater == 1)[0]
        self.mid = rho_mid
        self.prev = None  # mask of the components covering the heater at the previous sample
        self.onset = self.leave = self.lift = None
        self.D_leave = self.D_lift = None
        self.nonfinite = None

    def sample(self, step: int, rho: np.ndarray):
        from scipy import ndimage

        if self.nonfinite is None and not np.isfinite(rho).all():
            self.nonfinite = step

        vap = rho < self.mid
        lab, _ = ndimage.label(vap, structure=np.ones((3, 3)))
        on = np.unique(lab[0, self.hx])
        on = on[on > 0]
        if self.onset is None and len(on):
            self.onset = step
        if self.prev is not None:
            ids = np.unique(lab[self.prev & vap])
            ids = ids[ids > 0]
            if self.lift is None:
                for i in ids:
                    comp = lab == i
                    if not comp[0].any():
                        self.lift, self.D_lift = step, 2.0 * math.sqrt(comp.sum() / math.pi)
                        break
            if self.leave is None and self.onset is not None and not len(on):
                area = int(np.isin(lab, ids).sum()) if len(ids) else 0
                self.leave, self.D_leave = step, 2.0 * math.sqrt(area / math.pi)
        self.prev = np.isin(lab, on) if len(on) else None

    def result(self):
        return {"onset": self.onset, "leave": self.leave, "D_leave": self.D_leave, "lift": self.lift,
                "D_lift": self.D_lift, "nonfinite": self.nonfinite}


def runs_default():
    """(label, Channel) pairs: Re_in, superheat and wettability sweeps around
    the 200x50 channel (u_in 0.005, superheat 0.1 T_sat, rho_w 3.8)."""
    import workloads as W

    out = []
    for u in (0.002, 0.0025, 0.003, 0.004, 0.005, 0.007):
        out.append(("u_in", u, W.Channel(u_in=u)))
    for sh in (0.08, 0.12, 0.15, 0.2):
        out.append(("superheat", sh, W.Channel(superheat=sh)))
    for rw in (3.0, 3.4, 4.2):  # ~83, 71, 49 degrees (60 at 3.8), sessile-drop table at 0.86 Tc
        out.append(("rho_w", rw, W.Channel(rho_w=rw)))
    return out


def runs_c2():
    """(label, value, Channel): the nine 1600x200 channels of the benchmark
    sweep, superheat in {0.05, 0.1, 0.15} T_sat x u_in in {0.002, 0.005,
    0.01}, 80-cell heater."""
    import workloads as W

    return [("c2", f"superheat {s} u_in {u}", W.c2(s, u)) for s, u in W.C2_SWEEP]


def run(steps: int = 18000, K: int = 50, storage: str = "F32_DEV", runs=None, fields: bool = False):
    """Step the runs as one batch, sampling every K steps; fields=True also
    returns each run's final rho, u_act and T (key "fields")."""
    import torch

    import workloads as W
    from paper_2009_05264_amd import lbmflow as L

    torch.cuda.set_device(0)
    runs = runs_default() if runs is None else runs
    st = getattr(L, "STORE_" + storage)
    doms, trk = [], []
    for _, _, cfg in runs:
        p = L.default_params(storage=st, rho_ref=W.RHO_L, T_ref=cfg.T_sat, **cfg.params())
        d = L.Domain(p)
        Ts, rws, heat, Tn, rwn = cfg.walls()
        d.set_wall(L.SIDE_S, Ts, rws, heat)
        d.set_wall(L.SIDE_N, Tn, rwn)
        d.init(**cfg.init_args())
        doms.append(d)
        trk.append(Tracker(cfg.heater(), cfg.params()["rho_mid"]))
    b = L.Batch(doms)
    t0 = time.time()
    for k in range(steps // K):
        b.step(K)
        b.sync()
        for d, t in zip(doms, trk):
            t.sample((k + 1) * K, d.fields()["rho"])
    wall = time.time() - t0
    nodes = sum(d.nx * d.ny for d in doms)
    out = []
    for (name, val, cfg), d, t in zip(runs, doms, trk):
        r = t.result()
        f = d.fields()
        r.update({"param": name, "value": val, "Re_in": cfg.u_in * cfg.ny / ((1.0 - 0.5) / 3.0),
                  "finite": bool(np.isfinite(f["rho"]).all())})
        if fields:
            r["fields"] = f
        out.append(r)
    b.close()
    for d in doms:
        d.close()
    fit = fit_power([(r["Re_in"], r["D_leave"]) for r in out if r["param"] == "u_in"])
    return {"steps": steps, "K": K, "storage": storage, "runs": out, "fit_D_leave_vs_Re": fit,
            "wall_s": round(wall, 2), "batched_MLUPS_incl_readback": round(nodes * steps / wall / 1e6, 1)}


def fit_power(pts):
    """Least-squares fit of log D = log c + k log x over the points with a value."""
    pts = [(x, y) for x, y in pts if y is not None and y > 0]
    if len(pts) < 2:
        return None
    k, lc = np.polyfit(np.log([p[0] for p in pts]), np.log([p[1] for p in pts]), 1)
    return {"c": float(math.exp(lc)), "k": float(k), "n": len(pts)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=18000)
    ap.add_argument("--K", type=int, default=50)
    ap.add_argument("--storage", default="F32_DEV")
    ap.add_argument("--c2", action="store_true", help="the nine 1600x200 channels of the benchmark sweep")
    a = ap.parse_args()
    print(json.dumps(run(a.steps, a.K, a.storage, runs=runs_c2() if a.c2 else None)), flush=True)


if __name__ == "__main__":
    main()
