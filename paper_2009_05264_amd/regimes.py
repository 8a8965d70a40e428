"""Flow-boiling regimes of the paper's channel (Sec. 2C, Sec. 3C) from one
batched ensemble: inlet Reynolds number x wall superheat, every run a domain
of one batch (one launch per step for all of them).

Channel: 40 x 1000 at T_in = T_sat = 0.9 Tc (R134a, omega 0.32), the
constant-pressure exit at rho_l, 10 000 unheated steps, then the heater (at
L/5 on the bottom wall) on.  Every K heated steps the density fields are read
back; the vapour (rho < rho_mid) is labelled into 8-connected components and
each run is classified over the heated window:

* slug: a vapour component spans at least 3/4 of the channel height;
* departing bubbles: a component descended from the heater's vapour leaves
  the bottom wall;
* attached bubble: vapour on the heater that neither spans nor departs;
* none: no vapour.

    python3 paper_2009_05264_amd/regimes.py --heated 15000
    python3 paper_2009_05264_amd/regimes.py --thermal-search
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

NX, NY = 1000, 40


def channel_params(Re, rho_l, rho_v, Tc):
    Tin = 0.9 * Tc
    return dict(nx=NX, ny=NY, bc_x=2, bc_y=1, rho_out=rho_l, u_in=Re * (1.0 / 6.0) / NY, T_in=Tin, T_iso=Tin,
                rho_mid=0.5 * (rho_l + rho_v), ga_y=-5e-5, tau_f=1.0, tau_g=0.6, c_v=6.0, omega=0.32)


def classify(trace, depart):
    """trace: (step, vapour nodes, largest vertical span) per sample."""
    if not any(v for _, v, _ in trace):
        return "none"
    if max(s for _, _, s in trace) >= 0.75 * NY:
        return "slug"
    return "departing bubbles" if depart else "attached bubble"


def run(Res=(0.48, 0.96, 1.92), Ths=(1.2, 1.4), heater_len=11, heated=15000, K=500, warmup=10000):
    from scipy import ndimage
    import torch

    import workloads as W
    from paper_2009_05264_amd import lbmflow as L

    torch.cuda.set_device(0)
    Tc = W.TC
    rl, rv = W.RHO_L_POOL, W.RHO_V_POOL  # saturated at 0.9 Tc, omega 0.32
    Tin = 0.9 * Tc
    rw = rv + 0.6 * (rl - rv)
    heat = np.zeros(NX, np.int32)
    x0 = NX // 5 - heater_len // 2
    heat[x0: x0 + heater_len] = 1
    runs, doms = [], []
    for Re in Res:
        for Th in Ths:
            d = L.Domain(L.default_params(storage=L.STORE_F32_DEV, rho_ref=rl, T_ref=Tin,
                                          **channel_params(Re, rl, rv, Tc)))
            for side in (0, 1):
                d.set_wall(side, np.full(NX, Tin), np.full(NX, rw))
            d.init(rho_u=rl, T_u=Tin, noise=1e-3, seed=11)
            doms.append(d)
            runs.append({"Re_in": Re, "T_heater_over_Tc": Th, "trace": [], "depart": None})
    b = L.Batch(doms)
    b.step(warmup)
    b.close()
    for d, r in zip(doms, runs):
        d.set_wall(L.SIDE_S, np.where(heat == 1, r["T_heater_over_Tc"] * Tc, Tin), np.full(NX, rw), heat)
    b = L.Batch(doms)
    mid = 0.5 * (rl + rv)
    lineage = [None] * len(doms)
    t0 = time.time()
    for k in range(heated // K):
        b.step(K)
        b.sync()
        step = warmup + (k + 1) * K
        for i, (d, r) in enumerate(zip(doms, runs)):
            rho = d.fields()["rho"]
            if not np.isfinite(rho).all():
                r.setdefault("nonfinite", step)
                continue
            vap = rho < mid
            lab, n = ndimage.label(vap, structure=np.ones((3, 3)))
            span = 0
            for c in range(1, n + 1):
                ys = np.where((lab == c).any(axis=1))[0]
                span = max(span, int(ys.max() - ys.min() + 1))
            r["trace"].append((step, int(vap.sum()), span))
            keep = set(np.unique(lab[0, heat == 1]).tolist()) - {0}
            if lineage[i] is not None:
                for c in set(np.unique(lab[lineage[i] & vap]).tolist()) - {0}:
                    if (lab == c)[0].any():
                        keep.add(c)
                    elif r["depart"] is None:
                        r["depart"] = step
            lineage[i] = np.isin(lab, list(keep)) if keep else None
    b.close()
    for d in doms:
        d.close()
    for r in runs:
        r["regime"] = classify(r["trace"], r["depart"]) if "nonfinite" not in r else "diverged"
        r["max_span"] = max((s for _, _, s in r["trace"]), default=0)
        r["max_vapour"] = max((v for _, v, _ in r["trace"]), default=0)
        del r["trace"]
    return {"heater_len": heater_len, "warmup": warmup, "heated": heated, "K": K, "runs": runs,
            "wall_s": round(time.time() - t0, 1)}


def thermal_search(heaters=(5, 11), Ths=(1.1, 1.2, 1.4), cvs=(6.0, 12.0, 24.0), taus=(0.55, 0.6, 0.8),
                   wall_fracs=(0.6,), Re=0.96, heated=40000, K=250, warmup=10000):
    """The channel at one Re_in over the thermal parameters the paper does not
    print (c_v, tau_g), the heater length and temperature and the false wall
    density rho_v + f (rho_l - rho_v), all runs as one batch: bubble onset,
    departures of the heater's bubbles (a component of the heater's lineage
    that leaves the bottom wall, with its equivalent diameter), the step at
    which a run turned non-finite, the largest vapour span and area."""
    import itertools

    import torch
    from scipy import ndimage

    import workloads as W
    from paper_2009_05264_amd import lbmflow as L
    from paper_2009_05264_amd.pool import Departures

    torch.cuda.set_device(0)
    Tc = W.TC
    rl, rv = W.RHO_L_POOL, W.RHO_V_POOL
    Tin = 0.9 * Tc
    mid = 0.5 * (rl + rv)
    doms, runs = [], []
    for hl, Th, cv, tg, wf in itertools.product(heaters, Ths, cvs, taus, wall_fracs):
        prm = channel_params(Re, rl, rv, Tc)
        prm.update(c_v=cv, tau_g=tg)
        d = L.Domain(L.default_params(storage=L.STORE_F32_DEV, rho_ref=rl, T_ref=Tin, **prm))
        rw = rv + wf * (rl - rv)
        for side in (0, 1):
            d.set_wall(side, np.full(NX, Tin), np.full(NX, rw))
        d.init(rho_u=rl, T_u=Tin, noise=1e-3, seed=11)
        heat = np.zeros(NX, np.int32)
        x0 = NX // 5 - hl // 2
        heat[x0: x0 + hl] = 1
        doms.append(d)
        runs.append(dict(heater=hl, T_heater_over_Tc=Th, c_v=cv, tau_g=tg, wall_frac=wf, rw=rw, heat=heat,
                         trk=Departures(heat, mid, NY + 8), max_span=0, max_vapour=0))
    b = L.Batch(doms)
    b.step(warmup)
    b.close()
    for d, r in zip(doms, runs):
        d.set_wall(L.SIDE_S, np.where(r["heat"] == 1, r["T_heater_over_Tc"] * Tc, Tin), np.full(NX, r["rw"]),
                   r["heat"])
    b = L.Batch(doms)
    for k in range(heated // K):
        b.step(K)
        b.sync()
        step = warmup + (k + 1) * K
        for d, r in zip(doms, runs):
            if "nonfinite" in r:
                continue
            rho = d.fields()["rho"]
            if not np.isfinite(rho).all():
                r["nonfinite"] = step
                continue
            r["trk"].sample(step, rho)
            vap = rho < mid
            r["max_vapour"] = max(r["max_vapour"], int(vap.sum()))
            if vap.any():
                lab, n = ndimage.label(vap, structure=np.ones((3, 3)))
                for c in range(1, n + 1):
                    ys = np.where((lab == c).any(axis=1))[0]
                    r["max_span"] = max(r["max_span"], int(ys.max() - ys.min() + 1))
    b.close()
    out = []
    for d, r in zip(doms, runs):
        res = r.pop("trk").result()
        r.pop("heat")
        r.pop("rw")
        r.update(onset=res["onset"], departures=res["departures"], nonfinite=r.get("nonfinite"))
        out.append(r)
        d.close()
    return {"Re_in": Re, "warmup": warmup, "heated": heated, "K": K, "runs": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--heated", type=int, default=15000)
    ap.add_argument("--thermal-search", action="store_true",
                    help="the search over c_v, tau_g, heater length and temperature at Re_in 0.96")
    a = ap.parse_args()
    if a.thermal_search:
        print(json.dumps(thermal_search()), flush=True)
        print(json.dumps(thermal_search(Ths=(1.2, 1.4), cvs=(6.0, 12.0), taus=(0.6,),
                                        wall_fracs=(0.6, 0.75, 0.9, 1.0))), flush=True)
    else:
        print(json.dumps(run(heated=a.heated)), flush=True)


if __name__ == "__main__":
    main()
