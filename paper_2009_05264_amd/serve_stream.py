"""Serving stream: Poisson arrivals of flow-boiling solves driven through the
library's continuous-batching server (lbm_server_*), in real time.

Requests are drawn like the batched ensemble (Lx in {400, 800, 1200, 1600},
Ly in {50, 100, 200}, u_in ~ U[0.002, 0.01], superheat ~ U[0.05, 0.2],
contact angle ~ U[30, 120] degrees through the wall-density calibration
table) with step budgets ~ U{lo..hi}, FP16-deviation
storage with probability p16, and arrive with exponential gaps (seeded).
The host loop submits every request whose arrival time has passed and calls
the server's non-blocking pump, which retires a finished quantum, admits and
launches the next one; so arrivals are recorded as they happen, also while a
quantum runs, and a request that arrives while others are on the device
joins them at the next quantum (--blocking: the waiting pump instead, under
which an arrival is only submitted once the quantum on the device is over).  Reports aggregate MLUPS (lattice updates /
makespan), p50/p99 time to solution of the completed requests, the requests
the server failed (fields turned non-finite; they are retired and freed
while the others go on), and optionally checks sampled requests against the
same solve run alone, timing those solo runs (alone_MLUPS: the rate of the
same requests one at a time, the GPU to themselves).

    python3 paper_2009_05264_amd/serve_stream.py --requests 256 --rate 4
    python3 paper_2009_05264_amd/serve_stream.py --requests 256 --rate 1000   # saturated
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


def draw_stream(n, rate, lo, hi, p16, seed):
    import workloads as W

    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    t -= t[0]
    out = []
    for i in range(n):
        nx = int(rng.choice([400, 800, 1200, 1600]))
        ny = int(rng.choice([50, 100, 200]))
        cfg = W.Channel(nx=nx, ny=ny, u_in=float(rng.uniform(0.002, 0.01)),
                        superheat=float(rng.uniform(0.05, 0.2)), heater_len=int(0.4 * ny), seed=5000 + i)
        cfg.theta = float(rng.uniform(30.0, 120.0))
        cfg.rho_w = W.wall_density_for_angle(max(cfg.theta, W.MIN_PARTIAL_ANGLE))
        storage = "F16_DEV" if rng.uniform() < p16 else "F32_DEV"
        budget = int(rng.integers(lo, hi + 1))
        out.append((float(t[i]), cfg, storage, budget))
    return out


def params_of(L, W, cfg, storage):
    return L.default_params(storage=getattr(L, "STORE_" + storage), rho_ref=W.RHO_L, T_ref=cfg.T_sat,
                            **cfg.params())


def run_stream(n=64, rate=4.0, lo=5000, hi=50000, p16=0.5, seed=5, cap_gb=200.0, quantum=500,
               slots=512, check=0, stream=None, blocking=False):
    import workloads as W
    from paper_2009_05264_amd import lbmflow as L

    reqs = draw_stream(n, rate, lo, hi, p16, seed)
    srv = L.Server(int(cap_gb * 1e9), max_slots=slots, quantum=quantum, stream=stream)
    ids, tts = {}, {}
    check_set = set(np.random.default_rng(seed + 1).choice(n, size=min(check, n), replace=False).tolist())
    kept = {}
    failed = {}
    nxt = 0
    t0 = time.perf_counter()
    last_report = 0.0
    while len(tts) < n:
        now = time.perf_counter() - t0
        if now - last_report > 10.0:
            last_report = now
            print(f"[serve] t={now:.0f}s submitted={nxt} done={len(tts)}", file=sys.stderr, flush=True)
        while nxt < n and reqs[nxt][0] <= now:
            _, cfg, storage, budget = reqs[nxt]
            ia = cfg.init_args()
            rid = srv.submit(params_of(L, W, cfg, storage), budget, walls=cfg.walls(), rho_init=ia["rho_u"],
                             T_init=ia["T_u"], noise=ia["noise"], seed=ia["seed"])
            ids[rid] = nxt
            nxt += 1
        if blocking:
            running, in_flight = srv.pump(), False
        else:
            running, in_flight = srv.pump_async()
        for rid, k in list(ids.items()):
            st, t = srv.poll(rid)
            if st == L.REQ_FAILED:
                # its fields turned non-finite (the server freed it; the others go on)
                failed[k] = L.lib().lbm_last_error().decode()
                tts[k] = None
                del ids[rid]
                continue
            if st == L.REQ_DONE:
                tts[k] = t
                if k in check_set:
                    cfg = reqs[k][1]
                    kept[k] = srv.fields(rid, cfg.nx, cfg.ny)["rho"]
                srv.release(rid)
                del ids[rid]
        if running == 0 and not ids and nxt < n:
            time.sleep(max(0.0, min(0.05, reqs[nxt][0] - (time.perf_counter() - t0))))
        elif in_flight:
            time.sleep(2e-4)
    makespan = time.perf_counter() - t0
    info = srv.stats()
    srv.close()
    lups = info["lups"]  # lattice updates the device did (failed requests up to their failure)
    t = np.array([tts[k] for k in range(n) if tts[k] is not None])
    out = {"requests": n, "rate_per_s": rate, "budget_range": [lo, hi], "p_fp16": p16, "seed": seed,
           "cap_GB": cap_gb, "quantum_steps": quantum, "pump": "blocking" if blocking else "async",
           "aggregate_MLUPS": round(lups / makespan / 1e6, 1), "makespan_s": round(makespan, 2),
           "device_busy_s": round(info["busy_seconds"], 2),
           "tts_p50_s": round(float(np.percentile(t, 50)), 3), "tts_p99_s": round(float(np.percentile(t, 99)), 3),
           "peak_resident_GB": round(info["peak_resident_bytes"] / 1e9, 3),
           "failed_nonfinite": sorted(failed), "completed": int(len(t))}
    if check:
        bad = []
        solo_lups, solo_s = 0.0, 0.0
        for k, rho_mix in kept.items():
            _, cfg, storage, budget = reqs[k]
            d = L.Domain(params_of(L, W, cfg, storage), stream=stream)
            Ts, rws, heat, Tn, rwn = cfg.walls()
            d.set_wall(L.SIDE_S, Ts, rws, heat)
            d.set_wall(L.SIDE_N, Tn, rwn)
            d.init(**cfg.init_args())
            d.step(0)  # replay graphs captured outside the timing
            d.sync()
            t1 = time.perf_counter()
            d.step(budget)
            d.sync()
            solo_s += time.perf_counter() - t1
            solo_lups += float(cfg.nx) * cfg.ny * budget
            if not np.array_equal(d.fields()["rho"], rho_mix):
                bad.append(k)
            d.close()
        out["alone_vs_mix_checked"] = len(kept)
        out["alone_vs_mix_mismatch"] = bad
        if solo_s > 0:
            out["alone_MLUPS"] = round(solo_lups / solo_s / 1e6, 1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=4.0)
    ap.add_argument("--budget-lo", type=int, default=5000)
    ap.add_argument("--budget-hi", type=int, default=50000)
    ap.add_argument("--p-fp16", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--cap-gb", type=float, default=200.0)
    ap.add_argument("--quantum", type=int, default=500)
    ap.add_argument("--check", type=int, default=16)
    ap.add_argument("--blocking", action="store_true", help="the waiting pump (lbm_server_pump)")
    args = ap.parse_args()
    import torch

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    res = run_stream(args.requests, args.rate, args.budget_lo, args.budget_hi, args.p_fp16, args.seed,
                     args.cap_gb, args.quantum, check=args.check, blocking=args.blocking)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
