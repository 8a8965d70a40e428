"""Pool boiling (Sec. 2D, Fig. 5) on the GPU: one pool box against the
oracle, and the departure diameter falling with gravity in one batched
ensemble (the paper fits D_d = 0.246 g^-0.49)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_pool_member_matches_oracle():
    """The 512x128 pool box at g = 5e-5 with its heater on from the start,
    100 steps, GPU against the oracle: 1e-5 on rho and T, 1e-4 on u.  The
    velocity error sits in the vapour layer above the pool: its populations
    are stored as deviations from the liquid reference (rho 0.59 against
    5.88, i.e. -5.3 w_i), whose FP32 rounding leaves ~6e-7 absolute in u_act
    there -- with or without heater and gravity (measured on MI355X) -- while
    the largest velocity, ~0.014, is the free surface's own relaxation: 5e-5
    of it.  (The vapour patch that nucleates on the 1.2 Tc heater within
    ~200 steps then amplifies rounding differences -- 2e-4 of max |u| by
    1500 steps -- so longer pool runs are compared through their departure
    statistics.)"""
    _torch()
    from oracle import oracle as O
    from paper_2009_05264_amd import lbmflow as L

    cfg = W.Pool(ga=5e-5)
    print("case: pool 512x128 vs oracle, 100 steps", flush=True)
    d = L.Domain(L.default_params(storage=L.STORE_F32_DEV, rho_ref=W.RHO_L_POOL, T_ref=cfg.T_sat, **cfg.params()))
    o = O.Oracle(O.Params(**cfg.params()))
    Ts, rws, heat, Tn, rwn = cfg.walls()
    d.set_wall(L.SIDE_S, Ts, rws, heat)
    d.set_wall(L.SIDE_N, Tn, rwn)
    o.set_wall(0, Ts, rws, heat)
    o.set_wall(1, Tn, rwn)
    d.init(**cfg.init_args())
    o.init(**cfg.init_args())
    d.step(100)
    o.step(100)
    g, r = d.fields(), o.fields()
    assert r["T"][0, heat == 1].min() > 1.05 * cfg.T_sat  # the heater has warmed its cells
    e = {k: float(np.abs(g[k] - r[k]).max() / np.abs(r[k]).max()) for k in ("rho", "T")}
    umax = max(np.abs(r["ux"]).max(), np.abs(r["uy"]).max())
    du = float(max(np.abs(g["ux"] - r["ux"]).max(), np.abs(g["uy"] - r["uy"]).max()))
    e["u"] = du / umax
    print(e, "max |u|", umax, "abs du", du, flush=True)
    assert e["rho"] < 1e-5 and e["T"] < 1e-5 and e["u"] < 1e-4, e


def test_departure_diameter_falls_with_gravity():
    """Three pool boxes (g = 5e-5, 1e-4, 1.5e-4) stepped as one batch for
    100 000 steps: the heater's bubble departs periodically in each, D_d
    (mean of the first five departures) falls as g rises, and the fitted
    exponent of D_d ~ g^k lies near Fritz's -1/2 (the paper: -0.49)."""
    _torch()
    from paper_2009_05264_amd import pool

    print("case: pool boiling, 3 boxes 512x128, 100000 steps", flush=True)
    res = pool.run(gs=(5e-5, 1e-4, 1.5e-4), steps=100000, K=400)
    for r in res["runs"]:
        print(r["g"], r["D_d"], r["period"], r["departures"][:6], flush=True)
    print(res["fit"], flush=True)
    assert all(r["finite"] for r in res["runs"])
    dd = [r["D_d"] for r in res["runs"]]
    assert None not in dd and dd[0] > dd[1] > dd[2]
    assert -0.7 < res["fit"]["k"] < -0.3
