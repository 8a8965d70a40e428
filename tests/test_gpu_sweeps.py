"""Parameter trends of the flow-boiling channel from one batched ensemble
(Sec. 3B-3D of the paper): the bubble leaving the heater is smaller at a
higher inlet Reynolds number, nucleation comes earlier at a higher wall
superheat, and the bubble is larger on a less wetting wall (larger contact
angle).  200x50 channel, 19000 steps.  Deterministic: the step is bitwise
reproducible, so these are checks of the trends, not of noise."""
import pytest

pytestmark = pytest.mark.gpu


def test_departure_trends_batched():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import workloads as W
    from paper_2009_05264_amd import sweeps

    runs = [("u_in", u, W.Channel(u_in=u)) for u in (0.003, 0.004, 0.005)]
    runs += [("superheat", s, W.Channel(superheat=s)) for s in (0.12, 0.15)]
    runs += [("rho_w", r, W.Channel(rho_w=r)) for r in (3.4, 4.2)]
    print("case: batched sweep, 7 channels 200x50, 19000 steps", flush=True)
    res = sweeps.run(steps=19000, K=50, runs=runs)
    by = {(r["param"], r["value"]): r for r in res["runs"]}
    print(res["runs"], flush=True)
    assert all(r["finite"] for r in res["runs"])
    base = by[("u_in", 0.005)]  # u_in 0.005, superheat 0.1, rho_w 3.8 (~60 degrees)
    d = [by[("u_in", u)]["D_leave"] for u in (0.003, 0.004)] + [base["D_leave"]]
    assert None not in d and d[0] > d[1] > d[2]
    onset = [base["onset"], by[("superheat", 0.12)]["onset"], by[("superheat", 0.15)]["onset"]]
    assert onset[0] > onset[1] > onset[2]
    dw = [by[("rho_w", 4.2)]["D_leave"], base["D_leave"], by[("rho_w", 3.4)]["D_leave"]]  # 49, 60, 71 degrees
    assert None not in dw and dw[0] < dw[1] < dw[2]
