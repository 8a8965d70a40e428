"""GPU tests of the serving loop (lbm_server_*): requests of different sizes,
parameters and storage kinds arrive while others run, are admitted under a
memory cap, and each result equals the same solve run alone."""
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05264_amd import lbmflow

    lbmflow.lib()
    return lbmflow


def request_set():
    """Ten small flow-boiling channels with different sizes, inlet speeds,
    superheats, wettabilities, seeds, storage kinds and step budgets."""
    rng = np.random.default_rng(11)
    sizes = [(130, 40), (200, 50), (250, 30), (190, 64), (67, 13)]
    out = []
    for i in range(10):
        nx, ny = sizes[i % len(sizes)]
        cfg = W.Channel(nx=nx, ny=ny, u_in=float(rng.uniform(0.002, 0.01)),
                        superheat=float(rng.uniform(0.05, 0.2)), heater_len=max(2, int(0.4 * ny)),
                        rho_w=float(rng.uniform(3.0, 4.6)), seed=100 + i)
        storage = "F16_DEV" if i % 3 == 2 else "F32_DEV"
        budget = int(rng.choice([60, 100, 140, 200]))
        out.append((cfg, storage, budget))
    return out


def params_of(L, cfg, storage):
    return L.default_params(storage=getattr(L, "STORE_" + storage), rho_ref=W.RHO_L, T_ref=cfg.T_sat,
                            **cfg.params())


def run_alone(L, cfg, storage, budget):
    d = L.Domain(params_of(L, cfg, storage))
    Ts, rws, heat, Tn, rwn = cfg.walls()
    d.set_wall(L.SIDE_S, Ts, rws, heat)
    d.set_wall(L.SIDE_N, Tn, rwn)
    d.init(**cfg.init_args())
    d.step(budget)
    f, g = d.fields(), d.diag()
    d.close()
    return f, g


def submit(L, srv, cfg, storage, budget):
    ia = cfg.init_args()
    return srv.submit(params_of(L, cfg, storage), budget, walls=cfg.walls(), rho_init=ia["rho_u"],
                      T_init=ia["T_u"], noise=ia["noise"], seed=ia["seed"])


def test_results_equal_alone_and_in_the_mix(L):
    reqs = request_set()
    fps = [L.required_bytes(params_of(L, c, s)) for c, s, _ in reqs]
    cap = sum(sorted(fps)[-4:])  # about four resident at a time: later arrivals queue
    srv = L.Server(cap, max_slots=6, quantum=40)
    print(f"case: server cap={cap} requests={len(reqs)}", flush=True)
    ids = {}
    # half arrive up front, the rest one per quantum while the first ones run
    for k in range(5):
        ids[submit(L, srv, *reqs[k])] = k
    pending = list(range(5, len(reqs)))
    results, tts = {}, {}
    for _ in range(1000):
        if pending:
            k = pending.pop(0)
            ids[submit(L, srv, *reqs[k])] = k
        running = srv.pump()
        for rid, k in list(ids.items()):
            st, t = srv.poll(rid)
            assert st != L.REQ_FAILED
            if st == L.REQ_DONE and k not in results:
                cfg = reqs[k][0]
                results[k] = (srv.fields(rid, cfg.nx, cfg.ny), srv.diag(rid))
                tts[k] = t
                srv.release(rid)
        info = srv.stats()
        assert info["peak_resident_bytes"] <= cap
        if not pending and running == 0 and info["queued"] == 0:
            break
    info = srv.stats()
    srv.close()
    assert len(results) == len(reqs), (len(results), info)
    assert info["resident_bytes"] == 0 and info["done"] == len(reqs)
    assert info["lups"] == pytest.approx(sum(c.nx * c.ny * b for c, _, b in reqs))
    for k, (cfg, storage, budget) in enumerate(reqs):
        f_mix, d_mix = results[k]
        f_alone, d_alone = run_alone(L, cfg, storage, budget)
        for key in f_alone:
            assert np.array_equal(f_mix[key], f_alone[key]), (k, key)
        assert d_mix["step"] == budget and d_mix["mass"] == d_alone["mass"], k
        assert tts[k] > 0


def test_server_member_matches_oracle(L):
    """A request served in a mix of requests against the oracle: the first
    FP32 request of the set (130x40), 1e-5 after its budget."""
    from oracle import oracle as O

    reqs = request_set()
    srv = L.Server(1 << 34, max_slots=8, quantum=30)
    print("case: server member vs oracle", flush=True)
    ids = [submit(L, srv, *r) for r in reqs[:4]]
    for _ in range(100):
        if srv.pump() == 0 and srv.stats()["queued"] == 0:
            break
    cfg, storage, budget = reqs[0]
    assert storage == "F32_DEV" and srv.poll(ids[0])[0] == L.REQ_DONE
    g = srv.fields(ids[0], cfg.nx, cfg.ny)
    srv.close()
    o = O.Oracle(O.Params(**cfg.params()))
    Ts, rws, heat, Tn, rwn = cfg.walls()
    o.set_wall(0, Ts, rws, heat)
    o.set_wall(1, Tn, rwn)
    o.init(**cfg.init_args())
    o.step(budget)
    r = o.fields()
    umax = max(np.abs(r["ux"]).max(), np.abs(r["uy"]).max())
    e = {k: float(np.abs(g[k] - r[k]).max() / np.abs(r[k]).max()) for k in ("rho", "T")}
    e["u"] = float(max(np.abs(g["ux"] - r["ux"]).max(), np.abs(g["uy"] - r["uy"]).max()) / umax)
    print(budget, e)
    assert max(e.values()) < 1e-5, e


def test_cancel_and_cap(L):
    cfg, storage, _ = request_set()[1]
    fp = L.required_bytes(params_of(L, cfg, storage))
    srv = L.Server(fp, max_slots=4, quantum=20)  # room for one at a time
    print("case: server cancel", flush=True)
    a = submit(L, srv, cfg, storage, 100)
    b = submit(L, srv, cfg, storage, 100)
    c = submit(L, srv, cfg, storage, 40)
    srv.pump()
    assert srv.poll(a)[0] == L.REQ_RUNNING and srv.poll(b)[0] == L.REQ_QUEUED
    srv.cancel(b)
    srv.cancel(a)
    assert srv.poll(a)[0] == L.REQ_CANCELLED and srv.poll(b)[0] == L.REQ_CANCELLED
    for _ in range(10):
        if srv.pump() == 0 and srv.stats()["queued"] == 0:
            break
    assert srv.poll(c)[0] == L.REQ_DONE
    f = srv.fields(c, cfg.nx, cfg.ny)
    f_alone, _ = run_alone(L, cfg, storage, 40)
    assert np.array_equal(f["rho"], f_alone["rho"])
    srv.release(c)
    assert srv.stats()["resident_bytes"] == 0
    # a request larger than the cap is refused, not queued
    big = W.Channel(nx=cfg.nx * 4, ny=cfg.ny)
    with pytest.raises(L.LbmError) as e:
        submit(L, srv, big, storage, 10)
    assert e.value.code == L.LBM_E_CAP
    srv.close()


@pytest.mark.parametrize("pump", ["blocking", "async"])
def test_non_finite_request_fails_alone(L, pump):
    """Failure isolation: among three ordinary requests, one whose buoyancy
    (g_a = -1 in lattice units) drives its fields non-finite within a few
    dozen steps is retired as failed (LBM_E_NAN) at the end of that quantum,
    with its memory freed; the other three finish and equal their solo runs
    bitwise.  With either pump."""
    reqs = request_set()[:3]
    bad = W.Channel(nx=67, ny=13, heater_len=5, seed=3, extra=dict(ga_y=-1.0))
    srv = L.Server(1 << 34, max_slots=8, quantum=40)
    print(f"case: server with one diverging request, {pump} pump", flush=True)
    ids = {submit(L, srv, *r): k for k, r in enumerate(reqs)}
    bad_id = submit(L, srv, bad, "F32_DEV", 120)
    results = {}
    for _ in range(100000):
        if pump == "async":
            running, in_flight = srv.pump_async()
            if in_flight:
                time.sleep(1e-4)
                continue
        else:
            running = srv.pump()
        for rid, k in ids.items():
            st, _ = srv.poll(rid)
            assert st != L.REQ_FAILED, k
            if st == L.REQ_DONE and k not in results:
                cfg = reqs[k][0]
                results[k] = srv.fields(rid, cfg.nx, cfg.ny)
                srv.release(rid)
        if running == 0 and srv.stats()["queued"] == 0:
            break
    st, t = srv.poll(bad_id)
    assert st == L.REQ_FAILED and t == -1.0
    assert "non-finite" in L.lib().lbm_last_error().decode()
    info = srv.stats()
    srv.close()
    assert info["failed"] == 1 and info["done"] == 3 and info["resident_bytes"] == 0
    for k, (cfg, storage, budget) in enumerate(reqs):
        f_alone, _ = run_alone(L, cfg, storage, budget)
        for key in f_alone:
            assert np.array_equal(results[k][key], f_alone[key]), (k, key)


def test_async_pump_takes_arrivals_while_a_quantum_runs(L):
    """The non-blocking pump: it launches a quantum and returns with it on
    the device; requests submitted meanwhile join at the next quantum; every
    result equals the same solve run alone (bitwise); a blocking pump after
    an asynchronous one settles the quantum left on the device."""
    reqs = request_set()
    srv = L.Server(1 << 34, max_slots=8, quantum=40)
    print("case: server async pump", flush=True)
    ids = {submit(L, srv, *reqs[k]): k for k in range(3)}
    running, in_flight = srv.pump_async()
    assert running == 3 and in_flight  # launched, not waited for
    pending = list(range(3, len(reqs)))
    results = {}
    saw_submit_in_flight = False
    for _ in range(200000):
        if pending and in_flight:
            k = pending.pop(0)
            ids[submit(L, srv, *reqs[k])] = k  # arrives while a quantum runs
            saw_submit_in_flight = True
        running, in_flight = srv.pump_async()
        for rid, k in list(ids.items()):
            st, t = srv.poll(rid)
            assert st != L.REQ_FAILED, k
            if st == L.REQ_DONE and k not in results:
                cfg = reqs[k][0]
                results[k] = srv.fields(rid, cfg.nx, cfg.ny)
                assert t > 0
                srv.release(rid)
        if not pending and running == 0 and not in_flight and srv.stats()["queued"] == 0:
            break
        if in_flight:
            time.sleep(1e-4)
    assert saw_submit_in_flight
    info = srv.stats()
    assert len(results) == len(reqs), (len(results), info)
    assert info["done"] == len(reqs) and info["resident_bytes"] == 0
    assert info["lups"] == pytest.approx(sum(c.nx * c.ny * b for c, _, b in reqs))
    assert 0 < info["busy_seconds"]
    for k, (cfg, storage, budget) in enumerate(reqs):
        f_alone, _ = run_alone(L, cfg, storage, budget)
        for key in f_alone:
            assert np.array_equal(results[k][key], f_alone[key]), (k, key)
    # a blocking pump settles what an asynchronous one left running
    cfg, storage, _ = reqs[0]
    rid = submit(L, srv, cfg, storage, 80)
    running, in_flight = srv.pump_async()
    assert in_flight
    srv.pump()  # retires the first quantum (40 steps), runs and retires the second
    assert srv.poll(rid)[0] == L.REQ_DONE
    f_alone, _ = run_alone(L, cfg, storage, 80)
    assert np.array_equal(srv.fields(rid, cfg.nx, cfg.ny)["rho"], f_alone["rho"])
    srv.close()
