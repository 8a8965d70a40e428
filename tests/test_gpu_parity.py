"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs, plus determinism, tiling invariance, checkpoint and
batching identities.  Tolerance: relative L-infinity after the given number
of steps, per field, normalised by the oracle's max |field| (velocity by the
max over both components) -- 1e-5 for FP32 storage."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _torch_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def L():
    _torch_gpu()
    from paper_2009_05264_amd import lbmflow

    lbmflow.lib()
    return lbmflow


def rel_errors(g, r):
    out = {}
    for k in ("rho", "T"):
        out[k] = float(np.abs(g[k] - r[k]).max() / np.abs(r[k]).max())
    umax = max(np.abs(r["ux"]).max(), np.abs(r["uy"]).max())
    out["u"] = float(max(np.abs(g["ux"] - r["ux"]).max(), np.abs(g["uy"] - r["uy"]).max()) / umax)
    return out


def make_gpu(L, cfg, storage=None, rows=None, **over):
    storage = L.STORE_F32_DEV if storage is None else storage
    kw = cfg.params()
    kw.update(over)
    ref = dict(rho_ref=W.RHO_L, T_ref=cfg.T_sat) if storage != L.STORE_F32 else {}
    p = L.default_params(storage=storage, **ref, **kw)
    d = L.Domain(p)
    if kw.get("bc_y", 1) == 1:
        Ts, rws, heat, Tn, rwn = cfg.walls()
        d.set_wall(L.SIDE_S, Ts, rws, heat)
        d.set_wall(L.SIDE_N, Tn, rwn)
    if rows:
        d.set_tile_rows(rows)
    return d


def make_oracle(cfg, **over):
    from oracle import oracle as O

    kw = cfg.params()
    kw.update(over)
    o = O.Oracle(O.Params(**kw))
    if kw.get("bc_y", 1) == 1:
        Ts, rws, heat, Tn, rwn = cfg.walls()
        o.set_wall(0, Ts, rws, heat)
        o.set_wall(1, Tn, rwn)
    return o


def run_pair(L, cfg, steps, storage=None, rows=None, init=None, **over):
    d = make_gpu(L, cfg, storage=storage, rows=rows, **over)
    o = make_oracle(cfg, **over)
    ia = cfg.init_args() if init is None else init
    d.init(**ia)
    o.init(**ia)
    d.step(steps)
    o.step(steps)
    return d, o


@pytest.mark.parametrize("storage", ["F32_DEV", "F32"])
def test_channel_200x50_100_steps(L, storage):
    """The 200x50 flow-boiling channel, 100 steps, FP32 compute.  Parity
    (1e-5) is claimed for FP32 deviation storage, the storage of every
    benchmark and parity run.  Plain FP32 storage of the whole populations
    rounds each f_i (up to ~2.9) to 24 bits every step; that rounding alone
    puts u at ~2e-5 after 100 steps (measured 2.1e-5 on MI355X), so it is a
    point of the precision study with the 5e-5 bound, not a parity case."""
    st = getattr(L, "STORE_" + storage)
    print(f"case: channel 200x50 storage={storage}", flush=True)
    d, o = run_pair(L, W.c1(), 100, storage=st)
    e = rel_errors(d.fields(), o.fields())
    print(e)
    tol = TOL if st == L.STORE_F32_DEV else 5 * TOL
    assert e["rho"] < tol and e["T"] < tol and e["u"] < tol, e


def test_channel_diagnostics(L):
    cfg = W.c1()
    d, o = run_pair(L, cfg, 60)
    gd, od = d.diag(), o.diag()
    for k in ("mass", "energy"):
        assert gd[k] == pytest.approx(od[k], rel=1e-6), k
    assert gd["heater_q"] == pytest.approx(od["heater_q"], rel=1e-3, abs=1e-7)
    assert gd["vapor_cells"] == od["vapor_cells"]
    assert gd["psi_clamped"] == 0 and gd["nonfinite"] == 0
    assert gd["p_in"] == pytest.approx(od["p_in"], rel=1e-4, abs=1e-6)
    assert gd["p_out"] == pytest.approx(od["p_out"], rel=1e-4, abs=1e-6)
    assert gd["step"] == 60
    # the derived numbers: heater Nusselt number from the oracle's heater flux
    # (R25: ny / (T_h - T_in) x mean over heater cells of (T_h - T) / (1/2))
    # and the centreline pressure drop, in the read-out and in the history
    n_heat = int(cfg.heater().sum())
    nu_o = cfg.ny / (cfg.T_heater - cfg.T_in) * od["heater_q"] / n_heat
    assert gd["nu_heater"] == pytest.approx(nu_o, rel=1e-3, abs=1e-6)
    assert gd["dp"] == pytest.approx(od["p_in"] - od["p_out"], rel=1e-3, abs=1e-6)
    h = d.diag_history(4)[-1]
    assert h["nu_heater"] == pytest.approx(cfg.ny / (cfg.T_heater - cfg.T_in) * h["heater_q"] / n_heat, rel=1e-12)
    assert h["dp"] == h["p_in"] - h["p_out"]


@pytest.mark.parametrize("nx,ny,bcx,bcy", [
    (7, 5, 0, 0),      # tiny periodic box (several wraps per strip)
    (67, 13, 0, 1),    # two strips, ragged tail, walls
    (121, 9, 1, 1),    # channel, 3 strips with a 1-column last strip
    (3, 4, 1, 1),      # smallest channel
    (61, 70, 1, 0),    # channel periodic in y, several row segments
    (121, 9, 2, 1),    # constant-pressure exit, walls
    (3, 4, 2, 1),      # smallest channel with the pressure exit
    (61, 70, 2, 0),    # pressure exit, periodic in y
])
def test_shapes_and_boundaries(L, nx, ny, bcx, bcy):
    """Ragged tiles and every boundary combination, 100 steps, with a vapour
    bubble (tanh interface) so that interfaces cross tile edges; 1e-5 on rho
    and T everywhere, and on u except in three cases whose velocity error is
    set by the FP32 resolution of the interface forces against a small or
    transient velocity scale (measured on MI355X):
      * 7x5, periodic: the fluid is nearly at rest (max |u| ~1.2e-3); the
        absolute error ~5e-8 is 6e-5 of that -> 1e-4;
      * 67x13 between walls: a radius-4 bubble filling a third of the gap,
        max |u| ~0.014; absolute error ~1.4e-7, 1.0e-5 -> 2e-5;
      * 61x70 channel periodic in y (either exit): the bubble's initial
        adjustment drives max |u| to ~0.13 within 20 steps, where the
        absolute error of ~1.5e-6 is set and then stays; 1.3e-5 -> 2e-5."""
    print(f"case: {nx}x{ny} bc=({bcx},{bcy})", flush=True)
    cfg = W.Channel(nx=nx, ny=ny, heater_len=max(1, nx // 5))
    y, x = np.mgrid[0:ny, 0:nx]
    rad = np.sqrt((x - nx / 3) ** 2 + (y - ny / 2) ** 2)
    r0 = W.RHO_V + (W.RHO_L - W.RHO_V) * 0.5 * (1 + np.tanh((rad - min(nx, ny) / 3) / 2.0))
    r0 = r0 * (1 + 1e-3 * np.sin(x + 2 * y))
    init = dict(rho0=r0, T_u=cfg.T_sat)
    extra = dict(rho_out=W.RHO_L) if bcx == 2 else {}
    d, o = run_pair(L, cfg, 100, init=init, bc_x=bcx, bc_y=bcy, rows=8, **extra)
    e = rel_errors(d.fields(), o.fields())
    print(e)
    tol_u = {(7, 5): 1e-4, (67, 13): 2e-5, (61, 70): 2e-5}.get((nx, ny), TOL)
    assert e["rho"] < TOL and e["T"] < TOL and e["u"] < tol_u, e


@pytest.mark.parametrize("rho_out_frac", [1.0, 0.97])
def test_pressure_outlet_channel_100_steps(L, rho_out_frac):
    """The 200x50 channel with the constant-pressure exit (Sec. 2C) at
    rho_out = rho_l, and at 0.97 rho_l (outflow driven by the exit pressure,
    rho_out differing from the storage reference density)."""
    print(f"case: pressure-exit channel 200x50 rho_out={rho_out_frac} rho_l", flush=True)
    d, o = run_pair(L, W.c1(), 100, bc_x=2, rho_out=rho_out_frac * W.RHO_L)
    e = rel_errors(d.fields(), o.fields())
    print(e)
    assert e["rho"] < TOL and e["T"] < TOL and e["u"] < TOL, e


@pytest.mark.parametrize("bc_x", [0, 1])
def test_random_wall_maps(L, bc_x):
    """Wall temperature and false wall density varying from column to column
    on both walls (ragged 253x37, periodic or channel ends, automatic tile
    rows): the per-column wall values reach the bounce-back, anti-bounce-back
    and adhesion terms of the right nodes, diagonal ones included.  100
    steps, 1e-5 (u at 2e-5 with periodic ends, where the flow decays to
    max |u| ~7.5e-3 and the ~9e-8 absolute error, the FP32 resolution of
    the forces, is 1.2e-5 of it; measured on MI355X)."""
    print(f"case: random wall maps 253x37 bc_x={bc_x}", flush=True)
    rng = np.random.default_rng(17 + bc_x)
    cfg = W.Channel(nx=253, ny=37, heater_len=40)
    d = make_gpu(L, cfg, bc_x=bc_x)
    o = make_oracle(cfg, bc_x=bc_x)
    maps = []
    for side in (0, 1):
        Tw = cfg.T_sat * (1 + 0.1 * rng.uniform(-1, 1, cfg.nx))
        rw = rng.uniform(1.5, 5.5, cfg.nx)
        heat = (rng.uniform(0, 1, cfg.nx) < 0.3).astype(np.int32) if side == 0 else None
        d.set_wall(side, Tw, rw, heat)
        o.set_wall(side, Tw, rw, heat)
        maps.append((Tw, rw))
    d.init(**cfg.init_args())
    o.init(**cfg.init_args())
    d.step(100)
    o.step(100)
    e = rel_errors(d.fields(), o.fields())
    print(e)
    assert e["rho"] < TOL and e["T"] < TOL and e["u"] < (2 * TOL if bc_x == 0 else TOL), e
    gd, od = d.diag(), o.diag()
    assert gd["heater_q"] == pytest.approx(od["heater_q"], rel=1e-5)


def test_isothermal_and_single_phase_flags(L):
    cfg = W.Channel(nx=90, ny=20, heater_len=10)
    for over in (dict(isothermal=1), dict(single_phase=1, fb_x=1e-6, ga_y=0.0),
                 dict(isothermal=1, bc_x=2, rho_out=W.RHO_L)):
        print(f"case: flags {over}", flush=True)
        d, o = run_pair(L, cfg, 50, **over)
        e = rel_errors(d.fields(), o.fields())
        assert e["rho"] < TOL and e["T"] < TOL and e["u"] < TOL, (over, e)


def test_tiling_invariance_bitwise(L):
    """Per-node arithmetic does not depend on the tile shape: fields after 30
    steps are bitwise equal for every rows-per-tile setting, the automatic
    one (None) included; 7, 11 and 15 rows cut the column-edge strips into
    chunks of (rows + 1) / 4, one row more than rows / 4."""
    cfg = W.c1()
    ref = None
    for rows in (4, None, 5, 7, 8, 11, 15, 17, 32, 64):
        print(f"case: c1 rows {rows}", flush=True)
        d = make_gpu(L, cfg, rows=rows)
        d.init(**cfg.init_args())
        d.step(30)
        f = d.fields()
        if ref is None:
            ref = f
        else:
            for k in f:
                assert np.array_equal(f[k], ref[k]), (rows, k)


def test_tiling_invariance_ragged_bitwise(L):
    """The same on a ragged channel (253x37: a partial last strip, uneven row
    chunks) with a periodic variant, automatic and explicit tile heights."""
    for bc_x in (L.BCX_CHANNEL, L.BCX_PERIODIC):
        cfg = W.Channel(nx=253, ny=37, heater_len=14)
        ref = None
        for rows in (None, 5, 6, 7, 11):
            print(f"case: 253x37 bc_x {bc_x} rows {rows}", flush=True)
            d = make_gpu(L, cfg, rows=rows, bc_x=bc_x)
            d.init(**cfg.init_args())
            d.step(30)
            f = d.fields()
            d.close()
            if ref is None:
                ref = f
            else:
                for k in f:
                    assert np.array_equal(f[k], ref[k]), (bc_x, rows, k)


def test_repeatable_and_graph_equals_plain(L):
    """Same run twice is bitwise identical; 75 steps through the replayed
    graphs (single launches first, then graphs of up to 64 launches starting
    at an odd launch phase, or at an even one, then short calls launched
    singly) equal 75 single launches."""
    cfg = W.c1()
    out = []
    for split in ((75,), (1,) * 75, (75,), (1, 33, 9, 32), (64, 11)):
        d = make_gpu(L, cfg)
        d.init(**cfg.init_args())
        for n in split:
            d.step(n)
        out.append(d.fields())
    for k in out[0]:
        for o in out[1:]:
            assert np.array_equal(out[0][k], o[k]), k


def test_long_graphs_equal_plain(L):
    """Calls long enough for the 256-launch replay graph and its repeats
    (700 steps from an odd and from an even step), and batch calls of 600
    steps (from an even and from an odd batch step), equal the same steps in
    calls of 50 single launches, bitwise."""
    cfg = W.c1()
    out = []
    for split in ((1, 700, 300), (2, 700, 299), (1,) + (50,) * 20):
        d = make_gpu(L, cfg)
        d.init(**cfg.init_args())
        for n in split:
            d.step(n)
        assert d.steps == 1001
        out.append(d.fields())
    for k in out[0]:
        for o in out[1:]:
            assert np.array_equal(out[0][k], o[k]), k
    # batch: 601 steps as 600 + 1, 1 + 600 and 1 + 12 calls of 50
    res = []
    for calls in ((600, 1), (1, 600), (1,) + (50,) * 12):
        doms = []
        for c in (W.c1(), W.Channel(nx=130, ny=30, heater_len=10, seed=5)):
            d = make_gpu(L, c)
            d.init(**c.init_args())
            doms.append(d)
        bt = L.Batch(doms)
        for n in calls:
            bt.step(n)
        bt.sync()
        bt.close()
        res.append([d.fields() for d in doms])
    for other in res[1:]:
        for fa, fb in zip(res[0], other):
            for k in fa:
                assert np.array_equal(fa[k], fb[k]), k


def test_checkpoint_resume_bitwise(L, tmp_path):
    cfg = W.c1()
    a = make_gpu(L, cfg)
    a.init(**cfg.init_args())
    a.step(37)
    a.save(str(tmp_path / "ck.bin"))
    a.step(25)
    b = make_gpu(L, cfg)
    b.load(str(tmp_path / "ck.bin"))
    assert b.steps == 37
    b.step(25)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k


def test_checkpoint_across_tilings(L, tmp_path):
    """A checkpoint does not depend on the tiling: saved at 4 rows per tile,
    loaded into a domain at 12 rows, the run continues bitwise like the
    saved one (fields, diagnostics and the per-step records, whose pending
    reductions and the buoyancy's mean cross the change)."""
    cfg = W.c1()
    a = make_gpu(L, cfg, rows=4)
    a.init(**cfg.init_args())
    a.step(37)
    a.save(str(tmp_path / "ck.bin"))
    a.step(25)
    b = make_gpu(L, cfg, rows=12)
    b.load(str(tmp_path / "ck.bin"))
    b.step(25)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    da, db = a.diag(), b.diag()
    assert da == db
    # records restart at the load: the 25 launches record states 35 to 59
    # (state n is recorded during step n + 2)
    ha, hb = a.diag_history()[-25:], b.diag_history()
    assert [r["step"] for r in hb] == list(range(35, 60))
    assert ha == hb


def test_diag_history_records_every_step(L):
    cfg = W.c1()
    d = make_gpu(L, cfg)
    d.init(**cfg.init_args())
    d.step(25)
    h = d.diag_history()
    steps = [r["step"] for r in h]
    assert steps == list(range(0, 23))  # state n is recorded during step n + 2
    o = make_oracle(cfg)
    o.init(**cfg.init_args())
    o.step(10)
    assert h[10]["mass"] == pytest.approx(o.diag()["mass"], rel=1e-6)


def test_batch_equals_solo(L):
    """Uneven domains stepped as one batch give the same fields as each
    stepped alone (bitwise); a batched domain cannot be retiled on its own;
    after the batch the domains (back on their own tile heights, with the
    pending reductions carried over) keep stepping alone like the solo runs."""
    cfgs = [W.Channel(nx=130, ny=30, heater_len=10, seed=5), W.Channel(nx=250, ny=41, heater_len=16, seed=6),
            W.Channel(nx=64, ny=64, heater_len=20, seed=7)]
    solo = []
    for c in cfgs:
        d = make_gpu(L, c)
        d.init(**c.init_args())
        d.step(1)  # odd start: exercises the parity offsets
        d.step(70)
        solo.append(d.fields())
    doms = []
    for c in cfgs:
        d = make_gpu(L, c)
        d.init(**c.init_args())
        d.step(1)
        doms.append(d)
    doms[1].step(0)
    b = L.Batch(doms)
    for call in (lambda: doms[0].set_tile_rows(5), lambda: doms[1].init(**cfgs[1].init_args())):
        with pytest.raises(L.LbmError) as e:
            call()
        assert e.value.code == L.LBM_E_STATE
    b.step(70)  # a first pair, then replay graphs of 64 and 4 launches
    # a read-out of a domain stepped on another stream waits for the batch
    early = doms[2].fields()
    for k in early:
        assert np.array_equal(early[k], solo[2][k]), k
    b.sync()
    b.close()
    for s, d in zip(solo, doms):
        f = d.fields()
        assert d.steps == 71
        for k in f:
            assert np.array_equal(f[k], s[k]), k
    # 25 more steps alone on both sides: fields and diagnostics agree
    for c, d in zip(cfgs, doms):
        ref = make_gpu(L, c)
        ref.init(**c.init_args())
        ref.step(71)
        ref.step(25)
        d.step(25)
        fr, fd = ref.fields(), d.fields()
        for k in fr:
            assert np.array_equal(fr[k], fd[k]), k
        dr, dd = ref.diag(), d.diag()
        assert dr["step"] == dd["step"] and dr["mass"] == dd["mass"] and dr["vapor_cells"] == dd["vapor_cells"]


def test_batch_member_matches_oracle(L):
    """A domain stepped inside a batch of uneven domains (as the ensemble and
    the serving loop run them) against the oracle: the middle member of
    three, 100 steps from an odd start, 1e-5."""
    cfgs = [W.Channel(nx=130, ny=30, heater_len=10, seed=5), W.Channel(nx=250, ny=41, heater_len=16, seed=6),
            W.Channel(nx=64, ny=64, heater_len=20, seed=7)]
    print("case: batch member 250x41 vs oracle, 101 steps", flush=True)
    doms = []
    for c in cfgs:
        d = make_gpu(L, c)
        d.init(**c.init_args())
        d.step(1)
        doms.append(d)
    b = L.Batch(doms)
    b.step(100)
    b.sync()
    b.close()
    o = make_oracle(cfgs[1])
    o.init(**cfgs[1].init_args())
    o.step(101)
    e = rel_errors(doms[1].fields(), o.fields())
    print(e)
    assert e["rho"] < TOL and e["T"] < TOL and e["u"] < TOL, e


def test_channel_1600x200_parity(L):
    """Full single-instance size, 100 steps (the same launch configuration as
    the benchmark), compared on every node."""
    cfg = W.c2()
    print("case: channel 1600x200 100 steps", flush=True)
    d, o = run_pair(L, cfg, 100)
    e = rel_errors(d.fields(), o.fields())
    print(e)
    assert e["rho"] < TOL and e["T"] < TOL and e["u"] < TOL, e


def test_hbm_resident_channel_parity(L):
    """The 8192x1024 channel of the HBM measurement (18 574 tiles, about nine
    rounds of resident waves, every XCD with a long contiguous tile run), 6
    steps against the oracle on every node."""
    cfg = W.roofline_channel()
    print("case: channel 8192x1024 6 steps", flush=True)
    d, o = run_pair(L, cfg, 6)
    e = rel_errors(d.fields(), o.fields())
    print(e, flush=True)
    assert e["rho"] < TOL and e["T"] < TOL and e["u"] < TOL, e


def test_near_maximum_size_parity(L):
    """8192 x 2880 FP32 thermal channel (23.6 M nodes): the 9-plane state,
    with the two-plane base shift of the boundary pulls, sits just under the
    2 GB reach of 32-bit byte offsets (the limit lbm_create enforces).  3
    steps against the oracle on every node."""
    import psutil

    if psutil.virtual_memory().available < 24 * 2**30:
        pytest.skip("needs ~12 GB of host memory for the oracle")
    cfg = W.Channel(nx=8192, ny=2880, heater_len=1150, steps=3)
    p = L.default_params(storage=L.STORE_F32_DEV, rho_ref=W.RHO_L, T_ref=cfg.T_sat, **cfg.params())
    assert 11 * 8192 * (2880 + 2) * 8 > 0.95 * (2**31 - 2**24)  # within 5 % of the limit
    assert L.required_bytes(p) > 0
    print("case: channel 8192x2880 3 steps", flush=True)
    d, o = run_pair(L, cfg, 3)
    e = rel_errors(d.fields(), o.fields())
    print(e, flush=True)
    assert e["rho"] < TOL and e["T"] < TOL and e["u"] < TOL, e


@pytest.mark.parametrize("storage,tol", [("F16_DEV", 3e-3), ("BF16_DEV", 3e-2)])
def test_half_precision_storage_error(L, storage, tol):
    """Precision study: FP16/BF16 deviation storage against the FP64 oracle
    after 100 steps; the bound is the measured error with margin (reported,
    not a parity claim)."""
    st = getattr(L, "STORE_" + storage)
    d, o = run_pair(L, W.c1(), 100, storage=st)
    e = rel_errors(d.fields(), o.fields())
    print(storage, e)
    assert max(e.values()) < tol, e


def test_pressure_exit_paper_cross_section_long_run(L):
    """The paper's channel cross-section (40 rows, Re_in = 0.96, T_in =
    0.9 Tc, exit density rho_l) on 40 x 250 with the constant-pressure exit,
    20000 steps unheated: the GPU stays bounded with the oracle and matches
    it to the 100-step tolerance (steady laminar flow with wall-adhesion
    layers; measured 3e-7 on rho and T, 4e-6 on u)."""
    from oracle import oracle as O

    Tc = W.TC
    Tin = 0.9 * Tc
    rl, rv, _ = O.maxwell(Tin)
    nx, ny = 250, 40
    kw = dict(nx=nx, ny=ny, bc_x=2, bc_y=1, rho_out=rl, u_in=0.96 / 6.0 / ny, T_in=Tin, T_iso=Tin,
              rho_mid=0.5 * (rl + rv), ga_y=-5e-5, tau_f=1.0, tau_g=0.6, c_v=6.0, omega=0.344)
    rw = rv + 0.6 * (rl - rv)
    print("case: pressure exit 40x250, 20000 steps", flush=True)
    d = L.Domain(L.default_params(storage=L.STORE_F32_DEV, rho_ref=rl, T_ref=Tin, **kw))
    o = O.Oracle(O.Params(**kw))
    for side in (0, 1):
        d.set_wall(side, np.full(nx, Tin), np.full(nx, rw))
        o.set_wall(side, np.full(nx, Tin), np.full(nx, rw))
    ia = dict(rho_u=rl, T_u=Tin, noise=1e-3, seed=11)
    d.init(**ia)
    o.init(**ia)
    d.step(20000)
    o.step(20000)
    g, r = d.fields(), o.fields()
    assert np.isfinite(g["rho"]).all() and np.isfinite(g["T"]).all()
    e = rel_errors(g, r)
    print(e, flush=True)
    assert e["rho"] < TOL and e["T"] < TOL and e["u"] < TOL, e


def test_heated_paper_channel(L):
    """The paper's channel (Sec. 2C): 40 x 1000, constant-pressure exit at
    rho_l, T_in = T_sat = 0.9 Tc, Re_in = 0.96, 10 000 unheated steps, then a
    5-node heater at L/5 switched on at 1.2 Tc through the wall maps, 3000
    heated steps: GPU against the oracle at 1e-5 on every node (the heated
    spot on the wall -- a near-critical low-density region of ~11 nodes --
    forms in this window)."""
    from oracle import oracle as O

    Tc = W.TC
    Tin = 0.9 * Tc
    rl, rv, _ = O.maxwell(Tin)
    nx, ny = 1000, 40
    kw = dict(nx=nx, ny=ny, bc_x=2, bc_y=1, rho_out=rl, u_in=0.96 / 6.0 / ny, T_in=Tin, T_iso=Tin,
              rho_mid=0.5 * (rl + rv), ga_y=-5e-5, tau_f=1.0, tau_g=0.6, c_v=6.0, omega=0.344)
    rw = rv + 0.6 * (rl - rv)
    heater = np.zeros(nx, np.int32)
    heater[nx // 5 - 2: nx // 5 + 3] = 1
    print("case: paper channel 40x1000, 10000 + 3000 heated steps", flush=True)
    d = L.Domain(L.default_params(storage=L.STORE_F32_DEV, rho_ref=rl, T_ref=Tin, **kw))
    o = O.Oracle(O.Params(**kw))
    for side in (0, 1):
        d.set_wall(side, np.full(nx, Tin), np.full(nx, rw))
        o.set_wall(side, np.full(nx, Tin), np.full(nx, rw))
    ia = dict(rho_u=rl, T_u=Tin, noise=1e-3, seed=11)
    d.init(**ia)
    o.init(**ia)
    d.step(10000)
    o.step(10000)
    Th = np.where(heater == 1, 1.2 * Tc, Tin)
    d.set_wall(L.SIDE_S, Th, np.full(nx, rw), heater)
    o.set_wall(0, Th, np.full(nx, rw), heater)
    d.step(3000)
    o.step(3000)
    g, r = d.fields(), o.fields()
    assert np.isfinite(g["rho"]).all() and r["rho"].min() < 3.0  # the heated spot is there
    e = rel_errors(g, r)
    print(e, flush=True)
    assert e["rho"] < TOL and e["T"] < TOL and e["u"] < TOL, e
    gd, od = d.diag(), o.diag()
    assert gd["heater_q"] == pytest.approx(od["heater_q"], rel=1e-4)


def test_autotuner_and_cache(L, tmp_path):
    """The batch autotuner times rows-per-tile x grid configurations with real
    steps and writes its choice to the cache; the tuned batch still equals
    the domains stepped alone (bitwise), and a second batch of the same shape
    reads the cache instead of tuning."""
    cfgs = [W.Channel(nx=130, ny=30, heater_len=10, seed=5), W.Channel(nx=250, ny=41, heater_len=16, seed=6)]
    cache = tmp_path / "tune.txt"

    def fresh():
        out = []
        for c in cfgs:
            d = make_gpu(L, c)
            d.init(**c.init_args())
            out.append(d)
        return out

    print("case: autotuner with cache file", flush=True)
    doms = fresh()
    b = L.Batch(doms, tune_cache=str(cache))
    tuned = doms[0].steps
    assert tuned > 0 and all(d.steps == tuned for d in doms)  # tuning steps are real steps
    b.step(40)
    b.sync()
    b.close()
    lines = cache.read_text().split()
    assert len(lines) == 3 and lines[0].startswith("v2_n2_")
    # the autotuner's options (rows 4, 6, 7, 8, 12; grids 0, 8, 16 per CU),
    # as documented at lbm_batch_create
    assert int(lines[1]) in (4, 6, 7, 8, 12) and int(lines[2]) in (0, 8, 16)
    for c, d in zip(cfgs, doms):
        s = make_gpu(L, c)
        s.init(**c.init_args())
        s.step(tuned + 40)
        fs, fd = s.fields(), d.fields()
        for k in fs:
            assert np.array_equal(fs[k], fd[k]), k
    doms2 = fresh()
    b2 = L.Batch(doms2, tune_cache=str(cache))
    assert all(d.steps == 0 for d in doms2)  # read from the cache, no tuning steps
    b2.step(10)
    b2.sync()
    b2.close()
    assert cache.read_text().split() == lines


def test_caller_memory_and_device_readout(L):
    """A domain in caller-supplied device memory steps bitwise like one the
    library allocates; the device read-out writes the same float32 fields
    into caller tensors; a buffer below lbm_required_bytes is rejected."""
    import torch

    cfg = W.Channel(nx=130, ny=30, heater_len=10, seed=9)
    p = L.default_params(storage=L.STORE_F32_DEV, rho_ref=W.RHO_L, T_ref=cfg.T_sat, **cfg.params())
    need = L.required_bytes(p)
    print(f"case: caller memory {need} bytes", flush=True)
    with pytest.raises(L.LbmError) as e:
        L.Domain(p, device_buffer=torch.empty(need - 256, dtype=torch.uint8, device="cuda"))
    assert e.value.code == L.LBM_E_INVALID
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    outs = []
    for dev in (buf, None):
        d = L.Domain(p, device_buffer=dev)
        Ts, rws, heat, Tn, rwn = cfg.walls()
        d.set_wall(L.SIDE_S, Ts, rws, heat)
        d.set_wall(L.SIDE_N, Tn, rwn)
        d.init(**cfg.init_args())
        d.step(50)
        outs.append((d, d.fields()))
    for k in outs[0][1]:
        assert np.array_equal(outs[0][1][k], outs[1][1][k]), k
    d, f = outs[1]
    t = {k: torch.full((cfg.ny, cfg.nx), float("nan"), dtype=torch.float32, device="cuda")
         for k in ("rho", "ux", "uy", "T")}
    d.fields_device(t["rho"], t["ux"], t["uy"], t["T"])
    torch.cuda.synchronize()
    for k in t:
        assert np.array_equal(t[k].cpu().numpy().astype(np.float64), f[k]), k
    for dd, _ in outs:
        dd.close()
