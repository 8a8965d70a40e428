"""CPU-side checks of the boundary: the shared library loads and exports every
entry point that include/lbmflow.h declares, the parameter struct matches
the binding, and the seeded inputs agree with the oracle (no GPU calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmflow.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def so():
    from paper_2009_05264_amd import build_lib

    if build_lib.stale():
        build_lib.build()
    return C.CDLL(build_lib.LIB)


def test_every_declared_symbol_is_exported(so):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(so, n), n


def test_binding_struct_sizes():
    from paper_2009_05264_amd import lbmflow as L

    txt = open(HEADER).read()
    assert C.sizeof(L.Params) == 8 * 4 + 26 * 8
    assert C.sizeof(L.Diag) == 8 + 10 * 8
    assert "double rho_ref, T_ref;" in txt
    # rho_out, then G_wet, close lbm_params
    assert txt.index("double rho_out;") > txt.index("double rho_ref, T_ref;")
    assert txt.index("double rho_out;") < txt.index("double G_wet;") < txt.index("} lbm_params;")
    assert [f[0] for f in L.Params._fields_][-2:] == ["rho_out", "G_wet"]


def test_default_G_wet_is_neutral(oracle_mod):
    """The library's default adhesion strength (Eq. 15) equals the oracle's
    neutral value, and follows beta and g when they change."""
    from paper_2009_05264_amd import lbmflow as L

    O = oracle_mod
    assert L.default_params().G_wet == pytest.approx(O.Params().neutral_G_wet, rel=1e-15)
    p = L.default_params(beta=1.3, g=-2.0)
    assert p.G_wet == pytest.approx(O.Params(beta=1.3, g=-2.0).neutral_G_wet, rel=1e-15)
    assert L.default_params(G_wet=-7.0).G_wet == -7.0


def test_binding_names_match_header():
    from paper_2009_05264_amd import lbmflow as L
    import inspect

    src = inspect.getsource(L)
    for n in declared_functions():
        assert f'"{n}"' in src, n


def test_workload_constants_match_oracle(oracle_mod):
    import workloads as W

    O = oracle_mod
    assert W.TC == pytest.approx(O.crit_temperature(), rel=1e-15)
    rl, rv, _ = O.maxwell(W.TSAT_FRAC * W.TC, omega=0.344)
    assert W.RHO_L == pytest.approx(rl, rel=1e-9)
    assert W.RHO_V == pytest.approx(rv, rel=1e-9)
    rl, rv, _ = O.maxwell(0.9 * W.TC, omega=0.32)
    assert W.RHO_L_POOL == pytest.approx(rl, rel=1e-9)
    assert W.RHO_V_POOL == pytest.approx(rv, rel=1e-9)


def test_ensemble_is_seeded():
    import workloads as W

    a, b = W.ensemble(), W.ensemble()
    assert [(c.nx, c.ny, c.u_in) for c in a] == [(c.nx, c.ny, c.u_in) for c in b]
    assert len(a) == 64 and {c.nx for c in a} <= {400, 800, 1200, 1600} and {c.ny for c in a} <= {50, 100, 200}


def test_server_structs_match_header():
    from paper_2009_05264_amd import lbmflow as L

    assert C.sizeof(L.Request) == 5 * 8 + 3 * 8 + 8
    assert C.sizeof(L.ServerInfo) == 3 * 8 + 2 * 8 + 2 * 8 + 8
    txt = open(HEADER).read()
    for st in ("LBM_REQ_QUEUED = 0", "LBM_REQ_RUNNING = 1", "LBM_REQ_DONE = 2", "LBM_REQ_CANCELLED = 3",
               "LBM_REQ_FAILED = 4"):
        assert st in txt, st


def test_admission_in_arrival_order_by_footprint():
    """First fit in arrival order: a request that does not fit is passed
    over without blocking smaller ones behind it; slots bound the count."""
    from paper_2009_05264_amd import lbmflow as L

    assert L.admission_plan([5, 3, 8, 1, 2], cap=10, used=0, free_slots=3) == [0, 1, 3]
    assert L.admission_plan([5, 3, 8, 1, 2], cap=10, used=0, free_slots=10) == [0, 1, 3]
    assert L.admission_plan([5, 3, 8, 1, 2], cap=10, used=4, free_slots=10) == [0, 3]
    assert L.admission_plan([10], cap=10, used=0, free_slots=1) == [0]  # exact fit
    assert L.admission_plan([1, 1], cap=10, used=11, free_slots=5) == []  # already over the cap
    assert L.admission_plan([1, 1, 1], cap=10, used=0, free_slots=0) == []
    assert L.admission_plan([], cap=10, used=0, free_slots=3) == []
    # never exceeds the cap, whatever the order
    rng = np.random.default_rng(0)
    for _ in range(200):
        fp = rng.integers(1, 50, size=20)
        cap, used = 100, int(rng.integers(0, 60))
        adm = L.admission_plan(list(fp), cap=cap, used=used, free_slots=int(rng.integers(0, 20)))
        assert used + sum(fp[i] for i in adm) <= cap
        assert adm == sorted(adm)
        # every passed-over request before the last admitted one did not fit at its turn
        tot = used
        for i in range(max(adm) + 1 if adm else 0):
            if i in adm:
                tot += fp[i]
            else:
                assert tot + fp[i] > cap


def test_admission_plan_rejects_bad_arguments():
    from paper_2009_05264_amd import lbmflow as L

    lib = L.lib()
    na = C.c_int()
    assert lib.lbm_admission_plan(None, -1, 10, 0, 1, None, C.byref(na)) == L.LBM_E_INVALID
    assert lib.lbm_admission_plan(None, 2, 10, 0, 1, None, C.byref(na)) == L.LBM_E_INVALID


def test_parameter_validation():
    """lbm_required_bytes validates parameters on the host (no GPU call)."""
    from paper_2009_05264_amd import lbmflow as L

    ok = L.default_params()
    assert L.required_bytes(ok) > 0
    bad = [dict(nx=2), dict(ny=2), dict(tau_f=0.5), dict(tau_g=0.4), dict(c_v=0.0), dict(u_in=0.2),
           dict(T_in=0.0), dict(storage=7), dict(bc_x=5), dict(a=0.0), dict(s_q=2.5),
           dict(bc_x=L.BCX_CHANNEL_P, rho_out=0.0),
           dict(nx=16384, ny=2048, storage=L.STORE_F32_DEV)]  # beyond 32-bit state offsets
    for kw in bad:
        with pytest.raises(L.LbmError) as e:
            L.required_bytes(L.default_params(**kw))
        assert e.value.code == L.LBM_E_INVALID, kw
    assert L.required_bytes(L.default_params(bc_x=L.BCX_CHANNEL_P)) > 0  # default rho_out = rho_l
    # the same size fits with half-precision storage or isothermal FP32
    assert L.required_bytes(L.default_params(nx=16384, ny=2048, storage=L.STORE_F16_DEV)) > 0
    assert L.required_bytes(L.default_params(nx=16384, ny=2048, storage=L.STORE_F32_DEV, isothermal=1)) > 0


def test_required_bytes_scale_with_storage():
    from paper_2009_05264_amd import lbmflow as L

    b32 = L.required_bytes(L.default_params(nx=1024, ny=512, storage=L.STORE_F32_DEV))
    b16 = L.required_bytes(L.default_params(nx=1024, ny=512, storage=L.STORE_F16_DEV))
    state32 = 2 * 9 * 1024 * 512 * 8  # A/B, 9 planes of (f, g) pairs
    assert state32 <= b32 < state32 * 1.25
    assert b16 < b32 and b32 - b16 >= state32 // 2 * 0.99


def _build_c_example(out):
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    pkg = os.path.join(os.path.dirname(HEADER), "..", "paper_2009_05264_amd")
    src = os.path.join(pkg, "examples", "channel.c")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Werror", src, "-I", os.path.dirname(HEADER), "-L", pkg,
           "-llbmflow", "-Wl,-rpath," + os.path.abspath(pkg), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


def test_c_example_builds_against_the_header(tmp_path):
    """The C example uses only include/lbmflow.h and links against the library."""
    assert os.path.exists(_build_c_example(tmp_path / "channel"))


def test_library_maxwell_matches_oracle():
    """lbm_maxwell (host, in the library) against the oracle's independent
    equal-area construction, 0.6-0.95 Tc, both acentric factors used here."""
    import workloads as W
    from oracle import oracle as O
    from paper_2009_05264_amd import lbmflow as L

    for omega in (0.344, 0.32):
        p = L.default_params(omega=omega)
        for frac in (0.6, 0.7, 0.8, 0.86, 0.9, 0.95):
            T = frac * W.TC
            rl, rv, ps = L.maxwell(p, T)
            ol, ov, ops = O.maxwell(T, omega=omega)
            assert rl == pytest.approx(ol, rel=1e-8) and rv == pytest.approx(ov, rel=1e-8)
            assert ps == pytest.approx(ops, rel=1e-8)
