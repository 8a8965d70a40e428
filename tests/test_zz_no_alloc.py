"""The allocation-free initialisation (lbm_init_fields_noalloc) against
lbm_init_fields: called through the C ABI on two domains in a row (the
second smaller), with density and temperature arrays, the resulting run
equals the allocating entry point's bitwise; sizes beyond the fixed staging
array are refused with LBM_E_INVALID."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _domain(L, cfg):
    p = L.default_params(storage=L.STORE_F32_DEV, rho_ref=W.RHO_L, T_ref=cfg.T_sat, **cfg.params())
    d = L.Domain(p)
    Ts, rws, heat, Tn, rwn = cfg.walls()
    d.set_wall(L.SIDE_S, Ts, rws, heat)
    d.set_wall(L.SIDE_N, Tn, rwn)
    return d


def test_noalloc_init_matches_allocating_init():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05264_amd import lbmflow as L

    lib = L.lib()
    rng = np.random.default_rng(21)
    for cfg in (W.Channel(nx=300, ny=60, heater_len=24, seed=3), W.Channel(nx=67, ny=13, heater_len=5, seed=4)):
        print(f"case: no-alloc init {cfg.nx}x{cfg.ny}", flush=True)
        rho0 = np.ascontiguousarray(W.RHO_L * (1 + 1e-3 * rng.uniform(-1, 1, (cfg.ny, cfg.nx))))
        rho0[cfg.ny // 3: cfg.ny // 2, cfg.nx // 3: cfg.nx // 2] = W.RHO_V
        T0 = np.ascontiguousarray(cfg.T_sat * (1 + 1e-2 * rng.uniform(-1, 1, (cfg.ny, cfg.nx))))
        out = []
        for fn in (lib.lbm_init_fields, lib.lbm_init_fields_noalloc):
            d = _domain(L, cfg)
            rc = fn(d.h, _dp(rho0), _dp(T0), C.c_double(1.0), C.c_double(1.0), C.c_double(0.0), C.c_uint64(0))
            assert rc == L.LBM_OK, lib.lbm_last_error().decode()
            d.step(25)
            out.append((d.fields(), d.diag()))
            d.close()
        (fa, da), (fb, db) = out
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), k
        assert da == db
    # uniform initial states need no staging; arrays beyond the limit are refused
    big = W.Channel(nx=1100, ny=1000, heater_len=400)
    d = _domain(L, big)
    assert 1100 * 1000 > L.NOALLOC_MAX_NODES
    arr = np.full((1000, 1100), W.RHO_L)
    rc = lib.lbm_init_fields_noalloc(d.h, _dp(arr), None, C.c_double(1.0), C.c_double(big.T_sat), C.c_double(0.0),
                                     C.c_uint64(0))
    assert rc == L.LBM_E_INVALID and "staging" in lib.lbm_last_error().decode()
    rc = lib.lbm_init_fields_noalloc(d.h, None, None, C.c_double(W.RHO_L), C.c_double(big.T_sat),
                                     C.c_double(1e-3), C.c_uint64(1))
    assert rc == L.LBM_OK
    d.close()
