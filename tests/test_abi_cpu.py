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
    assert C.sizeof(L.Params) == 8 * 4 + 24 * 8
    assert C.sizeof(L.Diag) == 8 + 8 * 8
    assert "double rho_ref, T_ref;" in txt


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


def test_ensemble_is_seeded():
    import workloads as W

    a, b = W.ensemble(), W.ensemble()
    assert [(c.nx, c.ny, c.u_in) for c in a] == [(c.nx, c.ny, c.u_in) for c in b]
    assert len(a) == 64 and {c.nx for c in a} <= {400, 800, 1200, 1600} and {c.ny for c in a} <= {50, 100, 200}
