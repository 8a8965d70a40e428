"""The C example (paper_2009_05264_amd/examples/channel.c) runs on the GPU
through the C ABI alone and prints the same diagnostics as the same channel
stepped through the Python binding (one library, bitwise-equal steps)."""
import os
import re
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_c_example_matches_binding(tmp_path):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from test_abi_cpu import _build_c_example

    exe = _build_c_example(tmp_path / "channel")
    print("case: C example, 200x50 channel, 2000 steps", flush=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    m = re.search(r"step (\d+): mass ([\d.eE+-]+) energy ([\d.eE+-]+) heater flux ([\d.eE+-]+) vapour cells (\d+)",
                  out.stdout)
    assert m, out.stdout
    step, mass, energy = int(m.group(1)), float(m.group(2)), float(m.group(3))
    assert step == 2000

    from paper_2009_05264_amd import lbmflow as L

    p = L.default_params()
    rl, rv, _ = L.maxwell(p, p.T_iso)
    p = L.default_params(storage=L.STORE_F32_DEV, rho_ref=rl, T_ref=p.T_iso)
    d = L.Domain(p)
    heat = np.zeros(p.nx, np.int32)
    heat[p.nx // 2 - 10: p.nx // 2 + 10] = 1
    d.set_wall(L.SIDE_S, np.where(heat == 1, 1.1 * p.T_iso, p.T_in), 3.8, heat)
    d.set_wall(L.SIDE_N, p.T_in, 3.8)
    d.init(rho_u=rl, T_u=p.T_iso, noise=1e-3, seed=1)
    d.step(2000)
    g = d.diag()
    d.close()
    assert g["step"] == 2000
    assert mass == pytest.approx(g["mass"], rel=1e-6) and energy == pytest.approx(g["energy"], rel=1e-6)
