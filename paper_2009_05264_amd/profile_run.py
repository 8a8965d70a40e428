"""Profiling driver for rocprofv3.

Runs a fixed number of time steps of one synthetic flow-boiling channel on
cuda:0 (one step kernel launch per step, no graph), then a device copy of a
known byte count through the library's copy kernel.  The copy is the
calibration of the FETCH_SIZE / WRITE_SIZE counters: bytes moved by the copy
divided by what the counters read for it gives the scale applied to the step
kernel's readings.

    rocprofv3 --kernel-trace --stats -- python3 paper_2009_05264_amd/profile_run.py
    rocprofv3 --pmc FETCH_SIZE -- python3 paper_2009_05264_amd/profile_run.py
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="channel_1600x200",
                    choices=["channel_1600x200", "channel_8192x1024"])
    ap.add_argument("--storage", default="F32_DEV", choices=["F32", "F32_DEV", "F16_DEV", "BF16_DEV"])
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args()

    import torch

    import workloads as W
    from paper_2009_05264_amd import lbmflow as L

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    ts = torch.cuda.Stream()
    torch.cuda.set_stream(ts)
    cfg = W.c2() if args.workload == "channel_1600x200" else W.roofline_channel()
    st = getattr(L, "STORE_" + args.storage)
    ref = dict(rho_ref=W.RHO_L, T_ref=cfg.T_sat) if st != L.STORE_F32 else {}
    d = L.Domain(L.default_params(storage=st, **ref, **cfg.params()), stream=ts.cuda_stream)
    Ts, rws, heat, Tn, rwn = cfg.walls()
    d.set_wall(L.SIDE_S, Ts, rws, heat)
    d.set_wall(L.SIDE_N, Tn, rwn)
    d.init(**cfg.init_args())
    for _ in range(args.steps):
        d.step(1)  # single launches: one kernel record per step
    d.sync()
    print(f"workload {args.workload} storage {args.storage}: {args.steps} steps", flush=True)
    d.close()

    n = args.copy_mib << 20
    a = torch.zeros(n // 4, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    for _ in range(3):
        L.stream_copy(c.data_ptr(), a.data_ptr(), n, ts.cuda_stream)
    torch.cuda.synchronize()
    print(f"copy: 3 x {n} bytes read + {n} bytes written", flush=True)


if __name__ == "__main__":
    main()
