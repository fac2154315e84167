"""RK4 stepping on the paper's own box shape at the largest single-GPU scale.

The paper's run (Section 4): a cube of edge L with 1280 points along x and z
and 2560 along y (h_y = h_x / 2), 20 x 48 x 20 sub-domains (segments of 64
points along x, z and 2560/48 = 53.3 along y, uneven), 100 K air over 300 K
air, dt* = 7.69e-8 s.  Here: 512 x 1024 x 512 points (2.7e8, a sixteenth of
the paper's), 8 x 19 x 8 segments (64 points along x, z; 53.9 along y, uneven),
the same temperatures and the same time step in units of sqrt(L/g).  Seeded
synthetic interface noise as in the RK benchmark.  HIP events on the launch
stream around `steps` steps after `warmup` untimed steps.  Prints one JSON line.

    python -m paper_2203_00879_amd.paper_setup_bench [--n 512] [--steps 10] [--precision fp64|mixed]
"""
import argparse
import json
import math
import os
import sys

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    __package__ = "paper_2203_00879_amd"

from . import inputs, nopcs  # noqa: E402


def run(n=512, steps=10, warmup=2, precision="fp64"):
    import torch
    shape = (n, 2 * n, n)
    nseg = (max(1, n // 64), max(1, round(2 * n / 53.3)), max(1, n // 64))
    p = dict(inputs.AIR)
    ts = math.sqrt(p["L"] / p["g"])
    dt = 7.69e-8 / ts
    g = nopcs.make_grid(shape, nseg)
    prm = nopcs.make_params(p)
    Q = torch.from_numpy(inputs.rti_state(shape, T_upper=100.0, T_lower=300.0, seed=0)).to("cuda")
    prec = nopcs.MIXED if precision == "mixed" else nopcs.FP64
    ws = nopcs.alloc_workspace(g, prec)
    stream = torch.cuda.current_stream()
    nopcs.rk_step(prm, g, Q, dt, warmup, ws, precision=prec, stream=stream)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(stream)
    nopcs.rk_step(prm, g, Q, dt, steps, ws, precision=prec, stream=stream)
    e.record(stream)
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / steps
    N = shape[0] * shape[1] * shape[2]
    return {"metric": "Mpoint-stage updates/s (paper box shape %dx%dx%d, %s)" % (shape + (precision,)),
            "shape_xyz": shape, "segments_xyz": nseg, "points": N, "dt": dt, "steps": steps,
            "ms_per_step": ms, "Mpoint_stage_per_s": 4 * N / (ms * 1e-3) / 1e6,
            "finite": bool(torch.isfinite(Q).all())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    a = ap.parse_args()
    print(json.dumps(run(a.n, a.steps, a.warmup, a.precision)), flush=True)


if __name__ == "__main__":
    main()
