"""Throughput of the vorticity budget (nopcs_vorticity_budget, Eq. eqn12_1) on
one GPU.

Workload (seeded, synthetic): the RTI box of the RK benchmark, 512^3 points, 4
segments per direction, a few steps after the partition is removed (so that
velocity, vorticity and every source term are non-zero).  Algorithmic bytes per
point: primitives 72 (read rho, rho u, rho v, rho w, E'; write u, v, w, p'),
15 first derivatives 240 (read a field, write its gradient component),
combination 224 (read 15 gradients and rho, write 12 outputs): 536 in all.
Timed with HIP events on the launch stream over `reps` calls after one untimed
call; the derivative share comes from the library's own per-kernel timing.

Prints one JSON line.

    python -m paper_2203_00879_amd.vort_bench [--n 512] [--nseg 4] [--reps 5]
"""
import argparse
import ctypes
import json
import os
import sys

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    __package__ = "paper_2203_00879_amd"

from . import inputs, nopcs  # noqa: E402

HBM_PEAK_GBS = 8000.0
BYTES_PER_POINT = 536
DERIV_BYTES_PER_POINT = 16      # one first derivative: read f, write f'
K_DERIV = 5                     # NOPCS_K_DERIV
K_VORT = 9                      # NOPCS_K_VORT


def run(n=512, nseg=4, reps=5, steps=4, dt=1e-5):
    import torch
    p = nopcs.make_params(inputs.AIR)
    g = nopcs.make_grid(n, nseg)
    Q = torch.from_numpy(inputs.rti_state(n, seed=0)).to("cuda")
    ws = nopcs.alloc_workspace(g)
    nopcs.rk_step(p, g, Q, dt, steps, ws)
    del ws
    out = torch.empty((12,) + tuple(Q.shape[1:]), dtype=torch.float64, device="cuda")
    vws = torch.empty(nopcs.vorticity_workspace_bytes(g), dtype=torch.uint8, device="cuda")
    nopcs.vorticity_budget(p, g, Q, out, vws)
    torch.cuda.synchronize()
    lib = nopcs.lib()
    lib.nopcs_timing_enable.argtypes = [ctypes.c_int]
    lib.nopcs_timing_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    stream = torch.cuda.current_stream()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(stream)
    for _ in range(reps):
        nopcs.vorticity_budget(p, g, Q, out, vws, stream=stream)
    e.record(stream)
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    # per-kernel split in a second pass (the timing events serialise launches)
    lib.nopcs_timing_enable(1)
    for _ in range(reps):
        nopcs.vorticity_budget(p, g, Q, out, vws, stream=stream)
    torch.cuda.synchronize()
    tot, cnt = ctypes.c_double(), ctypes.c_int64()
    nopcs._check(lib.nopcs_timing_read(K_DERIV, ctypes.byref(tot), ctypes.byref(cnt)))
    vtot, vcnt = ctypes.c_double(), ctypes.c_int64()
    nopcs._check(lib.nopcs_timing_read(K_VORT, ctypes.byref(vtot), ctypes.byref(vcnt)))
    lib.nopcs_timing_enable(0)
    N = n ** 3
    deriv_ms = tot.value / max(cnt.value, 1)
    gbs = BYTES_PER_POINT * N / (ms * 1e-3) / 1e9
    return {"metric": "vorticity budget throughput (RTI box %d^3, %d segments/direction, FP64)" % (n, nseg),
            "points": N, "reps": reps, "ms": ms, "Gpoint_per_s": N / (ms * 1e-3) / 1e9,
            "alg_bytes_per_point": BYTES_PER_POINT, "alg_GBps": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
            "derivative_launches": int(cnt.value), "derivative_ms_mean": deriv_ms,
            "derivative_alg_GBps": DERIV_BYTES_PER_POINT * N / (deriv_ms * 1e-3) / 1e9,
            "pointwise_ms_per_call": vtot.value / reps, "derivative_ms_per_call": tot.value / reps,
            "max_abs": {"omega": float(out[0:3].abs().max()), "stretching": float(out[3:6].abs().max()),
                        "dilatation": float(out[6:9].abs().max()), "baroclinic": float(out[9:12].abs().max())}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--nseg", type=int, default=4)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    print(json.dumps(run(a.n, a.nseg, a.reps)), flush=True)


if __name__ == "__main__":
    main()
