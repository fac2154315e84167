"""Time of one right-hand side on one GPU: nse_rhs (explicit second-order
viscous terms, the paper's scheme) against nse_rhs_compact_viscous (viscous
terms by the compact first derivative: 24 extra derivative launches and three
point-wise kernels), and one RK4 step of rk_step against rk_step_compact_viscous.

Workload (seeded, synthetic): the RTI box of the RK benchmark, 512^3 points,
4 segments per direction.  HIP events on the launch stream over `reps` calls
after one untimed call of each.  Prints one JSON line.

    python -m paper_2203_00879_amd.rhs_variant_bench [--n 512] [--nseg 4] [--reps 5]
"""
import argparse
import json
import os
import sys

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    __package__ = "paper_2203_00879_amd"

from . import inputs, nopcs  # noqa: E402


def run(n=512, nseg=4, reps=5):
    import torch
    p = nopcs.make_params(inputs.AIR)
    g = nopcs.make_grid(n, nseg)
    Q = torch.from_numpy(inputs.rti_state(n, seed=0)).to("cuda")
    R = torch.empty_like(Q)
    ws = torch.empty(nopcs.compact_viscous_workspace_bytes(g), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    out = {"metric": "right-hand side time (RTI box %d^3, %d segments/direction, FP64)" % (n, nseg),
           "points": n ** 3, "reps": reps}
    for name, fn in (("explicit_viscous", nopcs.nse_rhs), ("compact_viscous", nopcs.nse_rhs_compact_viscous)):
        fn(p, g, Q, R, ws=ws, stream=stream)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        for _ in range(reps):
            fn(p, g, Q, R, ws=ws, stream=stream)
        e.record(stream)
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        out[name] = {"ms": ms, "Mpoint_per_s": n ** 3 / (ms * 1e-3) / 1e6, "finite": bool(torch.isfinite(R).all())}
    # one RK4 step of each (dt = 1e-6), after one untimed step
    for name, fn in (("rk_step_explicit_viscous", lambda: nopcs.rk_step(p, g, Q, 1e-6, 1, ws, stream=stream)),
                     ("rk_step_compact_viscous",
                      lambda: nopcs.rk_step_compact_viscous(p, g, Q, 1e-6, 1, ws, stream=stream))):
        fn()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        for _ in range(reps):
            fn()
        e.record(stream)
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        out[name] = {"ms_per_step": ms, "Mpoint_stage_per_s": 4 * n ** 3 / (ms * 1e-3) / 1e6,
                     "finite": bool(torch.isfinite(Q).all())}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--nseg", type=int, default=4)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    print(json.dumps(run(a.n, a.nseg, a.reps)), flush=True)


if __name__ == "__main__":
    main()
