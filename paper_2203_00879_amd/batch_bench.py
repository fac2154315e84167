"""Throughput of RK4 stepping for a batch of uneven boxes on one GPU: the boxes
one after the other on one stream (rk_step, direct launches) against
rk_step_batch in its four modes -- one launch per stage kernel over all boxes
as a graph (0) or issued directly (2), one graph branch per box (1), and
branches for boxes of 2^21 points or more beside shared launches for the
others (3, the default).

Workloads (seeded, synthetic RTI boxes, 2 segments per direction from 64
points up, dt = 1e-5): "uneven", eight boxes of 32^3 ... 192^3 points (the sizes
of the serving stream); "small", 48 boxes of 24^3 ... 48^3 points (many boxes
none of which fills the GPU alone).
`steps` timed steps after one untimed step, HIP events on the launch stream.
Prints one JSON line.

    python -m paper_2203_00879_amd.batch_bench [--steps 10] [--precision fp64|mixed] [--set uneven|small]
"""
import argparse
import json
import os
import sys

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    __package__ = "paper_2203_00879_amd"

from . import inputs, nopcs  # noqa: E402

SETS = {"uneven": [32, 48, 64, 96, 128, 160, 192, 40],
        "small": [24 + 4 * (i % 7) for i in range(48)]}


def run(steps=10, precision="fp64", which="uneven"):
    import torch
    SIZES = SETS[which]
    prec = nopcs.MIXED if precision == "mixed" else nopcs.FP64
    prm = nopcs.make_params(inputs.AIR)
    boxes = []
    for i, n in enumerate(SIZES):
        g = nopcs.make_grid(n, 1 if n < 64 else 2)
        Q = torch.from_numpy(inputs.rti_state(n, seed=i)).to("cuda")
        boxes.append((g, Q, nopcs.alloc_workspace(g, prec)))
    pts = sum(n ** 3 for n in SIZES)
    stream = torch.cuda.current_stream()
    nopcs.lib().nopcs_set_graphs(0)
    out = {"metric": "Mpoint-stage updates/s, batch of %d RTI boxes %s (%s)" % (len(SIZES), SIZES, precision),
           "points": pts, "steps": steps}

    def timed(fn):
        fn(1)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        fn(steps)
        e.record(stream)
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / steps
        return {"ms_per_step": ms, "Mpoint_stage_per_s": 4 * pts / (ms * 1e-3) / 1e6}

    def sequential(k):
        for _ in range(k):
            for g, Q, ws in boxes:
                nopcs.rk_step(prm, g, Q, 1e-5, 1, ws, precision=prec, stream=stream)

    out["sequential_one_stream"] = timed(sequential)
    for mode, name in ((0, "batch_launches_graph"), (2, "batch_launches_direct"), (1, "batch_graph_branches"),
                       (3, "batch_hybrid")):
        nopcs.set_batch_mode(mode)
        out[name] = timed(lambda k: nopcs.rk_step_batch(prm, boxes, 1e-5, k, precision=prec, stream=stream))
    nopcs.set_batch_mode(3)
    out["finite"] = all(bool(torch.isfinite(Q).all()) for _, Q, _ in boxes)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--set", choices=sorted(SETS), default="uneven")
    a = ap.parse_args()
    print(json.dumps(run(a.steps, a.precision, a.set)), flush=True)


if __name__ == "__main__":
    main()
