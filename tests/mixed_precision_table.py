"""Error table of the mixed-precision path (NOPCS_MIXED) on the Rayleigh-Taylor box.

(i)  128^3, 4 segments per direction, dt = 1e-6, 100 RK4 steps: the GPU in mixed
     precision against the FP64 CPU oracle (global line solves).
(ii) 512^3, same setup: mixed against FP64 on the GPU, over all points and over
     the central 128^3 block.
Per field: max and L2 error, each relative to the FP64 field's max and L2 norm
over the whole box, of the state and of its change over the run.  Prints a
markdown table.

    python tests/mixed_precision_table.py [--steps 100] [--small 128] [--large 512]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2203_00879_amd import inputs, nopcs  # noqa: E402

FIELDS = ["rho", "rho u", "rho v", "rho w", "E'"]


def gpu_run(n, steps, dt, prec, Q0):
    import torch
    g = nopcs.make_grid(n, 4)
    Q = torch.from_numpy(Q0).to("cuda")
    ws = nopcs.alloc_workspace(g, prec)
    nopcs.rk_step(nopcs.make_params(inputs.AIR), g, Q, dt, steps, ws, precision=prec)
    torch.cuda.synchronize()
    out = Q.cpu().numpy()
    del Q, ws
    torch.cuda.empty_cache()
    return out


def rows(tag, A, B, Q0, sl=None):
    """Errors of A against B per field; on a sub-block (sl) the norms are those
    of the whole field, so that a field that is round-off noise inside the
    block is not divided by its own noise."""
    out = []
    for c in range(5):
        a, b, q = A[c], B[c], Q0[c]
        m = np.max(np.abs(b)) or 1.0
        l2 = np.sqrt(np.mean(b * b)) or 1.0
        dm = np.max(np.abs(b - q)) or 1.0
        dl = np.sqrt(np.mean((b - q) ** 2)) or 1.0
        if sl is not None:
            a, b, q = a[sl], b[sl], q[sl]
        e = a - b
        da, db = a - q, b - q
        out.append("| %s | %s | %.2e | %.2e | %.2e | %.2e |" % (
            tag, FIELDS[c], np.max(np.abs(e)) / m, np.sqrt(np.mean(e * e)) / l2,
            np.max(np.abs(da - db)) / dm, np.sqrt(np.mean((da - db) ** 2)) / dl))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--small", type=int, default=128)
    ap.add_argument("--large", type=int, default=512)
    ap.add_argument("--dt", type=float, default=1e-6)
    a = ap.parse_args()
    print("| run | field | max err / max | L2 err / L2 | change: max err / max | change: L2 err / L2 |")
    print("|---|---|---|---|---|---|")
    t = time.time()
    Q0 = inputs.rti_state(a.small, seed=0)
    mix = gpu_run(a.small, a.steps, a.dt, nopcs.MIXED, Q0)
    ref = oracle.rk4(dict(inputs.AIR), Q0, a.dt, a.steps)
    for r in rows("%d^3 mixed vs FP64 oracle" % a.small, mix, ref, Q0):
        print(r, flush=True)
    print("(small run %.1f s)" % (time.time() - t), file=sys.stderr, flush=True)
    if a.large:
        Q0 = inputs.rti_state(a.large, seed=0)
        mix = gpu_run(a.large, a.steps, a.dt, nopcs.MIXED, Q0)
        f64 = gpu_run(a.large, a.steps, a.dt, nopcs.FP64, Q0)
        for r in rows("%d^3 mixed vs GPU FP64" % a.large, mix, f64, Q0):
            print(r, flush=True)
        c0 = (a.large - 128) // 2
        sl = (slice(c0, c0 + 128),) * 3
        for r in rows("%d^3 central 128^3 (norms of the whole box)" % a.large, mix, f64, Q0, sl):
            print(r, flush=True)


if __name__ == "__main__":
    main()
