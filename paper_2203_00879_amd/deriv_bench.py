"""Throughput of the standalone NOHAP derivative (nopcs_derivative) on one GPU.

Workload (seeded, synthetic): the 16-mode Fourier field of inputs.fourier_field
on a 256^3 box, 8 segments per direction (32 points each; default pieces).  Per
direction: D1 alone (16 algorithmic bytes per point: read f, write f') and D1
with D2 (24 bytes per point: read f, write f' and f'').  Timed with HIP events
on the launch stream over `reps` calls after one untimed call.  D1 alone along
y and z runs in the form --form selects: by size (the default: the line march
from 2^17 lines), pencil or march.

Prints one JSON line.

    python -m paper_2203_00879_amd.deriv_bench [--n 256] [--nseg 8] [--reps 20] [--form size|pencil|march]
"""
import argparse
import json
import os
import sys

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    __package__ = "paper_2203_00879_amd"

from . import inputs, nopcs  # noqa: E402

HBM_PEAK_GBS = 8000.0


FORMS = {"size": nopcs.DERIV_BY_SIZE, "pencil": nopcs.DERIV_PENCIL, "march": nopcs.DERIV_MARCH}


def run(n=256, nseg=8, reps=20, form="size"):
    import torch
    nopcs.set_deriv_form(FORMS[form])
    f = torch.from_numpy(inputs.fourier_field(n, inputs.fourier_modes(16, 64, seed=1))).to("cuda")
    g = nopcs.make_grid(n, nseg)
    d1, d2 = torch.empty_like(f), torch.empty_like(f)
    out = {"metric": "standalone NOHAP derivative throughput (Fourier field %d^3, %d segments/direction, FP64)" % (n, nseg),
           "points": n ** 3, "reps": reps, "d1_form_yz": form, "directions": {}}
    for d in range(3):
        row = {}
        for name, second, bpp in (("d1", False, 16), ("d1_d2", True, 24)):
            nopcs.nopcs_derivative(g, d, f, d1, d2 if second else None)
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            for _ in range(reps):
                nopcs.nopcs_derivative(g, d, f, d1, d2 if second else None)
            e.record()
            torch.cuda.synchronize()
            ms = s.elapsed_time(e) / reps
            gbs = bpp * n ** 3 / (ms * 1e-3) / 1e9
            row[name] = {"ms": ms, "Gpoint_per_s": n ** 3 / (ms * 1e-3) / 1e9, "alg_GBps": gbs,
                         "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
        out["directions"]["xyz"[d]] = row
    nopcs.set_deriv_form(nopcs.DERIV_BY_SIZE)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--nseg", type=int, default=8)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--form", choices=sorted(FORMS), default="size", help="form of D1 alone along y and z")
    a = ap.parse_args()
    print(json.dumps(run(a.n, a.nseg, a.reps, a.form)), flush=True)


if __name__ == "__main__":
    main()
