#!/usr/bin/env python3
"""Benchmark of the NOHAP/OUCS3 compressible-NSE hot path on one MI355X.

One "step" = one classical RK4 time step (4 stages) of the whole path: viscous
fluxes + gravity, NOHAP compact convective derivatives along x, y, z, the RK4
register update and the wall conditions, on a Rayleigh-Taylor box resident in
HBM (synthetic, seeded).  Default workload: 512^3 points, FP64, 4 segments per
direction, dt = 1e-6.

Prints ONE JSON line:
  metric/value/unit : Mpoint-stage updates/s (points x 4 stages x steps / s / 1e6)
  roofline          : dominant kernel: the method's algorithmic bytes of the stage
                      it completes (170 B per point-stage in FP64: three 5-field
                      RK4 registers) / its mean launch time (HIP events on its
                      stream, over the timed region); its own compulsory bytes
                      under roofline.kernel_compulsory
  step_counter_frac : counter-measured HBM bytes of the timed region / its time
  mixed             : a short pass of the same box in mixed precision
  serving           : p50/p99 latency of a small Poisson stream of RTI boxes
  cpu_baseline      : the FP64 oracle timed on the host cores on a bounded sample
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X FP64 vector

# timing ids of the library (NOPCS_K_* in include/nopcs.h), in order
KERNEL_NAMES = ["viscous", "sweep_x", "sweep_y", "sweep_z", "wall", "derivative", "rk_update", "closure_y",
                "closure_z"]
KERNEL_SOURCES = {
    "viscous": ["visc.hip", "common.hpp", "kernels.hpp", "batch.hpp"],
    "sweep_x": ["sweep.hip", "sweep.hpp", "common.hpp", "plan.cpp", "batch.hpp"],
    "sweep_y": ["march.hip", "common.hpp", "plan.cpp", "batch.hpp"],
    "sweep_z": ["march.hip", "common.hpp", "plan.cpp", "kernels.hpp", "batch.hpp"],
    "closure_y": ["march.hip", "common.hpp", "plan.cpp", "batch.hpp"],
    "closure_z": ["march.hip", "common.hpp", "plan.cpp", "batch.hpp"],
    "rk_update": ["sweep.hip"],
    "wall": ["visc.hip", "common.hpp"],
}


def kernel_bytes_per_point(name, precision, fused_rk=False):
    """Compulsory HBM bytes per grid point of one launch (each operand read or written once).
    Mixed precision stores the RHS register R in FP32 (4 bytes); everything else is FP64.
    fused_rk: the RK4 stage update rides on the z sweep (FP64 line march)."""
    w = 8                                          # state, K, Qn, Qs
    r = 4 if precision == "mixed" else 8           # R
    if name == "viscous":
        return 5 * w + 5 * r                       # read stage state, write R
    if name == "sweep_z" and fused_rk:
        # read state, R, Qn and (stages 1-3) K; write K and the next stage state
        # (stages 0-2) or Qn (stage 3); averaged over the 4 stages
        return 5 * w + 5 * r + 5 * w + (3 * 5 * w) / 4.0 + (3 * 10 * w + 5 * w) / 4.0
    if name in ("sweep_x", "sweep_y", "sweep_z"):
        return 5 * w + 5 * r + 5 * r               # read state, read R, write R
    if name in ("closure_y", "closure_z"):
        return 5 * w                               # read state (closure rows written: ~1/16 of a field)
    if name == "rk_update":
        # stage 0: R, Qn -> K, Qs; stages 1, 2: R, Qn, K -> K, Qs; stage 3: R, Qn, K -> Qn;
        # over the 4 stages: R read 4 times, FP64 fields read 7 and written 7 times
        return (4 * 5 * r + 14 * 5 * w) / 4.0
    return 0.0


def source_hash(name):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(name, []):
        p = os.path.join(ROOT, "paper_2203_00879_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def load_counter_record(name, workload_key, field):
    """A per-launch figure of a committed counter run (profiles/traffic.json: HBM
    bytes, FP64 flops), if taken on the kernel's current source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        rec = d.get(workload_key, {}).get(name)
        if rec and rec.get("source_hash") == source_hash(name):
            return rec.get(field)
    except Exception:
        return None
    return None


def load_traffic(name, workload_key):
    """HBM bytes per launch from committed counter runs, if taken on the current source."""
    return load_counter_record(name, workload_key, "bytes_per_launch")


def cpu_baseline(n=128, steps=1):
    import numpy as np  # noqa: F401

    import oracle
    from paper_2203_00879_amd import inputs
    p = dict(inputs.AIR)
    Q = inputs.rti_state(n, seed=0)
    oracle.lib()
    t0 = time.perf_counter()
    oracle.rk4(p, Q, 1e-6, steps)
    dt = time.perf_counter() - t0
    pts = n ** 3 * 4 * steps
    return {"value": pts / dt / 1e6, "unit": "Mpoint-stage/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "RTI box %d^3, %d RK4 step(s) (%d stages), FP64 oracle, %.1f s" % (n, steps, 4 * steps, dt)}


def time_steps(nopcs, lib, params, grid, Q, ws, dt, steps, warmup, prec, stream):
    """warmup untimed steps, then `steps` timed ones (HIP events on the launch
    stream around the whole region, per-kernel events from the library)."""
    import ctypes
    import torch
    nopcs.rk_step(params, grid, Q, dt, warmup, ws, precision=prec)
    torch.cuda.synchronize()
    lib.nopcs_timing_enable(1)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    nopcs.rk_step(params, grid, Q, dt, steps, ws, precision=prec)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lib.nopcs_timing_enable(0)
    per = {}
    for k, name in enumerate(KERNEL_NAMES):
        tot, cnt = ctypes.c_double(), ctypes.c_int64()
        nopcs._check(lib.nopcs_timing_read(k, ctypes.byref(tot), ctypes.byref(cnt)))
        if cnt.value:
            per[name] = (tot.value, cnt.value)
    return start.elapsed_time(stop), per, wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--nseg", type=int, default=4)
    ap.add_argument("--dt", type=float, default=1e-6)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the short mixed-precision pass")
    ap.add_argument("--no-serving", action="store_true", help="skip the small serving sample")
    ap.add_argument("--mixed-steps", type=int, default=10)
    ap.add_argument("--cpu-n", type=int, default=256)
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--calibrate-copy", type=float, default=0.0,
                    help="GiB: run one plain device copy of this size first (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (one box = one MI355X); "
              "--gpus %d is not supported." % args.gpus, file=sys.stderr)
        sys.exit(2)

    import ctypes

    import torch

    from paper_2203_00879_amd import inputs, nopcs

    dev = "cuda:0"
    if args.calibrate_copy > 0:
        nb = int(args.calibrate_copy * (1 << 30)) // 8
        a = torch.ones(nb, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    n = args.n
    p = dict(inputs.AIR)
    grid = nopcs.make_grid(n, args.nseg)
    params = nopcs.make_params(p)
    Q0 = inputs.rti_state(n, seed=0)
    Q = torch.from_numpy(Q0).to(dev)
    prec = nopcs.MIXED if args.precision == "mixed" else nopcs.FP64
    ws = nopcs.alloc_workspace(grid, prec)
    stream = torch.cuda.current_stream()
    lib = nopcs.lib()
    lib.nopcs_timing_enable.argtypes = [ctypes.c_int]
    lib.nopcs_timing_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]

    ms, per, wall = time_steps(nopcs, lib, params, grid, Q, ws, args.dt, args.steps, args.warmup, prec, stream)
    sec = ms / 1e3
    finite = bool(torch.isfinite(Q).all().item())
    del ws

    N3 = n ** 3
    pstage = N3 * 4 * args.steps
    value = pstage / sec / 1e6
    pr = args.precision
    fused = "rk_update" not in per
    bpp = lambda k: kernel_bytes_per_point(k, pr, fused)   # noqa: E731
    dom = max((k for k in per if k in KERNEL_SOURCES and bpp(k) > 0), key=lambda k: per[k][0])
    tot_ms, cnt = per[dom]
    avg_s = tot_ms / cnt / 1e3
    # the method's algorithmic bytes per point-stage: three 5-field RK4 registers
    # (FP64 170 B; mixed precision with the stage state in FP32, 125 B)
    alg_pps = 170.0 if pr == "fp64" else 125.0
    achieved = alg_pps * N3 / avg_s / 1e9
    bpl = bpp(dom) * N3
    workload_key = "rti_%d_fp64_seg%d" % (n, args.nseg)
    traffic = load_traffic(dom, workload_key) if pr == "fp64" else None
    flop = load_counter_record(dom, workload_key, "fp64_flop_per_launch") if pr == "fp64" else None
    # counter bytes of the whole timed region (per-kernel counter runs x launches)
    step_bytes = 0.0
    for k, (t, c) in per.items():
        tb = load_traffic(k, workload_key) if pr == "fp64" else None
        if tb is None and k != "wall":
            step_bytes = None
            break
        step_bytes += (tb or 0.0) * c
    kernels = {k: {"ms_per_launch": v[0] / v[1], "launches": v[1],
                   "alg_GBps": (bpp(k) * N3 / (v[0] / v[1] / 1e3) / 1e9) if bpp(k) else None}
               for k, v in per.items()}
    out = {
        "metric": "Mpoint-stage updates/s at 512\u00b3 FP64 vs mixed; p50/p99 batched solve latency",
        "value": value,
        "unit": "Mpoint-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if pr == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": "Rayleigh-Taylor box %d^3, %s, %d segments/direction, RK4 dt=%g, seeded "
                               "interface noise" % (n, "FP64" if pr == "fp64" else "mixed precision", args.nseg, args.dt),
                   "points": N3, "segments_per_direction": args.nseg, "precision": pr},
        "rk_update_fused_into_sweep_z": fused,
        # dominant kernel: the method's algorithmic bytes of the stage it completes
        # (alg_pps per point-stage x points) over its mean launch time
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_pps * N3, "alg_bytes_per_point_stage": alg_pps,
                     "mean_launch_ms": avg_s * 1e3,
                     # the kernel's own compulsory bytes (every operand it reads or writes once)
                     "kernel_compulsory": {"bytes_per_launch": bpl, "achieved": bpl / avg_s / 1e9,
                                           "frac": bpl / avg_s / 1e9 / HBM_PEAK_GBS}},
        "step_algorithmic_frac": alg_pps * pstage / sec / 1e9 / HBM_PEAK_GBS,
        # counter-measured HBM bytes of every launch in the timed region over its
        # time (null when a kernel's counters were taken on other sources)
        "step_counter_frac": None if step_bytes is None else step_bytes / sec / 1e9 / HBM_PEAK_GBS,
        "step_counter_bytes_per_point_stage": None if step_bytes is None else step_bytes / pstage,
        # FP64 VALU rate of the dominant kernel: counter-measured FP64 flops per
        # launch (64 lanes x (add + mul + trans + 2 fma) instructions) / its mean
        # launch time, against the FP64 vector peak (null if the counters were
        # taken on other sources)
        "fp64_valu": None if flop is None else {
            "kernel": dom, "achieved": flop / avg_s / 1e12, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": flop / avg_s / 1e12 / FP64_VALU_PEAK_TFLOPS},
        "kernels": kernels,
        "finite": finite,
        "wall_s": wall,
        "paper_context": {"Mpoint_stage_per_s": 19700.0,
                          "hardware": "19,200 Haswell cores, 4.19e9 points, FP64 (paper, other machine)"},
    }
    if pr == "fp64" and not args.no_mixed:
        # the metric's other precision: a short mixed-precision pass on the same box
        Q.copy_(torch.from_numpy(Q0))
        wsm = nopcs.alloc_workspace(grid, nopcs.MIXED)
        msm, _, _ = time_steps(nopcs, lib, params, grid, Q, wsm, args.dt, args.mixed_steps, 1, nopcs.MIXED, stream)
        del wsm
        out["mixed"] = {"steps": args.mixed_steps, "ms_per_step": msm / args.mixed_steps,
                        "Mpoint_stage_per_s": N3 * 4 * args.mixed_steps / (msm / 1e3) / 1e6,
                        "speedup_vs_fp64": (ms / args.steps) / (msm / args.mixed_steps),
                        "finite": bool(torch.isfinite(Q).all().item())}
    del Q
    torch.cuda.empty_cache()
    if not args.no_serving:
        # the metric's latency part: a small Poisson stream of RTI boxes through the
        # serving runtime, mixed precision, at an arrival rate the GPU sustains
        from paper_2203_00879_amd import serve_bench
        sv = serve_bench.run(n_req=24, step_scale=0.1, slots=8, budget_gb=60.0, precision="mixed",
                             mean_gap_s=0.1)
        out["serving"] = {k: sv[k] for k in ("requests", "all_ok", "Mpoint_stage_per_s", "p50_latency_s",
                                             "p99_latency_s", "p50_admission_s", "p99_admission_s",
                                             "offered_Mpoint_stage_per_s", "mean_gap_s", "step_scale", "precision")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
