"""Per-launch HBM bytes and FP64 flops of the RK4 step kernels from rocprofv3
counter runs, written to profiles/traffic.json under the kernels' source hashes
(bench.py reports them as roofline.traffic and fp64_valu while the sources
match), plus the markdown rows of the traffic, FP64 and trace summaries.

Inputs: the csv output directories of four runs of bench.py at 512^3 FP64
(one RK4 step each; see profiles/hbm_traffic_512_fp64.md for the commands):
a FETCH_SIZE pass and a WRITE_SIZE pass, both with --calibrate-copy 2 (a device
copy of 2 GiB whose counter values give the KiB-per-count factors), an FP64
VALU pass and a kernel trace.

    python3 -m paper_2203_00879_amd.counter_record --fetch DIR --write DIR --f64 DIR --trace DIR
"""
import argparse
import collections
import csv
import importlib.util
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WORKLOAD = "rti_512_fp64_seg4"
COPY_KIB = 2 * 1024 * 1024   # bench.py --calibrate-copy 2: 2 GiB copied
FP64_PEAK = 78.6e12


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def short(name):
    m = re.search(r"k_one<nopcs::(?:\(anonymous namespace\)::)?(\w+<[^>]*>)", name)
    return m.group(1) if m else name.split("(")[0][:90]


def key(sname):
    """The bench.py kernel key of a body kernel's short name (FP64 stepping)."""
    if sname.startswith("ViscBody<double>"):
        return "viscous"
    if sname.startswith("SweepBody<0, 512, double>"):
        return "sweep_x"
    if sname == "ClosureLineBody<1>":
        return "closure_y"
    if sname == "ClosureLineBody<2>":
        return "closure_z"
    if sname.startswith("MarchBody<1, true, double, double, -1"):
        return "sweep_y"
    if sname.startswith("MarchBody<2, true, double, double,"):
        return "sweep_z"
    return None


def counters(path, cname):
    per = collections.defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == cname:
                per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return per


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--f64", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--prefix", default="run", help="rocprofv3 -o name of the runs")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args()
    bench = _bench()
    csvf = lambda d, kind: os.path.join(d, "%s_%s.csv" % (args.prefix, kind))
    fetch = counters(csvf(args.fetch, "counter_collection"), "FETCH_SIZE")
    write = counters(csvf(args.write, "counter_collection"), "WRITE_SIZE")
    cal_f = [v for k, v in fetch.items() if "copyBuffer" in k][0][0]
    cal_w = [v for k, v in write.items() if "copyBuffer" in k][0][0]
    ff, fw = COPY_KIB / cal_f, COPY_KIB / cal_w
    print("calibration: copy of %d KiB reads %.0f KiB by FETCH_SIZE and writes %.0f KiB by WRITE_SIZE: "
          "factors %.3f (read), %.3f (write)" % (COPY_KIB, cal_f, cal_w, ff, fw))
    rows = []
    for k in fetch:
        s = short(k)
        if key(s) is None:
            continue
        rd = sum(fetch[k]) / len(fetch[k]) * ff * 1024 / 1e9
        wr = sum(write[k]) / len(write[k]) * fw * 1024 / 1e9 if k in write else float("nan")
        rows.append((s, len(fetch[k]), rd, wr))
    order = ["viscous", "sweep_x", "closure_y", "sweep_y", "closure_z", "sweep_z"]
    rows.sort(key=lambda r: (order.index(key(r[0])), r[0]))
    print("TRAFFIC (kernel | dispatches | read GB/launch | write GB/launch)")
    for r in rows:
        print("| `%s` | %d | %.2f | %.2f |" % r)
    dur = {}
    with open(csvf(args.trace, "kernel_stats")) as fh:
        trace = list(csv.DictReader(fh))
    print("TRACE (kernel | calls | total us | average us | %)")
    for r in trace:
        dur[short(r["Name"])] = float(r["AverageNs"])
        print("| `%s` | %s | %.1f | %.1f | %.2f |" % (short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e3,
                                                   float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    f64 = collections.defaultdict(lambda: collections.defaultdict(list))
    with open(csvf(args.f64, "counter_collection")) as fh:
        for r in csv.DictReader(fh):
            f64[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    frows = []
    for k, d in f64.items():
        s = short(k)
        if key(s) is None:
            continue
        avg = {c: sum(v) / len(v) for c, v in d.items()}
        flop = 64 * (avg.get("SQ_INSTS_VALU_ADD_F64", 0) + avg.get("SQ_INSTS_VALU_MUL_F64", 0)
                     + avg.get("SQ_INSTS_VALU_TRANS_F64", 0) + 2 * avg.get("SQ_INSTS_VALU_FMA_F64", 0))
        frows.append((s, avg.get("SQ_INSTS_VALU", 0), avg.get("SQ_INSTS_VALU_ADD_F64", 0),
                      avg.get("SQ_INSTS_VALU_MUL_F64", 0), avg.get("SQ_INSTS_VALU_FMA_F64", 0),
                      avg.get("SQ_INSTS_VALU_TRANS_F64", 0), flop))
    frows.sort(key=lambda r: (order.index(key(r[0])), r[0]))
    print("F64 (kernel | VALU | add | mul | fma | trans | flop/launch | ms | TFLOP/s | of peak)")
    for r in frows:
        ms = dur.get(r[0], 0.0) / 1e6
        rate = r[6] / (ms * 1e-3) if ms else 0.0
        print("| `%s` | %.3g | %.3g | %.3g | %.3g | %.3g | %.3g | %.2f | %.2f | %.1f %% |"
              % (r[0], r[1], r[2], r[3], r[4], r[5], r[6], ms, rate / 1e12, 100 * rate / FP64_PEAK))
    # per bench key: bytes (read + write) and flops per launch, the z march's
    # four stage kernels averaged
    agg = collections.defaultdict(list)
    for s, _, rd, wr in rows:
        agg[key(s)].append((rd + wr) * 1e9)
    fl = collections.defaultdict(list)
    for r in frows:
        fl[key(r[0])].append(r[6])
    out = {}
    for k in order:
        if k in agg:
            out[k] = {"source_hash": bench.source_hash(k), "bytes_per_launch": sum(agg[k]) / len(agg[k]),
                      "fp64_flop_per_launch": sum(fl[k]) / len(fl[k]) if fl[k] else None}
    with open(args.out, "w") as fh:
        json.dump({WORKLOAD: out}, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
