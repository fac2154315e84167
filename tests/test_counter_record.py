"""The committed counter record (profiles/traffic.json: HBM bytes and FP64
flops per launch of the RK4 step kernels at 512^3) was taken on the kernels'
current sources; otherwise the bench line reports no traffic for them."""
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_counter_record_matches_kernel_sources():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["rti_512_fp64_seg4"]
    for k in ("viscous", "sweep_x", "closure_y", "sweep_y", "closure_z", "sweep_z"):
        assert rec[k]["source_hash"] == bench.source_hash(k), k
        assert rec[k]["bytes_per_launch"] > 0 and rec[k]["fp64_flop_per_launch"] > 0, k
