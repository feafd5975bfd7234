"""bench.py on the host: the one-GPU rule, the CPU baseline's report and the
HBM-traffic figure's source check (no GPU needed)."""
import argparse
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_cpu_baseline_reports_the_oracle_rate():
    import bench
    from inputs import blosum62, synth
    qs, db = synth.workload1()
    out = bench.cpu_baseline(qs * 2, db, blosum62(), 0.5)
    assert out["kind"] == "oracle" and out["unit"] == "GCUPS"
    assert out["value"] > 0 and out["single_thread_gcups"] > 0 and out["cores"] >= 1
    assert "query 0 (m=144)" in out["sample"]
    host = out["host"]
    assert host["nproc"] >= 1 and host["threads_used"] == out["cores"] <= host["thread_cap"]
    json.dumps(out)


def test_traffic_figure_only_for_the_profiled_kernel_source():
    import bench
    path = os.path.join(ROOT, "profiles", "traffic_k_sweep_i16_sp570k_plain.json")
    with open(path) as f:
        doc = json.load(f)
    assert doc["launches"] == len(doc["fetch_kib_per_launch"]) == len(doc["write_kib_per_launch"])
    per = [(a * doc["fetch_size_scale"] + b * doc["write_size_scale"]) * 1024
           for a, b in zip(doc["fetch_kib_per_launch"], doc["write_kib_per_launch"])]
    assert abs(np.mean(per) - doc["hbm_bytes_per_launch_avg"]) <= 1e-6 * doc["hbm_bytes_per_launch_avg"] + 1
    plain = argparse.Namespace(form="plain", workload="sp570k", mode="local")
    got = bench.measured_traffic(plain)
    assert got is None or got == doc["hbm_bytes_per_launch_avg"]
    assert bench.measured_traffic(argparse.Namespace(form="plain", workload="sp570k", mode="global")) is None
    assert bench.measured_traffic(argparse.Namespace(form="batched", workload="sp570k", mode="local")) is None


def test_served_policies_are_checked_before_any_work():
    for bad in ("paired", "plain", "plain,bogus", "plain,plain"):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--form", "served", "--policies", bad],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode != 0 and "--policies" in r.stderr, bad
    import bench
    ns = argparse.Namespace(policies="plain,pipelined,paired", headline="paired")
    assert bench.served_policies(ns) == (["plain", "pipelined", "paired"], "paired")
    ns = argparse.Namespace(policies="plain,served", headline="paired")
    assert bench.served_policies(ns) == (["plain", "served"], "served")
