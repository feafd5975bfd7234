"""bench.py end to end on a small workload: one JSON line with the contract's
fields, a roofline fraction within (0, 1] and a CPU baseline from the oracle."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_on_the_small_workload():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "small2k", "--steps", "2",
                        "--warmup", "1", "--cpu-seconds", "1", "--no-batched-compare"],
                       capture_output=True, text=True, timeout=110)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1 and d["value"] > 0
    assert d["config"]["workload"] == "small2k"
    roof = d["roofline"]
    assert roof["bound"] == "alu" and 0 < roof["frac"] <= 1 and roof["launches"] >= 1
    assert roof["traffic"] is None                     # measured for the 570k-subject workload only
    assert d["cpu_baseline"]["kind"] == "oracle" and d["cpu_baseline"]["value"] > 0
    lat = d["extra"]["query_latency_ms"]
    assert 0 < lat["p50"] <= lat["p99"] <= lat["max"] and lat["queries"] == d["config"]["queries"]


def test_bench_line_of_the_pair_form():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--form", "pair", "--pair-len", "20000",
                        "--steps", "2", "--warmup", "1"], capture_output=True, text=True, timeout=110)
    assert r.returncode == 0, r.stderr[-2000:]
    d = json.loads([l for l in r.stdout.splitlines() if l.startswith("{")][0])
    assert d["config"]["workload"] == "pair20k" and d["value"] > 0
    assert 0 < d["roofline"]["frac"] <= 1
    # the GPU score equals the oracle's on the same pair (the baseline leg runs the whole 20k x 20k pair)
    assert d["cpu_baseline"]["score"] == d["extra"]["score"]
