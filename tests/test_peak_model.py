"""The paper's performance model (Eq. 4-5, Table 1) and its MI355X evaluation."""
import json
import os

import pytest

from paper_2309_09609_amd import perfmodel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_peaks.json")


def test_table1_peaks_reproduce():
    rows = json.load(open(GOLDEN))["rows"]
    assert len(rows) == 10
    for r in rows:
        p = perfmodel.theo_peak_gcups(r["cores"], r["lanes"], r["throughput"], r["clock_mhz"])
        # Table 1 prints 3-5 significant digits, truncated for the RTX 3090
        assert p == pytest.approx(r["peak_gcups"], abs=0.1), r["gpu"]


def test_mi355x_peaks():
    assert perfmodel.mi355x_peak_gcups() == pytest.approx(3276.8)
    assert perfmodel.mi355x_peak_gcups(cells_per_lane_op=2) == pytest.approx(6553.6)
    assert perfmodel.int_valu_lane_ops_per_s() == pytest.approx(39.3216e12)
