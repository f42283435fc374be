"""Host-side logic of bench.py (no GPU): the lane-op accounting, the per-CU
balance statistics from wave trace records, the workload statistics, the
committed traffic lookup and the refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_lane_op_counts():
    # a skip test for every examined / walked pair, plus the blend or contributor work
    assert bench.fwd_ops(0, 0) == 0 and bench.bwd_ops(0, 0) == 0
    assert bench.fwd_ops(10, 0) == 10 * bench.OPS_SKIP_TEST
    assert bench.fwd_ops(10, 4) == 10 * bench.OPS_SKIP_TEST + 4 * bench.OPS_FWD_BLEND
    assert bench.bwd_ops(10, 4) == 10 * bench.OPS_SKIP_TEST + 4 * bench.OPS_BWD_CONTRIB
    # a blend costs more than a skip in both directions, the backward's more than the forward's
    assert 0 < bench.OPS_FWD_BLEND < bench.OPS_BWD_CONTRIB


def test_balance_stats():
    # two CUs: CU a's last wave ends at 100 ticks after the first start, CU b's at 80
    rec = np.array([[1 + 5, 1000, 1060], [1 + 5, 1010, 1100], [1 + 9, 1000, 1080], [0, 0, 0]], np.int64)
    st = bench.balance_stats(rec)
    assert st["n_cu"] == 2 and st["n_waves"] == 3
    assert st["span_ms"] == pytest.approx(100 * 1e-5)
    assert st["spread"] == pytest.approx(0.2)
    assert st["mean_busy"] == pytest.approx(0.9)
    assert bench.balance_stats(np.zeros((4, 3), np.int64)) is None  # no wave recorded


def test_workload_stats():
    # a 32x16 image = two 16x16 tiles; every pixel examines 5 entries except one of 64 in tile 0
    ex = np.full((16, 32), 5, np.int64)
    ex[0, 0] = 69
    st = bench.workload_stats(ex, np.array([100, 7]))
    assert st["list_len"]["max"] == 100
    assert st["examined_per_pixel"]["max"] == 69
    assert st["examined_per_pixel"]["mean"] == pytest.approx(ex.mean())
    # static waves (16x4 pixels): 8 waves, one of cost 69, seven of cost 5
    total = 69 + 7 * 5
    assert st["tail_ratio_static"] == pytest.approx(69 / (total / 1024))
    assert st["lane_waste_static"] == pytest.approx(total * 64 / ex.sum())


def test_measured_traffic_lookup():
    assert bench.measured_traffic("no_such_kernel") is None
    v = bench.measured_traffic("k_bwd_wide")
    # committed figure for the current source, or None once the kernel's source has changed
    assert v is None or v > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
