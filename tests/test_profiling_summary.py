"""The profile bookkeeping behind the bench's roofline fields, on synthetic
rocprofv3 CSV files (no GPU): HBM bytes per launch scaled by the copy
reference, the warm-up dispatch left out of the kernel statistics, the
per-kernel issue counters kept beside the traffic, and the ratios the bench
reports from them, which are None once the kernel sources have changed."""
import csv
import json
import os

import pytest

from paper_2503_16955_amd import profiling

K = "void mrt::tk::trace_kernel<double, 1, 2, 1, false>(mrt::TraceParams)"


def _counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def _trace(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_kernel_trace.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for k, s, e in rows:
            w.writerow({"Kernel_Name": k, "Start_Timestamp": s, "End_Timestamp": e})


@pytest.fixture
def run(tmp_path, monkeypatch):
    d = str(tmp_path)
    # a 256 MiB copy reads 256 MiB, of which FETCH_SIZE shows half; writes all
    _counters(d + "/cf", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 131072.0)])
    _counters(d + "/cw", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 262144.0)])
    # two dispatches of the kernel
    _counters(d + "/f", [(K, "FETCH_SIZE", 100.0), (K, "FETCH_SIZE", 300.0)])
    _counters(d + "/w", [(K, "WRITE_SIZE", 1000.0), (K, "WRITE_SIZE", 1000.0)])
    _counters(d + "/sq", [(K, "SQ_INSTS_VALU", 6.0e9), (K, "SQ_INSTS_VALU", 6.0e9),
                          (K, "SQ_THREAD_CYCLES_VALU", 3.2e11), (K, "SQ_THREAD_CYCLES_VALU", 3.2e11),
                          (K, "TCC_ATOMIC_sum", 2.0e6), (K, "TCC_ATOMIC_sum", 2.0e6)])
    # a slow warm-up dispatch first, then three of 10 ms
    _trace(d + "/t", [(K, 0, 30_000_000), (K, 40_000_000, 50_000_000),
                      (K, 60_000_000, 70_000_000), (K, 80_000_000, 90_000_000)])
    out = tmp_path / "p.md"
    t = profiling.summarize(d + "/t", [d + "/f", d + "/w", d + "/sq"], d + "/cf", d + "/cw", 256,
                            "cmd", str(out), "label")
    js = tmp_path / "traffic.json"
    js.write_text(json.dumps(t))
    monkeypatch.setattr(profiling, "TRAFFIC_JSON", str(js))
    return t, out.read_text(), js


def test_traffic_counters_and_warm_up(run):
    t, md, _ = run
    k = t["kernels"][K]
    # (200 KiB x 2 + 1000 KiB x 1) per launch
    assert k["hbm_bytes_per_launch"] == pytest.approx((200.0 * 2.0 + 1000.0) * 1024.0)
    assert k["counters"] == {"SQ_INSTS_VALU": 6.0e9, "SQ_THREAD_CYCLES_VALU": 3.2e11,
                             "TCC_ATOMIC_sum": 2.0e6}
    # the warm-up dispatch is left out: 3 kept, average 10 ms
    row = [l for l in md.splitlines() if l.startswith(f"| `{K[:90]}`")][0]
    assert "| 4 | 3 | 10000.0 |" in row
    assert profiling.traffic_per_launch(K) == pytest.approx(k["hbm_bytes_per_launch"])


def test_reported_ratios(run):
    r = profiling.issue_ratios(K, useful_lane_ops=2.56e11, kernel_ms=10.0, cus=256)
    # 6e9 wave instructions in 10 ms against 256 CUs x 2.4 GHz
    assert r["valu_insts_per_cu_clock"] == pytest.approx(6.0e9 / (0.010 * 256 * 2.4e9), rel=1e-3)
    assert r["lane_efficiency"] == pytest.approx(2.56e11 / (6.0e9 * 64), rel=1e-3)
    assert r["lanes_per_valu_inst"] == pytest.approx(53.33, abs=0.01)
    assert r["atomics_per_s"] == pytest.approx(2.0e8)
    assert profiling.issue_ratios("other kernel", 1.0, 1.0, 256) is None


def test_stale_counters_are_not_reported(run, monkeypatch):
    _, _, js = run
    t = json.loads(js.read_text())
    t["sources_sha256"] = "0" * 64
    js.write_text(json.dumps(t))
    assert profiling.traffic_per_launch(K) is None
    assert profiling.issue_ratios(K, 1.0, 10.0, 256) is None
