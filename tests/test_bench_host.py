"""Host logic of bench.py (no GPU): the one-GPU guard and the counter
summary that turns rocprofv3 FETCH_SIZE / WRITE_SIZE readings into HBM bytes."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

LZ = "void tmk::row_kernel<tmk::Plan<7, 6, -1, 0>, 13, float, true>(tmk::RowArgs)"
ERC = "void tmk::row_kernel<tmk::Plan<7, 6, -1, 0>, 12, float, false>(tmk::RowArgs)"
ERC_S = "void tmk::row_kernel<tmk::Plan<7, 6, -1, 0>, 12, float, true>(tmk::RowArgs)"
LZ8 = "void tmk::row_kernel_w<tmk::Plan<7, 6, 3, 1>, 13, float, true, 1024>(tmk::RowArgs)"
COPY = "__amd_rocclr_copyBuffer"
DOTS = "tmk::(anonymous namespace)::k_dir_dots(tmk::(anonymous namespace)::LbArgs, double*)"
SOLVE = "tmk::(anonymous namespace)::k_dir_solve(tmk::(anonymous namespace)::LbArgs, double const*, int)"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, v in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_counter_summary_scales_by_the_copy_and_tracks_the_sources(tmp_path, monkeypatch):
    f, w, cf, cw = (str(tmp_path / s) for s in ("f", "w", "cf", "cw"))
    # a stray dispatch of another plan (fewer dispatches) is not mixed in
    _counters(f, "FETCH_SIZE", [(LZ, 100.0), (LZ, 200.0), (ERC, 40.0), (ERC_S, 60.0), (ERC, 40.0), (DOTS, 10.0),
                                (SOLVE, 20.0), (LZ8, 999.0)])
    _counters(w, "WRITE_SIZE", [(LZ, 50.0), (LZ, 50.0), (ERC, 30.0), (ERC_S, 30.0), (ERC, 30.0), (DOTS, 1.0),
                                (SOLVE, 2.0), (LZ8, 999.0)])
    # a 512 MiB copy reads as half its size on the fetch counter, its size on the write counter
    _counters(cf, "FETCH_SIZE", [(COPY, 262144.0), (COPY, 262144.0), ("small", 1.0)])
    _counters(cw, "WRITE_SIZE", [(COPY, 524288.0), (COPY, 524288.0), ("small", 1.0)])
    out = str(tmp_path / "traffic.json")
    bench.pmc_summary(f, w, cf, cw, out)
    d = json.load(open(out))
    assert d["copy"]["kernel"] == COPY and d["copy"]["fetch_kib"] == 262144.0
    assert d["kernels"]["lanczos"] == {"fetch_kib": 150.0, "write_kib": 50.0, "dispatches": [2, 2],
                                       "plan": "Plan<7, 6, -1, 0>"}
    # dispatches with and without sums are averaged by count
    assert abs(d["kernels"]["er_cyclic"]["fetch_kib"] - 140.0 / 3) < 1e-12
    assert "spectral" not in d["kernels"]
    monkeypatch.setattr(bench, "TRAFFIC_FILE", out)
    t = bench.measured_traffic(2286, 8192)
    assert t["lanczos"] == (150 * 2 + 50 * 1) * 1024
    assert bench.measured_traffic(2286, 4096) is None
    # row-kernel figures only for the launch configuration they were taken on
    assert bench.plan_tag(7, 6, 0) == "Plan<7, 6, -1, 0>" and bench.plan_tag(7, 6, 3) == "Plan<7, 6, 3, 1>"
    assert bench.measured_traffic(2286, 8192, bench.plan_tag(7, 6, 0))["lanczos"] == t["lanczos"]
    t3 = bench.measured_traffic(2286, 8192, bench.plan_tag(7, 6, 3))
    assert "lanczos" not in t3 and "lbfgs_direction" in t3
    # the L-BFGS direction's HBM pass is k_dir_dots (the solve reads only its partial sums)
    assert t["lbfgs_direction"] == (10 * 2 + 1 * 1) * 1024
    # each figure is dropped once the sources it was taken on change
    d["sources_sha256"] = "0" * 64
    json.dump(d, open(out, "w"))
    t = bench.measured_traffic(2286, 8192)
    assert "lanczos" not in t and "lbfgs_direction" in t
    d["lbfgs_sources_sha256"] = "0" * 64
    json.dump(d, open(out, "w"))
    assert bench.measured_traffic(2286, 8192) == {}


def test_sources_digest_is_stable():
    assert bench.sources_digest() == bench.sources_digest()
    assert len(bench.sources_digest()) == 64


def test_trace_summary_keeps_the_timed_region(tmp_path):
    # kernels that start and end inside the roctx range are the timed region's
    d = str(tmp_path)
    with open(os.path.join(d, "x_marker_api_trace.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Domain", "Function", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerow({"Domain": "MARKER_CORE_API", "Function": bench.TIMED_RANGE, "Start_Timestamp": 1000,
                    "End_Timestamp": 5000})
        w.writerow({"Domain": "MARKER_CORE_API", "Function": "other", "Start_Timestamp": 0, "End_Timestamp": 9000})
    with open(os.path.join(d, "x_kernel_trace.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for a, b, n in ((500, 900, "k"), (1100, 1500, "k"), (2000, 2600, "k"), (4900, 5100, "k"), (3000, 3100, "j")):
            w.writerow({"Kernel_Name": n, "Start_Timestamp": a, "End_Timestamp": b})
    acc = bench.trace_summary(d)
    assert sorted(acc["k"]) == [0.4, 0.6] and acc["j"] == [0.1]
    with pytest.raises(SystemExit):
        bench.trace_summary(str(tmp_path / "missing"))
