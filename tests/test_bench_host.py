"""Host-side logic of bench.py: byte accounting, the counter summaries and their staleness
check, and the one-GPU contract (no GPU needed)."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import synth  # noqa: E402


def test_algorithmic_bytes_match_the_paper_sizes():
    # 2e7-row workload: 4.84 GB for aprod 1 and 4.72 GB for aprod 2 (24 nnz/row, int32 indices)
    sh = synth.WORKLOADS["stars1e6_obs20_dfa3e4_instr6e3"]
    m, n = 20_000_000, sh.n_cols
    ab = bench.algorithmic_bytes(m, n)
    assert ab["aprod1"] == 24 * m * 8 + 32 * m + 16 * m + 8 * n
    assert abs(ab["aprod1"] / 1e9 - 4.84) < 0.01 and abs(ab["aprod2"] / 1e9 - 4.72) < 0.01
    # the fused schedule moves less than the two products, and both passes together still
    # read every coefficient exactly once plus the attitude copy once
    pb = bench.pass_bytes(m, n, sh, fused=True)
    assert pb["pass1"] + pb["pass2"] < ab["aprod1"] + ab["aprod2"]
    assert pb["pass1"] >= 24 * m * 8 and pb["pass2"] >= 12 * m * 8
    assert bench.pass_bytes(m, n, sh, fused=False) == {"pass1": ab["aprod1"], "pass2": ab["aprod2"]}
    # binary32 values halve the coefficient bytes only
    ab32 = bench.algorithmic_bytes(m, n, value_bytes=4)
    assert ab["aprod1"] - ab32["aprod1"] == 24 * m * 4


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, (name, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": v})


def test_counter_summary_scaling_and_staleness(tmp_path, monkeypatch):
    gib_kib = (1 << 30) / 1024
    copy = "__amd_rocclr_copyBuffer(void*, void*)"
    kern = "void gsr::k_aprod12<double, 1, false, false>(gsr::Geo, ...)"
    init = "void gsr::k_aprod12<double, 1, false, true>(gsr::Geo, ...)"  # a solve's first pass
    # FETCH reads half of the copy's true bytes, WRITE all of them
    _write_counters(tmp_path / "f", "FETCH_SIZE",
                    [(copy, gib_kib / 2)] * 3 + [(copy, 5.0), (init, 1e6), (kern, 3e6),
                                                 (kern, 3e6)])
    _write_counters(tmp_path / "w", "WRITE_SIZE",
                    [(copy, gib_kib)] * 3 + [(init, 7.0), (kern, 1e5), (kern, 1e5)])
    monkeypatch.setattr(bench, "traffic_path",
                        lambda k, wl: str(tmp_path / f"{k}_{wl}_hbm_traffic.txt"))
    out = bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"),
                            "k_aprod12<double, 1, false, false>", "wl", "cmd")
    assert out.endswith("k_aprod12_wl_hbm_traffic.txt")
    text = open(out).read()
    assert "fetch_scale: 2.0000" in text and "write_scale: 1.0000" in text
    assert "dispatches_fetch: 2" in text  # the initial pass is not averaged in
    traffic = 3e6 * 1024 * 2 + 1e5 * 1024
    got = bench.stored_traffic("k_aprod12", "wl", algorithmic=traffic * 0.99)
    assert got == pytest.approx(traffic, rel=1e-6)
    # below the algorithmic bytes: the counters missed traffic, nothing is reported
    assert bench.stored_traffic("k_aprod12", "wl", algorithmic=traffic * 2) is None
    # kernels changed since the counters were taken: stale, nothing is reported
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.stored_traffic("k_aprod12", "wl", algorithmic=1.0) is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
