"""Host-side logic of bench.py (no GPU): the refusal of several GPUs, the HBM
traffic arithmetic from FETCH_SIZE / WRITE_SIZE with the copy calibration, the
per-non-zero counter summary, the staleness check of the committed traffic
figure, and the kernel names the summaries select on.
"""
import csv
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Kernel_Name", "Counter_Name", "Counter_Value"], r)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_kernel_names(bench):
    assert bench.win_kernel_name(32, 3) == "k_mttkrp_win<16, 2, float, 3, false, true>"
    assert bench.win_kernel_name(16, 4, "uint16_t", False, False) == \
        "k_mttkrp_win<16, 1, uint16_t, 4, false, false>"
    assert bench.win_kernel_name(64, 3, big=True) == "k_mttkrp_win<16, 4, float, 3, true, true>"
    assert bench.short_kernel_name(32, 4) == "k_mttkrp_short<2, float, 4, false>"


def test_traffic_scaled_by_the_copy(bench, tmp_path):
    k = "void " + bench.win_kernel_name(32, 3)
    fetch, write, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.txt"
    # two MTTKRP dispatches (mean 300 KiB fetched), a small copy and the 1 MiB
    # calibration copy that the counter reports as 512 KiB fetched, 1024 written
    write_csv(fetch, [(k + "(blco::KParams)", "FETCH_SIZE", 200.0),
                      (k + "(blco::KParams)", "FETCH_SIZE", 400.0),
                      ("copyBuffer small", "FETCH_SIZE", 3.0),
                      ("copyBuffer big", "FETCH_SIZE", 512.0),
                      ("other", "FETCH_SIZE", 1e9)])
    write_csv(write, [(k + "(blco::KParams)", "WRITE_SIZE", 100.0),
                      (k + "(blco::KParams)", "WRITE_SIZE", 100.0),
                      ("copyBuffer big", "WRITE_SIZE", 1024.0)])
    bench.summarize_pmc(str(fetch), str(write), 1 << 20, out=str(out))
    vals = dict(line.split(": ") for line in out.read_text().splitlines() if not line.startswith("#"))
    assert vals["mttkrp_dispatches"] == "2"
    assert float(vals["fetch_scale"]) == pytest.approx(2.0)
    assert float(vals["write_scale"]) == pytest.approx(1.0)
    assert float(vals["hbm_fetch_bytes_per_launch"]) == pytest.approx(300 * 1024 * 2)
    assert float(vals["hbm_write_bytes_per_launch"]) == pytest.approx(100 * 1024)
    assert vals["kernel_source_sha256_16"] == bench.kernel_source_hash()


def test_counter_summary_per_nonzero(bench, tmp_path):
    k = bench.win_kernel_name(32, 3)
    a, b, out = tmp_path / "a.csv", tmp_path / "b.csv", tmp_path / "c.txt"
    write_csv(a, [("void " + k + "(blco::KParams)", "SQ_INSTS_VALU", 800.0),
                  ("void " + k + "(blco::KParams)", "SQ_INSTS_VALU", 1200.0),
                  ("void k_other(blco::KParams)", "SQ_INSTS_VALU", 5.0)])
    write_csv(b, [("void " + k + "(blco::KParams)", "TCC_EA0_ATOMIC_sum", 58.0)])
    bench.summarize_counters("zipf3", k, 100, str(out), str(a), str(b))
    rows = {ln.split()[0]: ln.split()[1:] for ln in out.read_text().splitlines()
            if ln and not ln.startswith("#") and ":" not in ln and not ln.startswith("counter")}
    assert rows["SQ_INSTS_VALU"] == ["2", "1000.0", "10.0000"]
    assert rows["TCC_EA0_ATOMIC_sum"] == ["1", "58.0", "0.5800"]


def test_stale_traffic_is_not_reported(bench, tmp_path, monkeypatch):
    f = tmp_path / "t.txt"
    f.write_text(f"kernel_source_sha256_16: {bench.kernel_source_hash()}\n"
                 "hbm_bytes_per_launch: 1234\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() == 1234.0
    f.write_text("kernel_source_sha256_16: 0000000000000000\nhbm_bytes_per_launch: 1234\n")
    assert bench.measured_traffic() is None
