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
    assert bench.win_kernel_name(32, 3) == "k_mttkrp_win<16, 2, float, 3, false, true, false, false, 1>"
    assert bench.win_kernel_name(16, 4, "uint16_t", False, False) == \
        "k_mttkrp_win<16, 1, uint16_t, 4, false, false, false, false, 2>"
    assert bench.win_kernel_name(64, 3, big=True) == \
        "k_mttkrp_win<16, 4, float, 3, true, true, false, false, 1>"
    assert bench.win_kernel_name(32, 4, "unsigned short") == \
        "k_mttkrp_win<16, 2, unsigned short, 4, false, true, false, true, 1>"
    assert bench.win_kernel_name(33, 4, "unsigned short") == \
        "k_mttkrp_win<16, 4, unsigned short, 4, false, true, false, false, 1>"
    assert bench.win_kernel_name(32, 6, stash=False) == \
        "k_mttkrp_win<16, 2, float, 6, false, false, false, false, 1>"
    assert bench.win_kernel_name(64, 4, stash=False) == \
        "k_mttkrp_win<16, 4, float, 4, false, false, false, false, 4>"
    assert bench.win_kernel_name(100, 4, stash=False) == \
        "k_mttkrp_win<64, 2, float, 4, false, false, false, false, 1>"
    assert bench.short_kernel_name(32, 4) == "k_mttkrp_short<2, float, 4, false, false>"
    assert bench.short_kernel_name(32, 4, "unsigned short") == \
        "k_mttkrp_short<2, unsigned short, 4, false, true>"
    assert bench.short_kernel_name(33, 3, "unsigned short") == \
        "k_mttkrp_short<4, unsigned short, 3, false, false>"


def test_kernel_names_exist_in_the_library(bench):
    """The names the bench reads counters and statistics by are the library's kernels."""
    so = os.path.join(ROOT, "paper_2201_12523_amd", "libblco.so")
    if not os.path.exists(so):
        pytest.skip("library not built")
    syms = subprocess.run(["nm", "-C", so], capture_output=True, text=True, check=True).stdout
    names = set()
    for line in syms.splitlines():
        if line.endswith("(blco::KParams)") or line.endswith("(blco::KParams, long)"):
            names.add(line.split(" ", 2)[2].removeprefix("void ").split("(")[0])
    for R in (16, 32, 33, 64, 100):
        for N in (3, 4, 6):
            for ft in ("float", "unsigned short"):
                for stash in (True, False):
                    assert bench.win_kernel_name(R, N, ft, False, stash) in names
                assert bench.short_kernel_name(R, N, ft) in names


def test_counters_traffic_and_atomics(bench, tmp_path):
    """Per-dispatch means per kernel, the copy-calibrated HBM traffic and the row-ops derived
    from TCC_EA0_ATOMIC with the probe kernel as the per-row-op reference."""
    k = "void " + bench.win_kernel_name(32, 4, stash=False) + "(blco::KParams)"
    probe = "k_atomic_probe(float*, long, unsigned int const*, long, int)"
    fetch, write, atom, out = (tmp_path / x for x in ("f.csv", "w.csv", "a.csv", "c.txt"))
    # two MTTKRP dispatches (mean 300 KiB fetched), a small copy and the 1 MiB
    # calibration copy that the counter reports as 512 KiB fetched, 1024 written
    write_csv(fetch, [(k, "FETCH_SIZE", 200.0), (k, "FETCH_SIZE", 400.0),
                      ("copyBuffer small", "FETCH_SIZE", 3.0),
                      ("copyBuffer big", "FETCH_SIZE", 512.0)])
    write_csv(write, [(k, "WRITE_SIZE", 100.0), (k, "WRITE_SIZE", 100.0),
                      ("copyBuffer big", "WRITE_SIZE", 1024.0)])
    # the probe makes 1000 row-ops and the counter reads 2 requests per row-op
    write_csv(atom, [(k, "TCC_EA0_ATOMIC_sum", 500.0), (probe, "TCC_EA0_ATOMIC_sum", 2000.0)])
    bench.summarize_counters(str(out), "test", str(fetch), str(write), str(atom),
                             copy_bytes=1 << 20, probe_row_ops=1000, commands=["cmd a"])
    c = bench.read_counters(str(out))
    assert c is not None
    head, per = c
    assert per[k]["FETCH_SIZE"] == pytest.approx(300.0)
    name = bench.win_kernel_name(32, 4, stash=False)
    tr = bench.counter_traffic(c, name)
    assert tr["fetch_scale"] == pytest.approx(2.0) and tr["write_scale"] == pytest.approx(1.0)
    assert tr["bytes"] == pytest.approx(300 * 1024 * 2 + 100 * 1024)
    ro = bench.counter_row_ops(c, name)
    assert ro["requests_per_row_op"] == pytest.approx(2.0)
    assert ro["row_ops"] == pytest.approx(250.0)
    assert bench.counter_traffic(c, "k_other") is None


def test_stale_counters_are_not_used(bench, tmp_path):
    f = tmp_path / "t.txt"
    f.write_text(f"kernel_source_sha256_16: {bench.kernel_source_hash()}\n"
                 "calibration_copy_bytes: 1\nprobe_row_ops: 1\nk | FETCH_SIZE | 1 | 5.0\n")
    assert bench.read_counters(str(f)) is not None
    f.write_text("kernel_source_sha256_16: 0000000000000000\nk | FETCH_SIZE | 1 | 5.0\n")
    assert bench.read_counters(str(f)) is None


def test_big_factor_rule(bench):
    # 2^24 x 64 fp32 = 4 GiB: the window kernel's fp32 gathers at 33-64 ranks reach it with
    # 32-bit offsets, buffer loads (hierarchical kernel) take 64-bit addresses; one row more
    # and every kernel does
    dims = (1 << 24, 1 << 22, 1 << 20, 1 << 10)
    assert not any(bench.big_factors(dims, 64, 4, n) for n in range(4))
    assert [bench.big_factors(dims, 64, 4, n, window=False) for n in range(4)] == \
        [False, True, True, True]
    past = ((1 << 24) + 1,) + dims[1:]
    assert [bench.big_factors(past, 64, 4, n) for n in range(4)] == [False, True, True, True]
    assert not any(bench.big_factors(dims, 32, 4, n) for n in range(4))
    assert not any(bench.big_factors(dims, 64, 2, n) for n in range(4))
    # bf16 at 128 ranks: 4 GiB through packed buffer loads, which stop one byte short
    assert [bench.big_factors(dims, 128, 2, n) for n in range(4)] == [False, True, True, True]


def test_request_model(bench, tmp_path):
    """L2 read misses priced at the gather probe's rate plus atomics at the atomic probe's."""
    name = bench.win_kernel_name(32, 4)
    k = "void " + name + "(blco::KParams)"
    gp = "k_gather_probe(float const*, long, unsigned int const*, long, int, float*)"
    f, out = tmp_path / "m.csv", tmp_path / "c.txt"
    # 3500 misses of which 500 are the kernel's memory-side atomics
    write_csv(f, [(k, "TCC_MISS_sum", 3500.0), (k, "TCC_MISS_sum", 3500.0),
                  (k, "TCC_EA0_ATOMIC_sum", 500.0), (gp, "TCC_MISS_sum", 1000.0)])
    bench.summarize_counters(str(out), "test", str(f), copy_bytes=1 << 20, probe_row_ops=1000)
    c = bench.read_counters(str(out))
    # the probe makes 1000 misses in 1 ms: 3000 misses take 3 ms, plus 4 ms of atomics
    m = bench.request_model(c, name, 10.0, {"bound_ms": 4.0}, {"ms": 1.0})
    assert m["miss_ms"] == pytest.approx(3.0) and m["overlap_ms"] == pytest.approx(4.0)
    assert m["serial_ms"] == pytest.approx(7.0) and m["frac"] == pytest.approx(0.7)
    assert bench.request_model(c, name, 10.0, {"bound_ms": None}, {"ms": 1.0}) is None
    assert bench.request_model(None, name, 10.0, {"bound_ms": 4.0}, {"ms": 1.0}) is None


def test_summaries_of_bench_and_sweep_lines(bench, tmp_path):
    """The markdown summaries carry the line's figures: value, roofline with traffic,
    atomics and request pricing, per-configuration times, errors and secondary legs."""
    import json

    roof = {"bound": "hbm", "kernel": "k", "modes": [0], "avg_kernel_ms": 2.0,
            "algorithmic_bytes_per_launch": 4e9, "achieved": 2000.0, "frac": 0.25,
            "traffic": 8e9, "traffic_over_algorithmic": 2.0,
            "atomics": {"row_ops_per_launch": 1e6, "frac": 0.5},
            "request_model": {"miss_ms": 0.5, "atomic_ms": 1.0, "serial_ms": 1.5, "frac": 0.75}}
    line = {"metric": "m", "value": 12.5, "unit": "Gnnz/s", "ms_per_step": 8.0,
            "config": {"workload": "w: shape"}, "roofline": roof,
            "per_config": {"R32_fp32": {"ms_per_step": 8.0, "gnnz_s": 12.5, "kernel_ms": [2.0],
                                        "resolution": ["register"]}},
            "errors": {"R32_fp32": {"max": 1.5e-7}},
            "secondary": {"oom": {"value": 3.0, "unit": "Gnnz/s", "ms_per_step": 100.0,
                                  "roofline": {"bound": "pcie", "achieved": 50.0}}}}
    j = tmp_path / "b.json"
    j.write_text("progress text\n" + json.dumps(line) + "\n")
    out = tmp_path / "b.md"
    bench.summarize_bench(str(out), "test", str(j), "python3 bench.py")
    md = out.read_text()
    for want in ("12.500 Gnnz/s", "0.250 of 8 TB/s", "counter traffic 8.00 GB", "(2.0x)",
                 "atomic row-updates 1.0M = 0.50", "= 1.50 ms = 0.75", "R32_fp32: 8.000 ms",
                 "R32_fp32 1.50e-07", "## secondary: oom", "host link: 50.0 GB/s"):
        assert want in md, want
    sweep = {"rank": 32, "cus": 256, "rows": [
        {"I": 4, "register_ms": 1.2, "hierarchical_ms": 1.0, "auto": "hierarchical"},
        {"I": 512, "register_ms": 0.9, "hierarchical_ms": None, "auto": "register"}]}
    j2, out2 = tmp_path / "s.json", tmp_path / "s.md"
    j2.write_text(json.dumps(sweep) + "\n")
    bench.summarize_sweep(str(out2), str(j2), "python3 bench.py --resolution-sweep")
    md2 = out2.read_text()
    assert "| 4 | 1.200 | 1.000 | 1.20 | hierarchical |" in md2
    assert "| 512 | 0.900 | - | - | register |" in md2
    skew = {"updates": 4, "table_rows": 16, "rank": 32, "results": [
        {"rows": "uniform", "ms": 0.5, "row_updates_per_s": 8e9, "most_updates_on_one_row": 1}]}
    j3, out3 = tmp_path / "k.json", tmp_path / "k.md"
    j3.write_text(json.dumps(skew) + "\n")
    bench.summarize_skew(str(out3), str(j3), "python3 bench.py --atomic-skew")
    assert "| uniform | 0.500 | 8.00G | 1 |" in out3.read_text()
