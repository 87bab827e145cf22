"""Benchmark: BLCO sparse MTTKRP on one MI355X.

Default run (no ``--workload``): the headline is the 4-mode workload on which
the metric's fp32-versus-bf16 factor comparison is quoted:

  zipf4    2^24 x 2^22 x 2^20 x 2^10 (76-bit index, blocked on its top 12 bits),
           200M distinct non-zeros, Zipf(1.2) indices on modes 1-2, uniform on
           modes 3-4, lognormal(0,1) values.  `value` is R = 32 with fp32
           factors: MTTKRP in all four modes from one BLCO copy, Gnnz/s per
           mode-MTTKRP; R = 32 bf16 and R = 64 fp32 / bf16 are reported beside it.

and the other workloads are reported in the same JSON line under ``secondary``:

  zipf3    3-mode 2^22 x 2^21 x 2^20 (63 bits, one block), 50M, Zipf(1.1), R = 32;
  cpgrad4  sparse CP loss + gradient step, 4-mode 2^20 x 2^18 x 2^16 x 2^12, 80M
           non-zeros holding a planted rank-8 model plus noise, R = 32;
  oom3     3-mode 2^23 x 2^23 x 2^17, 1.5B non-zeros in pinned host memory,
           streamed under an 8 GB device budget (per-mode passes and one pass
           for all modes; copy/compute overlap).  Skipped, with the reason in
           the line, when the run is already past its time budget.

A step is one MTTKRP per mode (output zero-fill included); inputs are resident
in device memory before timing starts (pinned host memory for oom3).  Every
time is from HIP events on the stream the library launches on.

``roofline`` describes the kernel that takes the most time in the headline
step.  `achieved` is its ALGORITHMIC (compulsory) HBM bytes per launch,
12*nnz + sum_{m != n} U_m*R*s_f + I_n*R*4 (U_m: distinct mode-m indices), over
its mean launch time; `frac` divides that by the 8 TB/s HBM peak.  `traffic`
is the HBM bytes per launch measured by FETCH_SIZE/WRITE_SIZE counters
(committed under profiles/, copy-calibrated), null when those counters were
taken on other kernel sources.  `atomics` prices the memory-side atomic
row-updates the kernel issues (counter-measured) at the rate of a distinct-row
atomic calibration kernel timed in this run.

Single legs: ``--workload zipf3|zipf4|uniform3|short4|small|oom3|cpgrad4|cpals4``.
Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MTTKRP Gnnz/s per mode & % HBM peak; bf16 vs fp32 factors at stated rel error"
def counters_file(workload):
    """The committed rocprofv3 counter summary of a workload's MTTKRP kernels."""
    return os.path.join(ROOT, "profiles", f"counters_mttkrp_{workload}.txt")


COUNTERS_FILE = counters_file("zipf4")
T_START = time.time()


def log(msg):
    print(f"[bench {time.time() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """First 16 hex digits of the SHA-256 of the kernel sources' code: comments, blank
    lines and trailing blanks are removed first, so a summary of counters taken on a
    kernel stays valid across edits of its comments, and no longer after any other."""
    import re

    h = hashlib.sha256()
    for f in ("blco_device.hip", "blco_kernels.h"):
        with open(os.path.join(ROOT, "paper_2201_12523_amd", "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()[:16]


class Timer:
    """Average milliseconds of `fn` over `steps` calls: `warmup` untimed calls, a
    synchronisation, HIP events around the timed calls on torch's current stream
    (the stream the library launches on), and a synchronisation."""

    def __init__(self, torch):
        self.torch = torch

    def __call__(self, fn, steps, warmup=1):
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / max(steps, 1)


# --------------------------------------------------------------------------- CPU baseline

def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_oracle_baseline(oracle, coords, vals, A, modes, sample_1t, sample_all):
    """The fp64 oracle as it stands, over a bounded prefix of the workload's non-zeros,
    every mode: the serial oracle on one thread, and its OpenMP form on every thread the
    process may use (OMP_NUM_THREADS).  `value` is the all-core rate."""
    Ad = [a.astype(np.float64) for a in A]
    dims = [a.shape[0] for a in A]

    def run(S, omp):
        cs = [np.ascontiguousarray(c[:S]) for c in coords]
        v = vals[:S].astype(np.float64)
        used, atomic = 1, False
        t0 = time.time()
        for n in modes:
            if omp:
                _, _, used, at = oracle.mttkrp_omp(cs, v, Ad, n, dims=dims, with_scale=False)
                atomic = atomic or at
            else:
                oracle.mttkrp(cs, v, Ad, n, dims=dims, with_scale=False)
        return time.time() - t0, used, atomic

    s1 = min(sample_1t, len(vals))
    dt1, _, _ = run(s1, False)
    log(f"cpu oracle, 1 thread: {s1} non-zeros x {len(modes)} modes in {dt1:.1f}s")
    sa = min(sample_all, len(vals))
    dta, used, atomic = run(sa, True)
    log(f"cpu oracle, {used} threads: {sa} non-zeros x {len(modes)} modes in {dta:.1f}s")
    return {"value": sa * len(modes) / dta / 1e9, "unit": "Gnnz/s", "cores": used,
            "kind": "oracle",
            "sample": f"first {sa} non-zeros of the workload, all {len(modes)} modes, fp64 "
                      f"oracle on {used} threads ({'atomic' if atomic else 'private'} outputs), "
                      f"{dta:.1f}s",
            "single_thread": {"value": s1 * len(modes) / dt1 / 1e9, "unit": "Gnnz/s",
                              "sample": f"first {s1} non-zeros, all {len(modes)} modes, "
                                        f"serial fp64 oracle, {dt1:.1f}s"},
            "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count(),
                     "usable_cores": len(os.sched_getaffinity(0)),
                     "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}}


# --------------------------------------------------------------------------- counters

def read_counters(path=COUNTERS_FILE):
    """{kernel: {counter: mean per dispatch}} and the header fields of a committed
    counter summary, or None when it is missing or was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    head, per = {}, {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            if " | " in line:
                k, c, _, v = [x.strip() for x in line.split(" | ")]
                per.setdefault(k, {})[c] = float(v)
            elif ":" in line:
                a, b = line.split(":", 1)
                head[a.strip()] = b.strip()
    if head.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return head, per


def _kernel_entry(per, name):
    for k, v in per.items():
        if k == name or k.startswith(name + "(") or k.startswith("void " + name + "("):
            return v
    return None


def counter_traffic(counters, kernel):
    """HBM bytes per launch of `kernel`: FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by calibration_copy_bytes / (that counter for the calibration copy)."""
    if counters is None:
        return None
    head, per = counters
    k = _kernel_entry(per, kernel)
    cp = per.get("calibration_copy")
    if not k or not cp or "FETCH_SIZE" not in k or "WRITE_SIZE" not in k:
        return None
    nbytes = float(head["calibration_copy_bytes"])
    fs = nbytes / (cp["FETCH_SIZE"] * 1024.0)
    ws = nbytes / (cp["WRITE_SIZE"] * 1024.0)
    return {"bytes": k["FETCH_SIZE"] * 1024.0 * fs + k["WRITE_SIZE"] * 1024.0 * ws,
            "fetch_scale": fs, "write_scale": ws}


def counter_row_ops(counters, kernel):
    """Memory-side atomic row-updates per launch of `kernel`: its TCC_EA0_ATOMIC over
    the same counter per row-update of the calibration probe (known row-ops)."""
    if counters is None:
        return None
    head, per = counters
    k = _kernel_entry(per, kernel)
    pr = _kernel_entry(per, "k_atomic_probe")
    if not k or not pr or "TCC_EA0_ATOMIC_sum" not in k or "TCC_EA0_ATOMIC_sum" not in pr:
        return None
    per_op = pr["TCC_EA0_ATOMIC_sum"] / float(head["probe_row_ops"])
    return {"row_ops": k["TCC_EA0_ATOMIC_sum"] / per_op, "requests_per_row_op": per_op,
            "requests": k["TCC_EA0_ATOMIC_sum"]}


SUMMARY_KERNELS = ("k_mttkrp", "k_atomic_probe", "k_gather_probe", "k_loss_tile")


def summarize_counters(out, title, *csvs, copy_bytes=0, probe_row_ops=0, commands=()):
    """Mean per dispatch of every counter of the MTTKRP, loss and atomic-probe kernels in
    rocprofv3 --pmc CSVs, written as `kernel | counter | dispatches | mean`.  The largest
    device copy is recorded as `calibration_copy` (its size is copy_bytes)."""
    import csv

    vals = {}
    copies = {}
    for path in csvs:
        for r in csv.DictReader(open(path)):
            name, c, v = r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])
            if "copyBuffer" in name:
                copies.setdefault(c, []).append(v)
                continue
            if not any(k in name for k in SUMMARY_KERNELS):
                continue
            vals.setdefault((name, c), []).append(v)
    lines = [f"# {title}", "# rocprofv3 counters, mean per dispatch. Commands, one pass each:"]
    lines += [f"#   {c}" for c in commands]
    lines += [f"kernel_source_sha256_16: {kernel_source_hash()}",
              f"calibration_copy_bytes: {copy_bytes}", f"probe_row_ops: {probe_row_ops}"]
    for (name, c), v in sorted(vals.items()):
        lines.append(f"{name} | {c} | {len(v)} | {float(np.mean(v)):.1f}")
    for c, v in sorted(copies.items()):
        lines.append(f"calibration_copy | {c} | 1 | {max(v):.1f}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_stats(out, title, stats_csv, command):
    """Short text form of a rocprofv3 --stats kernel_stats.csv."""
    import csv

    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# {title}", f"# command: {command}", f"# kernel_source_sha256_16: {kernel_source_hash()}",
             "# name | calls | total ns | average ns | percent | min ns | max ns"]
    for r in rows:
        lines.append(" | ".join([r["Name"], r["Calls"], r["TotalDurationNs"], r["AverageNs"],
                                 f"{float(r['Percentage']):.2f}", r["MinNs"], r["MaxNs"]]))
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines[:20]))


def summarize_overlap(out, title, copy_csv, kernel_csv, per_call_copies, command):
    """Copy/compute overlap of streamed MTTKRP calls from a rocprofv3 --kernel-trace
    --memory-copy-trace run: the host-to-device copies of the library's copy stream (the
    stream with the most copy time) taken in groups of per_call_copies (2 per chunk: keys
    and values), the MTTKRP kernels between one group's first copy and the next group's;
    per call t_copy = sum of its copy times, t_comp = sum of its kernel times, t_total =
    last end - first copy start, overlap = (t_copy + t_comp - t_total) / min(t_copy, t_comp)."""
    import csv

    cps = [r for r in csv.DictReader(open(copy_csv)) if "HOST_TO_DEVICE" in r["Direction"]]
    by_stream = {}
    for r in cps:
        by_stream.setdefault(r["Stream_Id"], []).append((int(r["Start_Timestamp"]),
                                                         int(r["End_Timestamp"])))
    copies = sorted(max(by_stream.values(), key=lambda v: sum(e - b for b, e in v)))
    kern = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                  for r in csv.DictReader(open(kernel_csv)) if "k_mttkrp" in r["Kernel_Name"])
    ncalls = len(copies) // per_call_copies
    lines = [f"# {title}", f"# command: {command}",
             f"# {len(copies)} chunk copies on the library's copy stream, {len(kern)} MTTKRP "
             f"kernels, {per_call_copies} copies per call",
             "# call | copies | kernels | t_copy ms | t_comp ms | t_total ms | overlap"]
    for c in range(ncalls):
        grp = copies[c * per_call_copies:(c + 1) * per_call_copies]
        lo = grp[0][0]
        hi = copies[(c + 1) * per_call_copies][0] if c + 1 < ncalls else float("inf")
        ks = [k for k in kern if lo <= k[0] < hi]
        tc = sum(e - b for b, e in grp) / 1e6
        tk = sum(e - b for b, e in ks) / 1e6
        tt = (max([e for _, e in grp] + [e for _, e in ks]) - lo) / 1e6
        ov = (tc + tk - tt) / min(tc, tk) if ks else float("nan")
        lines.append(f"{c} | {len(grp)} | {len(ks)} | {tc:.1f} | {tk:.1f} | {tt:.1f} | {ov:.3f}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))



def _roofline_text(r):
    if not r:
        return "n/a"
    if r.get("bound") == "pcie":
        return f"bound by the host link: {r['achieved']:.1f} GB/s host-to-device"
    s = (f"dominant kernel `{r['kernel']}` (modes {r['modes']}): {r['avg_kernel_ms']:.3f} ms, "
         f"compulsory {r['algorithmic_bytes_per_launch'] / 1e9:.2f} GB per launch = "
         f"{r['achieved']:.0f} GB/s = {r['frac']:.3f} of 8 TB/s")
    if r.get("traffic"):
        s += (f"; counter traffic {r['traffic'] / 1e9:.2f} GB per launch "
              f"({r['traffic_over_algorithmic']:.1f}x)")
    else:
        s += "; counter traffic null (no counter summary for this kernel source)"
    a = r.get("atomics") or {}
    if a.get("frac") is not None:
        s += (f"; atomic row-updates {a['row_ops_per_launch'] / 1e6:.1f}M = {a['frac']:.2f} of "
              f"the time at the probe's rate")
    m = r.get("request_model")
    if m:
        s += (f"; requests priced at the probes' rates: L2 read misses {m['miss_ms']:.2f} ms + "
              f"atomics {m['atomic_ms']:.2f} ms = {m['serial_ms']:.2f} ms = {m['frac']:.2f} of the "
              f"kernel's time")
    return s


def summarize_bench(out, title, json_path, command):
    """Markdown form of one bench.py JSON line (the last line of json_path): the headline
    leg, its per-configuration figures, errors and CPU baseline, then every secondary leg."""
    d = json.loads(open(json_path).read().strip().splitlines()[-1])
    md = [f"# bench.py, {title} (MI355X, one GPU)", "", "Command (GPU box, repository root):", "",
          f"    {command}", "", f"* workload: {d['config']['workload']}",
          f"* value: {d['value']:.3f} {d['unit']} ({d['metric']}); {d['ms_per_step']:.3f} ms per step"]

    def legs(v, full):
        o = []
        if "roofline" in v:
            o.append(f"* roofline: {_roofline_text(v['roofline'])}")
        for k, c in v.get("per_config", {}).items():
            o.append(f"* {k}: {c['ms_per_step']:.3f} ms per step ({c['gnnz_s']:.2f} Gnnz/s), kernel "
                     f"ms per mode {[round(x, 3) for x in c['kernel_ms']]}"
                     + (f", resolution {c['resolution']}" if full and "resolution" in c else ""))
        if "per_storage" in v:
            o.append("* " + ", ".join(f"{k}: {c['ms_per_step']:.3f} ms per step"
                                      for k, c in v["per_storage"].items()))
        for pm in v.get("per_mode", []):
            o.append(f"* mode {pm['mode'] + 1}: {pm['call_ms']:.1f} ms per call, copy "
                     f"{pm['copy_ms']:.1f} ms, kernels {pm['kernel_ms']:.1f} ms, host-to-device "
                     f"{pm['h2d_gbs']:.1f} GB/s, overlap {pm['overlap']:.3f}, {pm['chunks']} chunks")
        if "one_pass" in v:
            o.append(f"* every mode per chunk: {json.dumps(v['one_pass'])}")
        if "errors" in v:
            o.append("* max normalised error vs the fp64 oracle: " +
                     ", ".join(f"{k} {e['max']:.2e}" for k, e in v["errors"].items()))
        return o

    md += legs(d, True)
    for k in ("mttkrp_kernel_ms", "mttkrp_share_of_iteration", "fits", "pinv_fallbacks"):
        if k in d:
            v = d[k]
            v = [round(x, 4) for x in v] if isinstance(v, list) else (
                round(v, 4) if isinstance(v, float) else v)
            md.append(f"* {k}: {v}")
    c = d.get("cpu_baseline")
    if c:
        md.append(f"* cpu baseline: {c['value']:.5f} {c['unit']} on {c['cores']} cores "
                  f"({c['sample']}); one thread {c['single_thread']['value']:.5f}")
    if "build_s" in d:
        md.append(f"* construction of the headline tensor: host builder {d['build_s']:.2f} s, GPU "
                  f"builder {d['build_gpu_s'] * 1e3:.1f} ms; wall time of the whole run "
                  f"{d['wall_s']:.0f} s")
    for k, v in d.get("secondary", {}).items():
        md += ["", f"## secondary: {k}", f"* {v.get('config', {}).get('workload', '')}",
               f"* value: {v['value']:.3f} {v['unit']}; {v['ms_per_step']:.3f} ms per step"]
        md += legs(v, False)
    with open(out, "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


def summarize_sweep(out, json_path, command):
    """Markdown table of a --resolution-sweep JSON line."""
    d = json.loads(open(json_path).read().strip().splitlines()[-1])
    md = ["# Conflict resolution vs target-mode length (Sections 5.1-5.3), MI355X, one GPU", "",
          "Command (GPU box, repository root):", "", f"    {command}", "",
          "3-mode 2^21 x 2^17 x I tensors, 50M distinct non-zeros (Zipf(1.1) indices on the two "
          "long modes, uniform on the short one, U(0,1) values), rank "
          f"{d['rank']} fp32 factors; kernel time of the mode-3 (length I) MTTKRP, output "
          "accumulated. The register-based path includes its frequent-row stash (all I rows fit "
          f"for I <= 255). The device reports {d['cus']} compute units; `auto` is the Section 5.3 "
          "choice (hierarchical when I is below the compute-unit count).", "",
          "| I | register ms | hierarchical ms | register / hierarchical | auto |",
          "|---:|---:|---:|---:|---|"]
    for r in d["rows"]:
        h = r.get("hierarchical_ms")
        hs = "-" if h is None else f"{h:.3f}"
        ratio = "-" if h is None else f"{r['register_ms'] / h:.2f}"
        md.append(f"| {r['I']} | {r['register_ms']:.3f} | {hs} | {ratio} | {r['auto']} |")
    with open(out, "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


def summarize_skew(out, json_path, command):
    """Markdown table of an --atomic-skew JSON line."""
    d = json.loads(open(json_path).read().strip().splitlines()[-1])
    md = ["# fp32 atomic row-updates vs row skew (MI355X, one GPU)", "",
          "Command (GPU box, repository root):", "", f"    {command}", "",
          f"The library's atomic probe (`blco_atomic_probe`: one row-update of R = {d['rank']} "
          f"floats by 16 lanes, as the MTTKRP flushes) over {d['updates']} updates of a "
          f"{d['table_rows']}-row fp32 output.", "",
          "| rows | ms | row-updates/s | most updates on one row |", "|---|---:|---:|---:|"]
    for r in d["results"]:
        md.append(f"| {r['rows']} | {r['ms']:.3f} | {r['row_updates_per_s'] / 1e9:.2f}G | "
                  f"{r['most_updates_on_one_row']} |")
    with open(out, "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


# --------------------------------------------------------------------------- helpers

def win_kernel_name(R, N, ft="float", big=False, stash=True):
    """Template name of the window MTTKRP kernel the library launches for rank R
    (stash: the mode's frequent rows are held in LDS)."""
    lpn, rpl = (16, 1) if R <= 16 else (16, 2) if R <= 32 else (16, 4) if R <= 64 else (64, 2)
    b = lambda v: "true" if v else "false"
    # then: the fused CP-gradient walk (never for the plain MTTKRP), vector gathers of
    # packed bf16 ranks (bf16 factors, two or more ranks per lane, even R), and the
    # non-zeros per thread (without a stash at R <= 64 and at most 5 modes: two, four at
    # R > 32)
    vec = ft != "float" and rpl > 1 and R % 2 == 0
    wpt = (4 if rpl == 4 else 2) if (not stash and lpn == 16 and N <= 5) else 1
    return (f"k_mttkrp_win<{lpn}, {rpl}, {ft}, {N}, {b(big)}, {b(stash)}, false, {b(vec)}, "
            f"{wpt}>")


def short_kernel_name(R, N, ft="float", big=False):
    """Template name of the hierarchical MTTKRP kernel for a single rank slice of width R
    (vector gathers of packed bf16 ranks: bf16, two or more ranks per lane, even R)."""
    rpl = 1 if R <= 16 else 2 if R <= 32 else 4
    vec = ft != "float" and rpl > 1 and R % 2 == 0
    b = lambda v: "true" if v else "false"
    return f"k_mttkrp_short<{rpl}, {ft}, {N}, {b(big)}, {b(vec)}>"


def big_factors(dims, R, sf, n, window=True):
    """Whether mode n's MTTKRP gathers with 64-bit addresses, as the library decides: a row
    of 2 GiB or more, or another factor of 4 GiB or more (above 4 GiB for the window
    kernel's fp32 gathers at 33-64 ranks, which reach exactly 4 GiB with 32-bit offsets)."""
    lim = (1 << 32) if (window and sf == 4 and 32 < R <= 64) else 0xFFFFFFFF
    return R * sf >= (1 << 31) or any(d * R * sf > lim for m, d in enumerate(dims) if m != n)


def mode_kernel(T, n, R, N, ft, dims):
    """The kernel one mode's MTTKRP launches (the library's rule, read back)."""
    sf = 4 if ft == "float" else 2
    if T.resolution(n, R) == "hierarchical":
        return short_kernel_name(R, N, ft, big_factors(dims, R, sf, n, window=False))
    return win_kernel_name(R, N, ft, big_factors(dims, R, sf, n), stash=T.stash_rows(n, R) > 0)


def describe(w, nnz):
    dist = "/".join(f"{d[0]}({d[1]})" if d[0] == "zipf" else d[0] for d in w.index_dist)
    vals = {"u01": "U(0,1)", "lognormal": "lognormal(0,1)", "cp8": "rank-8 CP model + N(0,0.01)"}
    return (f"{w.name}: {len(w.dims)}-mode {'x'.join(str(d) for d in w.dims)}, {nnz} distinct "
            f"non-zeros, per-mode {dist} indices, {vals[w.value_dist]} values, ranks "
            f"{'/'.join(str(r) for r in w.ranks)}")


def base_result(args, w, nnz, value, ms_step, dtype="f32"):
    return {
        "metric": METRIC, "value": value, "unit": "Gnnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": describe(w, nnz), "nnz": nnz, "dims": list(w.dims),
                   "modes": len(w.dims)},
    }


def check_rows_for(counts, I, rng, k=48):
    """Rows compared with the oracle: the 16 most frequent, rows 0-7, k random, the last."""
    hot = np.argsort(-counts, kind="stable")[:16]
    return np.unique(np.concatenate([hot, np.arange(min(8, I)), rng.integers(0, I, k), [I - 1]])
                     ).astype(np.uint32)


def atomic_calibration(torch, blco, R, steps, rows=1 << 22):
    """Distinct-row fp32 atomic rate: one row-update (R floats by 16-lane groups, the
    MTTKRP flush) on each row of a rows x R output, in a random order."""
    dev = torch.device("cuda:0")
    out = torch.zeros((rows, R), dtype=torch.float32, device=dev)
    g = torch.Generator(device="cpu").manual_seed(12523)
    ids = torch.randperm(rows, generator=g).to(torch.int32).to(dev)
    ms = Timer(torch)(lambda: blco.atomic_probe(out, ids), steps, 2)
    del out, ids
    return {"rows": rows, "rank": R, "ms": ms, "row_ops_per_s": rows / (ms * 1e-3)}


def gather_calibration(torch, blco, R, steps, rows=1 << 22):
    """Random-row gather rate: every row of a rows x R fp32 table read once, in a random
    order, by 16-lane groups with six rows per group in flight (the MTTKRP gathers)."""
    dev = torch.device("cuda:0")
    table = torch.rand((rows, R), dtype=torch.float32, device=dev)
    g = torch.Generator(device="cpu").manual_seed(2201)
    ids = torch.randperm(rows, generator=g).to(torch.int32).to(dev)
    sink = torch.empty(((rows + 5) // 6,), dtype=torch.float32, device=dev)
    ms = Timer(torch)(lambda: blco.gather_probe(table, ids, sink), steps, 2)
    del table, ids, sink
    return {"rows": rows, "rank": R, "ms": ms, "rows_per_s": rows / (ms * 1e-3)}


def counter_of(counters, kernel, counter):
    """Mean per dispatch of one counter of one kernel in a counter summary, or None."""
    if counters is None:
        return None
    k = _kernel_entry(counters[1], kernel)
    return k.get(counter) if k else None


def request_model(counters, kernel, kernel_ms, atomics, gcal):
    """A kernel's time priced by its memory-side requests: its L2 read misses (TCC_MISS
    less the memory-side atomics, which L2 also counts as misses) at the rate the gather
    probe makes them (the probe's TCC_MISS per dispatch over its live time), and its
    atomic row-updates at the atomic probe's rate.  serial_ms is their sum (the two kinds
    of request served one after the other), overlap_ms the larger (served side by side);
    frac = serial_ms / kernel time."""
    miss = counter_of(counters, kernel, "TCC_MISS_sum")
    atom = counter_of(counters, kernel, "TCC_EA0_ATOMIC_sum") or 0.0
    pmiss = counter_of(counters, "k_gather_probe", "TCC_MISS_sum")
    if miss is None or not pmiss or atomics.get("bound_ms") is None:
        return None
    miss = max(miss - atom, 0.0)
    miss_rate = pmiss / (gcal["ms"] * 1e-3)
    miss_ms = miss / miss_rate * 1e3
    serial = miss_ms + atomics["bound_ms"]
    return {"gather_calibration": gcal, "l2_read_misses_per_launch": miss,
            "probe_l2_misses_per_s": miss_rate, "miss_ms": miss_ms,
            "atomic_ms": atomics["bound_ms"], "serial_ms": serial,
            "overlap_ms": max(miss_ms, atomics["bound_ms"]), "frac": serial / kernel_ms}


# --------------------------------------------------------------------------- legs

def leg_inmemory(args, torch, blco, synth, w, *, check=True, cpu=False, gpu_build=True,
                 headline=False):
    dev = torch.device("cuda:0")
    timer = Timer(torch)
    t0 = time.time()
    coords, vals = synth.workload_tensor(w, nnz=args.nnz, log=log)
    nnz = len(vals)
    log(f"{w.name}: generated {nnz} non-zeros in {time.time() - t0:.1f}s")
    t0 = time.time()
    T = blco.build(coords, vals, w.dims)
    build_s = time.time() - t0
    inf = T.info()
    log(f"{w.name}: built BLCO in {build_s:.2f}s: T={inf['total_bits']} bits, "
        f"{inf['nblocks']} block(s), {inf['nruns']} run(s)")
    build_gpu = None
    if gpu_build:
        # the same construction on the GPU, from device-resident coordinates and values
        dc = [torch.from_numpy(c.view(np.int32)).to(dev) for c in coords]
        dv = torch.from_numpy(vals).to(dev)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.time()
            Tg = blco.build_device(dc, dv, w.dims)
            torch.cuda.synchronize()
            times.append(time.time() - t0)
            Tg.free()
        del dc, dv
        build_gpu = min(times)
        log(f"{w.name}: built BLCO on the GPU in {build_gpu * 1e3:.1f} ms")
    N = len(w.dims)
    modes = list(range(N))
    counts = [np.bincount(c, minlength=d) for c, d in zip(coords, w.dims)]
    distinct = [int(np.count_nonzero(c)) for c in counts]
    results = {}
    keep = {}
    for R in w.ranks:
        A = synth.workload_factors(w, R)
        F32 = [torch.from_numpy(a).to(dev) for a in A]
        BF16 = [blco.cast_bf16(f) for f in F32]
        outs = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in w.dims]
        torch.cuda.synchronize()
        for tag, F in (("fp32", F32), ("bf16", BF16)):
            def step(F=F, outs=outs):
                for n in modes:
                    blco.mttkrp(T, n, F, out=outs[n])
            ms_step = timer(step, args.steps, args.warmup)
            call = [timer(lambda n=n: blco.mttkrp(T, n, F, out=outs[n]), args.steps)
                    for n in modes]
            kern = [timer(lambda n=n: blco.mttkrp_acc(T, n, F, outs[n]), args.steps)
                    for n in modes]
            sf = 4 if tag == "fp32" else 2
            ft = "float" if tag == "fp32" else "unsigned short"
            names = [mode_kernel(T, n, R, N, ft, w.dims) for n in modes]
            compulsory = [12 * nnz + sum(distinct[m] * R * sf for m in modes if m != n) +
                          w.dims[n] * R * 4 for n in modes]
            alt = {}
            for n in modes:
                if T.resolution(n, R) == "hierarchical":
                    # the other mechanism on the same mode, for the Section 5.3 comparison
                    T.set_resolution("register")
                    alt[n] = timer(lambda n=n: blco.mttkrp_acc(T, n, F, outs[n]), args.steps)
                    T.set_resolution("auto")
            results[f"R{R}_{tag}"] = {
                "ms_per_step": ms_step, "gnnz_s": nnz * N / (ms_step * 1e-3) / 1e9,
                "resolution": [T.resolution(n, R) for n in modes],
                "register_kernel_ms_on_hierarchical_modes": {str(n): v for n, v in alt.items()},
                "call_ms": call, "kernel_ms": kern, "kernel": names,
                "per_mode_gnnz_s": [nnz / (x * 1e-3) / 1e9 for x in call],
                "compulsory_bytes": compulsory,
                "per_mode_hbm_frac": [b / (x * 1e-3) / 1e9 / HBM_PEAK_GBS
                                      for b, x in zip(compulsory, kern)],
                "requested_bytes_rate_gbs": [nnz * (12 + (N - 1) * R * sf) / (x * 1e-3) / 1e9
                                             for x in kern],
            }
            log(f"{w.name} R={R} {tag}: all-mode step {ms_step:.3f} ms, kernel ms/mode "
                f"{[round(x, 3) for x in kern]}, compulsory-HBM fraction "
                f"{[round(f, 3) for f in results[f'R{R}_{tag}']['per_mode_hbm_frac']]}")
        keep[R] = (A, F32, BF16, outs)
        if R != w.ranks[0]:
            del keep[R]
            del F32, BF16, outs
            torch.cuda.empty_cache()
    R = w.ranks[0]
    head = results[f"R{R}_fp32"]
    res = base_result(args, w, nnz, head["gnnz_s"], head["ms_per_step"])
    res["config"].update({"rank": R, "factors": "fp32", "key_bits": inf["total_bits"],
                          "blocks": inf["nblocks"], "runs": inf["nruns"]})
    # the kernel that takes the most time in the step, over the modes that launch it
    tot = {}
    for n in modes:
        tot.setdefault(head["kernel"][n], []).append(n)
    dom = max(tot, key=lambda k: sum(head["kernel_ms"][n] for n in tot[k]))
    dm = tot[dom]
    avg_ms = float(np.mean([head["kernel_ms"][n] for n in dm]))
    alg = float(np.mean([head["compulsory_bytes"][n] for n in dm]))
    achieved = alg / (avg_ms * 1e-3) / 1e9
    counters = read_counters(counters_file(w.name)) if args.nnz is None else None
    traffic = counter_traffic(counters, dom)
    calib = atomic_calibration(torch, blco, R, args.steps)
    rops = counter_row_ops(counters, dom)
    atomics = {"calibration": calib, "row_ops_per_launch": rops["row_ops"] if rops else None,
               "requests_per_row_op": rops["requests_per_row_op"] if rops else None,
               "bound_ms": rops["row_ops"] / calib["row_ops_per_s"] * 1e3 if rops else None}
    atomics["frac"] = atomics["bound_ms"] / avg_ms if rops else None
    gcal = gather_calibration(torch, blco, R, args.steps)
    res["roofline"] = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic["bytes"] if traffic else None,
        "kernel": dom, "modes": dm, "avg_kernel_ms": avg_ms,
        "algorithmic_bytes_per_launch": alg,
        "bytes_model": "compulsory: 12 B per non-zero (key + value) + each distinct row of the "
                       "other modes' factors once (U_m*R*s_f) + the output once (I_n*R*4)",
        "traffic_over_algorithmic": traffic["bytes"] / alg if traffic else None,
        "traffic_scales": [traffic["fetch_scale"], traffic["write_scale"]] if traffic else None,
        "all_modes_frac": sum(head["compulsory_bytes"]) / (sum(head["kernel_ms"]) * 1e-3) / 1e9
                          / HBM_PEAK_GBS,
        "atomics": atomics,
        "request_model": request_model(counters, dom, avg_ms, atomics, gcal),
    }
    log(f"{w.name}: dominant kernel {dom} (modes {dm}): {avg_ms:.3f} ms, {achieved:.0f} GB/s "
        f"compulsory = {achieved / HBM_PEAK_GBS:.3f} of HBM peak; atomics {atomics}")
    res["per_config"] = results
    res["distinct_indices"] = distinct
    res["build_s"] = build_s
    res["build_gpu_s"] = build_gpu
    res["cpu_baseline"] = None
    if check:
        import oracle

        rng = np.random.default_rng(7)
        errs = {}
        v64 = vals.astype(np.float64)   # the threaded row oracle takes fp64 values
        for R in w.ranks:
            if R in keep:
                A, F32, BF16, outs = keep[R]
            else:
                A = synth.workload_factors(w, R)
                F32 = [torch.from_numpy(a).to(dev) for a in A]
                BF16 = [blco.cast_bf16(f) for f in F32]
                outs = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in w.dims]
            Ab = [oracle.bf16_round(a) for a in A]
            e = {"fp32": [], "bf16": [], "bf16_vs_fp32": []}
            for n in modes:
                rows = check_rows_for(counts[n], w.dims[n], rng)
                ridx = torch.from_numpy(rows.astype(np.int64)).to(dev)
                M32, S32 = oracle.mttkrp_rows_omp(coords, v64, A, n, rows, w.dims)
                Mb, Sb = oracle.mttkrp_rows_omp(coords, v64, Ab, n, rows, w.dims)
                g32 = blco.mttkrp(T, n, F32, out=outs[n])[ridx].cpu().numpy().astype(np.float64)
                gb = blco.mttkrp(T, n, BF16, out=outs[n])[ridx].cpu().numpy().astype(np.float64)
                for key, got, M, S in (("fp32", g32, M32, S32), ("bf16", gb, Mb, Sb),
                                       ("bf16_vs_fp32", gb, M32, S32)):
                    nz = S > 0
                    e[key].append(np.abs(got - M)[nz] / S[nz])
                log(f"{w.name} R={R} mode {n}: {len(rows)} rows checked against the oracle")
            for key, v in e.items():
                a = np.concatenate(v)
                errs[f"R{R}_{key}"] = {"max": float(a.max()), "median": float(np.median(a))}
            del F32, BF16, outs
        res["errors"] = errs
        log(f"{w.name}: errors {errs}")
    if cpu:
        import oracle

        A = keep[w.ranks[0]][0]
        res["cpu_baseline"] = cpu_oracle_baseline(oracle, coords, vals, A, modes,
                                                  args.cpu_sample_nnz, args.cpu_sample_all_nnz)
    T.free()
    return res


def leg_oom(args, torch, blco, synth, w, *, check=True, cpu=False):
    dev = torch.device("cuda:0")
    timer = Timer(torch)
    t0 = time.time()
    coords, vals = synth.workload_tensor(w, nnz=args.nnz, log=log)
    nnz = len(vals)
    log(f"{w.name}: generated {nnz} non-zeros in {time.time() - t0:.1f}s")
    t0 = time.time()
    T = blco.build(coords, vals, w.dims, placement="pinned")
    build_s = time.time() - t0
    log(f"{w.name}: built pinned BLCO in {build_s:.1f}s")
    N = len(w.dims)
    modes = list(range(N))
    R = w.ranks[0]
    A = synth.workload_factors(w, R)
    F = [torch.from_numpy(a).to(dev) for a in A]
    outs = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in w.dims]
    budget = args.budget or w.budget_bytes
    steps, warm = (min(args.steps, 3), min(args.warmup, 1)) if not args.workload else \
        (args.steps, args.warmup)

    def overlap(c, k, t):
        return (c + k - t) / max(min(c, k), 1e-9)

    per = []
    for n in modes:
        ms = timer(lambda n=n: blco.mttkrp_stream(T, n, F, out=outs[n], device_budget=budget),
                   steps, warm)
        inf = T.info()
        c, k, t = inf["stream_copy_ms"], inf["stream_kernel_ms"], inf["stream_total_ms"]
        per.append({"mode": n, "call_ms": ms, "overall_gnnz_s": nnz / (ms * 1e-3) / 1e9,
                    "in_memory_gnnz_s": nnz / (k * 1e-3) / 1e9,
                    "h2d_gbs": nnz * 12 / (c * 1e-3) / 1e9, "copy_ms": c, "kernel_ms": k,
                    "total_ms": t, "overlap": overlap(c, k, t), "chunks": inf["stream_chunks"],
                    "chunk_nnz": inf["stream_chunk_nnz"],
                    "peak_device_bytes": inf["stream_peak_bytes"]})
        log(f"{w.name} mode {n}: {ms:.1f} ms/call, copy {c:.1f} ms, kernels {k:.1f} ms, span "
            f"{t:.1f} ms, overlap {per[-1]['overlap']:.3f}, {inf['stream_chunks']} chunks")
    ms_modes = sum(p["call_ms"] for p in per)
    ms_step = timer(lambda: blco.mttkrp_stream_all(T, F, outs=outs, device_budget=budget),
                    steps, warm)
    inf = T.info()
    c, k, t = inf["stream_copy_ms"], inf["stream_kernel_ms"], inf["stream_total_ms"]
    one = {"call_ms": ms_step, "overall_gnnz_s": nnz * N / (ms_step * 1e-3) / 1e9,
           "copy_ms": c, "kernel_ms": k, "total_ms": t, "overlap": overlap(c, k, t),
           "h2d_gbs": nnz * 12 / (c * 1e-3) / 1e9, "chunks": inf["stream_chunks"],
           "peak_device_bytes": inf["stream_peak_bytes"]}
    log(f"{w.name} all modes in one pass: {ms_step:.1f} ms/call, copy {c:.1f} ms, kernels "
        f"{k:.1f} ms, overlap {one['overlap']:.3f}")
    res = base_result(args, w, nnz, nnz * N / (ms_step * 1e-3) / 1e9, ms_step)
    res["steps"], res["warmup"] = steps, warm
    res["per_mode_passes_ms_per_step"] = ms_modes
    res["per_mode_passes_gnnz_s"] = nnz * N / (ms_modes * 1e-3) / 1e9
    res["one_pass"] = one
    res["per_mode"] = per
    res["config"].update({"rank": R, "device_budget_bytes": budget, "placement": "pinned"})
    res["roofline"] = {
        "bound": "pcie", "achieved": one["h2d_gbs"], "unit": "GB/s",
        "note": "the streamed step is bound by the host-to-device copies (12 B per non-zero "
                "per pass); the in-memory kernels are reported in per_mode kernel_ms",
    }
    res["build_s"] = build_s
    res["cpu_baseline"] = None
    if check:
        import oracle

        rng = np.random.default_rng(7)
        worst = 0.0
        v64 = vals.astype(np.float64)   # the threaded row oracle takes fp64 values
        for n in modes:
            o = blco.mttkrp_stream(T, n, F, out=outs[n], device_budget=budget)
            rows = np.unique(np.concatenate([np.arange(8), rng.integers(0, w.dims[n], 24),
                                             [w.dims[n] - 1]])).astype(np.uint32)
            M, S = oracle.mttkrp_rows_omp(coords, v64, A, n, rows, w.dims)
            got = o[torch.from_numpy(rows.astype(np.int64)).to(dev)].cpu().numpy()
            nz = S > 0
            worst = max(worst, float((np.abs(got - M)[nz] / S[nz]).max()))
        res["errors"] = {"fp32": {"max": worst}}
        log(f"{w.name}: max normalised error {worst:.2e}")
    if cpu:
        import oracle

        res["cpu_baseline"] = cpu_oracle_baseline(oracle, coords, vals, A, modes,
                                                  args.cpu_sample_nnz, args.cpu_sample_all_nnz)
    T.free()
    return res


def planted_values(torch, coords, G, sigma, seed, synth, chunk=8_000_000):
    """x_k = sum_r prod_m G^(m)[i_m^k, r] + N(0, sigma^2), formed with plain torch CPU ops in fp64."""
    nnz = len(coords[0])
    out = np.empty(nnz, dtype=np.float32)
    Gt = [torch.from_numpy(g) for g in G]
    noise = synth.draw_normal_f64(nnz, sigma, seed, synth.S_NOISE)
    for a in range(0, nnz, chunk):
        b = min(nnz, a + chunk)
        p = None
        for m, g in enumerate(Gt):
            rows = g[torch.from_numpy(coords[m][a:b].astype(np.int64))]
            p = rows if p is None else p * rows
        out[a:b] = (p.sum(dim=1).numpy() + noise[a:b]).astype(np.float32)
    return out


def leg_cpgrad(args, torch, blco, synth, w, *, check=True, cpu=False):
    dev = torch.device("cuda:0")
    timer = Timer(torch)
    t0 = time.time()
    coords, _ = synth.workload_tensor(w, nnz=args.nnz, log=log)
    nnz = len(coords[0])
    G = [synth.draw_u01_matrix(d, 8, w.seed, synth.S_TRUTH + m) for m, d in enumerate(w.dims)]
    vals = planted_values(torch, coords, G, 0.01, w.seed, synth)
    log(f"{w.name}: generated {nnz} non-zeros with planted values in {time.time() - t0:.1f}s")
    t0 = time.time()
    T = blco.build(coords, vals, w.dims)
    build_s = time.time() - t0
    N = len(w.dims)
    R = w.ranks[0]
    scale = R ** (-1.0 / (2 * N))
    A = [synth.draw_factor(d, R, w.seed, m, 0, scale) for m, d in enumerate(w.dims)]
    P = [torch.from_numpy(a).to(dev).requires_grad_(True) for a in A]
    out = {}
    for storage in ("fp32", "bf16"):
        def step(storage=storage):
            for p in P:
                p.grad = None
            loss = blco.CPLoss.apply(T, storage, *P)
            loss.backward()
            return loss
        ms = timer(step, args.steps, args.warmup)
        loss = step()
        torch.cuda.synchronize()
        out[storage] = {"ms_per_step": ms, "gnnz_s": nnz / (ms * 1e-3) / 1e9,
                        "loss": float(loss.detach())}
        log(f"{w.name}: CP loss + gradient ({storage}): {ms:.2f} ms/step")
    ms_step = out["fp32"]["ms_per_step"]
    res = base_result(args, w, nnz, nnz / (ms_step * 1e-3) / 1e9, ms_step)
    res["metric"] = "CP loss + gradient step Gnnz/s (sampled reconstruction + N residual MTTKRPs)"
    Pd = [p.detach() for p in P]
    loss_ms = timer(lambda: blco.sampled_loss(T, Pd), args.steps)
    res["config"].update({"rank": R, "model_rank": 8, "noise_sigma": 0.01})
    res["loss_kernel_ms"] = loss_ms
    res["per_storage"] = out
    res["build_s"] = build_s
    res["cpu_baseline"] = None
    if check:
        import oracle

        Ad = [a.astype(np.float64) for a in A]
        f_ref, _ = oracle.cp_loss(coords, vals, Ad)
        res["errors"] = {"loss_rel_fp32": abs(out["fp32"]["loss"] - f_ref) / f_ref,
                         "loss_rel_bf16_vs_fp64": abs(out["bf16"]["loss"] - f_ref) / f_ref}
        log(f"{w.name}: oracle loss {f_ref:.6e}, gpu {out['fp32']['loss']:.6e}")
    if cpu:
        import oracle

        S = min(args.cpu_sample_nnz, nnz)
        t0 = time.time()
        oracle.cp_grad([c[:S] for c in coords], vals[:S], [a.astype(np.float64) for a in A],
                       dims=w.dims)
        dt = time.time() - t0
        res["cpu_baseline"] = {"value": S / dt / 1e9, "unit": "Gnnz/s", "cores": 1,
                               "kind": "oracle", "sample": f"loss + {N}-mode gradient over the "
                               f"first {S} non-zeros, fp64, single thread, {dt:.1f}s"}
    T.free()
    return res


def leg_cpals(args, torch, blco, synth, w):
    """CP-ALS (Algorithm 1) on the planted-model tensor of the CP-gradient recipe."""
    dev = torch.device("cuda:0")
    timer = Timer(torch)
    t0 = time.time()
    coords, _ = synth.workload_tensor(w, nnz=args.nnz, log=log)
    nnz = len(coords[0])
    G = [synth.draw_u01_matrix(d, 8, w.seed, synth.S_TRUTH + m) for m, d in enumerate(w.dims)]
    vals = planted_values(torch, coords, G, 0.01, w.seed, synth)
    log(f"generated {nnz} non-zeros with planted values in {time.time() - t0:.1f}s")
    T = blco.build(coords, vals, w.dims)
    N = len(w.dims)
    R = args.rank
    A = [synth.draw_u01_matrix(d, R, w.seed, synth.S_FACTOR + m).astype(np.float32)
         for m, d in enumerate(w.dims)]
    F = [torch.from_numpy(a).to(dev) for a in A]
    outs = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in w.dims]
    mk = [timer(lambda n=n: blco.mttkrp_acc(T, n, F, outs[n]), args.steps) for n in range(N)]
    blco.cp_als(T, [f.clone() for f in F], max_iters=max(args.warmup, 1), tol=-1.0)
    torch.cuda.synchronize()
    iters = max(args.steps, 2)
    Fw = [f.clone() for f in F]
    torch.cuda.synchronize()
    t0 = time.time()
    fits, rep = blco.cp_als(T, Fw, max_iters=iters, tol=-1.0)
    torch.cuda.synchronize()
    ms_iter = (time.time() - t0) * 1e3 / rep["iters"]
    log(f"CP-ALS R={R}: {ms_iter:.2f} ms per iteration, MTTKRP kernels {[round(x, 3) for x in mk]} "
        f"ms, fits {[round(f, 5) for f in fits]}")
    res = base_result(args, w, nnz, nnz * N / (ms_iter * 1e-3) / 1e9, ms_iter)
    res["metric"] = "CP-ALS iteration Gnnz/s (N MTTKRPs + Gram, V pseudo-inverse, M V^+, fit)"
    res["config"].update({"rank": R, "model_rank": 8, "noise_sigma": 0.01, "iterations": iters})
    res["mttkrp_kernel_ms"] = mk
    res["mttkrp_share_of_iteration"] = sum(mk) / ms_iter
    res["fits"] = fits
    res["pinv_fallbacks"] = rep["pinv_fallbacks"]
    res["cpu_baseline"] = None
    return res


def atomic_skew(args, torch, blco):
    """The atomic probe (one 16-lane row-update per entry, R = 32) over 2^22 updates of a
    2^24-row output: rows uniform, or Zipf(1.2) ranks without the K most frequent (the rows
    a stash would hold), ranks spread over the rows by an odd multiplier mod 2^24."""
    rows, n, R = 1 << 24, 1 << 22, 32
    dev = torch.device("cuda:0")
    out = torch.zeros((rows, R), dtype=torch.float32, device=dev)
    cdf = np.cumsum(np.arange(1, rows + 1, dtype=np.float64) ** -1.2)
    rng = np.random.default_rng(1225)
    timer = Timer(torch)
    res = []
    for K in (None, 0, 256, 4096, 65536):
        if K is None:
            ids = rng.integers(0, rows, n)
        else:
            lo = cdf[K - 1] if K > 0 else 0.0
            ranks = np.searchsorted(cdf, lo + rng.random(n) * (cdf[-1] - lo), side="right")
            ids = (np.minimum(ranks, rows - 1).astype(np.uint64) * np.uint64(2654435761)) & \
                np.uint64(rows - 1)
        t = torch.from_numpy(ids.astype(np.uint32).view(np.int32)).to(dev)
        ms = timer(lambda: blco.atomic_probe(out, t), args.steps, 2)
        top = int(np.bincount(ids.astype(np.int64), minlength=rows).max())
        res.append({"rows": "uniform" if K is None else f"zipf1.2 without the top {K}",
                    "ms": ms, "row_updates_per_s": n / (ms * 1e-3), "most_updates_on_one_row": top})
        log(f"atomic skew {res[-1]}")
    return {"probe": "fp32 atomic row-updates vs row skew", "updates": n, "table_rows": rows,
            "rank": R, "results": res}


def resolution_sweep(args, torch, blco, synth):
    """Both conflict-resolution mechanisms (Sections 5.1-5.2) on the short mode of
    3-mode 2^21 x 2^17 x I tensors (Zipf(1.1) long modes, uniform short mode),
    for the Section 5.3 heuristic: kernel ms of the mode-3 MTTKRP per mechanism."""
    R = args.rank
    nnz = args.nnz or 50_000_000
    timer = Timer(torch)
    rows = []
    for I in (1, 2, 4, 8, 16, 32, 64, 128, 255, 512):
        dims = (1 << 21, 1 << 17, I)
        w = synth.Workload(f"short3_{I}", dims, nnz, (("zipf", 1.1), ("zipf", 1.1), ("uniform",)),
                           "u01", (R,), (0, 1, 2), synth.BASE_SEED * 100 + 50 + I % 41)
        coords, vals = synth.workload_tensor(w)
        T = blco.build(coords, vals, dims)
        A = synth.workload_factors(w, R)
        F = [torch.from_numpy(a).to("cuda:0") for a in A]
        out = torch.zeros((I, R), device="cuda:0")
        ms = {}
        for res in ("register", "hierarchical"):
            T.set_resolution(res)
            ms[res] = timer(lambda: blco.mttkrp_acc(T, 2, F, out), args.steps, args.warmup)
        T.set_resolution("auto")
        rows.append({"I": I, "nnz": len(vals), "register_ms": ms["register"],
                     "hierarchical_ms": ms["hierarchical"], "auto": T.resolution(2, R),
                     "register_over_hierarchical": ms["register"] / ms["hierarchical"]})
        log(f"I={I}: register {ms['register']:.3f} ms, hierarchical {ms['hierarchical']:.3f} ms, "
            f"auto picks {rows[-1]['auto']}")
        T.free()
        del F, A, coords, vals
    return {"sweep": "conflict resolution vs short-mode length", "rank": R,
            "cus": torch.cuda.get_device_properties(0).multi_processor_count, "rows": rows}


def leg_build(args, torch, blco, synth, w):
    """BLCO construction alone (Section 4): the host builder once, and the GPU builder
    (blco_build_device) from device-resident coordinates and values, `steps` times after
    `warmup` builds, with its per-stage stream times (linearize, sort, re-encode, runs of
    block keys, frequent rows)."""
    dev = torch.device("cuda:0")
    coords, vals = synth.workload_tensor(w, nnz=args.nnz, log=log)
    nnz = len(vals)
    t0 = time.time()
    Th = blco.build(coords, vals, w.dims, placement="host")
    host_s = time.time() - t0
    inf = Th.info()
    Th.free()
    log(f"{w.name}: host builder {host_s:.3f}s")
    dc = [torch.from_numpy(c.view(np.int32)).to(dev) for c in coords]
    dv = torch.from_numpy(vals).to(dev)
    torch.cuda.synchronize()
    totals, stages = [], []
    for i in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.time()
        Tg = blco.build_device(dc, dv, w.dims)
        torch.cuda.synchronize()
        dt = time.time() - t0
        st = Tg.info()["build_stage_ms"]
        Tg.free()
        if i >= args.warmup:
            totals.append(dt * 1e3)
            stages.append(st)
            log(f"{w.name}: GPU build {dt * 1e3:.2f} ms, stages {st}")
    med = {k: float(np.median([x[k] for x in stages])) for k in stages[0]}
    ms = float(np.median(totals))
    res = base_result(args, w, nnz, nnz / (ms * 1e-3) / 1e9, ms)
    res["metric"] = "BLCO construction (GPU builder) non-zeros per second"
    res["unit"] = "Gnnz/s"
    res["config"].update({"key_bits": inf["total_bits"], "blocks": inf["nblocks"],
                          "runs": inf["nruns"]})
    res["build_gpu_ms"] = totals
    res["build_stage_ms_median"] = med
    res["build_host_s"] = host_s
    return res


def secondary_summary(r):
    keep = ("metric", "value", "unit", "ms_per_step", "steps", "warmup", "config", "roofline",
            "per_config", "errors", "per_mode", "one_pass", "per_mode_passes_ms_per_step",
            "per_mode_passes_gnnz_s", "per_storage", "loss_kernel_ms", "build_s",
            "build_gpu_s", "distinct_indices")
    return {k: r[k] for k in keep if k in r}


def suite(args, torch, blco, synth):
    """The default run: the zipf4 headline, then zipf3, cpgrad4 and oom3 as secondary legs."""
    W = synth.WORKLOADS
    res = leg_inmemory(args, torch, blco, synth, W["zipf4"], check=not args.no_check,
                       cpu=not args.no_cpu_baseline, headline=True)
    sec = {}
    torch.cuda.empty_cache()
    sec["zipf3"] = secondary_summary(leg_inmemory(args, torch, blco, synth, W["zipf3"],
                                                  check=not args.no_check, gpu_build=True))
    torch.cuda.empty_cache()
    sec["cpgrad4"] = secondary_summary(leg_cpgrad(args, torch, blco, synth, W["cpgrad4"],
                                                  check=False))
    torch.cuda.empty_cache()
    elapsed = time.time() - T_START
    if elapsed > args.oom_start_limit_s:
        sec["oom3"] = {"skipped": f"run already at {elapsed:.0f}s, past the {args.oom_start_limit_s}s "
                                  "start limit of the 1.5B-non-zero leg"}
        log(sec["oom3"]["skipped"])
    else:
        sec["oom3"] = secondary_summary(leg_oom(args, torch, blco, synth, W["oom3"],
                                                check=not args.no_check))
    res["secondary"] = sec
    return res


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-counters":
        # OUT TITLE COPY_BYTES PROBE_ROW_OPS CSV... [-- COMMAND...]
        a = sys.argv[2:]
        cmds = []
        if "--" in a:
            i = a.index("--")
            a, cmds = a[:i], a[i + 1:]
        summarize_counters(a[0], a[1], *a[4:], copy_bytes=int(a[2]), probe_row_ops=int(a[3]),
                           commands=cmds)
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-overlap":
        # OUT TITLE COPY_CSV KERNEL_CSV COPIES_PER_CALL COMMAND
        summarize_overlap(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], int(sys.argv[6]),
                          sys.argv[7])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-bench":
        # OUT TITLE JSON COMMAND
        summarize_bench(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-skew":
        # OUT JSON COMMAND
        summarize_skew(sys.argv[2], sys.argv[3], sys.argv[4])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-sweep":
        # OUT JSON COMMAND
        summarize_sweep(sys.argv[2], sys.argv[3], sys.argv[4])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-stats":
        # OUT TITLE STATS_CSV COMMAND
        summarize_stats(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=None,
                    choices=["zipf3", "uniform3", "zipf4", "oom3", "cpgrad4", "cpals4", "short4",
                             "small"])
    ap.add_argument("--nnz", type=int, default=None, help="shrink the workload (same recipe)")
    ap.add_argument("--budget", type=int, default=None, help="device budget for oom3 (bytes)")
    ap.add_argument("--cpu-sample-nnz", type=int, default=4_000_000,
                    help="non-zeros of the single-thread oracle timing")
    ap.add_argument("--cpu-sample-all-nnz", type=int, default=16_000_000,
                    help="non-zeros of the all-core oracle timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--build-only", action="store_true",
                    help="time BLCO construction of --workload (host and GPU builders) only")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle row checks")
    ap.add_argument("--oom-start-limit-s", type=float, default=300.0,
                    help="default run: skip the 1.5B-non-zero leg when it would start later")
    ap.add_argument("--atomic-skew", action="store_true",
                    help="atomic probe rate over uniform and Zipf-distributed rows")
    ap.add_argument("--resolution-sweep", action="store_true",
                    help="time both conflict-resolution mechanisms over short-mode lengths")
    ap.add_argument("--rank", type=int, default=32,
                    help="rank of --resolution-sweep and of the cpals4 leg")
    ap.add_argument("--calibrate-copy-bytes", type=int, default=0,
                    help="also run one plain device-to-device copy of this many bytes "
                         "(the reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2201_12523_amd as blco
    import synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    log(f"device {torch.cuda.get_device_name(0)}")
    if args.calibrate_copy_bytes:
        n = args.calibrate_copy_bytes // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.resolution_sweep:
        print(json.dumps(resolution_sweep(args, torch, blco, synth)), flush=True)
        return
    if args.atomic_skew:
        print(json.dumps(atomic_skew(args, torch, blco)), flush=True)
        return
    W = synth.WORKLOADS
    check, cpu = not args.no_check, not args.no_cpu_baseline
    if args.build_only:
        res = leg_build(args, torch, blco, synth, W[args.workload or "zipf3"])
    elif args.workload is None:
        res = suite(args, torch, blco, synth)
    elif args.workload == "oom3":
        res = leg_oom(args, torch, blco, synth, W["oom3"], check=check, cpu=cpu)
    elif args.workload == "cpgrad4":
        res = leg_cpgrad(args, torch, blco, synth, W["cpgrad4"], check=check, cpu=cpu)
    elif args.workload == "cpals4":
        res = leg_cpals(args, torch, blco, synth, W["cpgrad4"])
    else:
        res = leg_inmemory(args, torch, blco, synth, W[args.workload], check=check, cpu=cpu)
    res["wall_s"] = time.time() - T_START
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
