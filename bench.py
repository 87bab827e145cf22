"""Benchmark: BLCO sparse MTTKRP on one MI355X.

Default workload (``zipf3``): 3-mode tensor 2^22 x 2^21 x 2^20 (63 key bits, one
block), 50M distinct non-zeros with per-mode Zipf(1.1) indices, U(0,1) values,
rank-32 N(0,1) factors; MTTKRP in all three modes from one BLCO copy.  A step is
one MTTKRP per mode (output zero-fill included) with fp32 factors; inputs are
resident in device memory before timing starts.  The bf16-factor form is timed
beside it, and both are checked against the fp64 oracle on sampled rows in the
CPU-baseline leg.

Other legs (``--workload``):
  zipf4    4-mode 2^24 x 2^22 x 2^20 x 2^10 (76 bits, blocked on the top 12),
           200M non-zeros, R = 32 and 64, fp32 and bf16 factors;
  oom3     3-mode 2^23 x 2^23 x 2^17, 1.5B non-zeros in pinned host memory,
           streamed under an 8 GB device budget; copy/compute overlap reported;
  cpgrad4  sparse CP loss + gradient step, 4-mode 2^20 x 2^18 x 2^16 x 2^12,
           80M non-zeros holding a planted rank-8 model plus noise, R = 32;
  cpals4   CP-ALS (Algorithm 1) iterations on the cpgrad4 tensor, R = --rank;
  uniform3 the zipf3 shape with uniform indices;
  short4   4-mode 2^21 x 2^17 x 24 x 168, 50M non-zeros, R = 32: the two short
           modes take hierarchical conflict resolution (Section 5.3 heuristic),
           and the register-based mechanism is timed beside it on those modes.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MTTKRP Gnnz/s per mode & % HBM peak; bf16 vs fp32 factors at stated rel error"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mttkrp_win_zipf3.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("blco_device.hip", "blco_kernels.h"):
        with open(os.path.join(ROOT, "paper_2201_12523_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, if it matches this kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


class Timer:
    """Average milliseconds of `fn` over `steps` calls, with HIP events on torch's stream."""

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
        return e0.elapsed_time(e1) / steps


def sampled_rows(rng, I, k=120):
    return np.unique(np.concatenate([np.arange(min(8, I)), rng.integers(0, I, k), [I - 1]])
                     ).astype(np.uint32)


def row_errors(oracle, blco, torch, T, coords, vals, A_ref, F, outs, dims, modes, rng, dev):
    """Max / median of |gpu - oracle| / sum|terms| over sampled rows of each mode."""
    worst, meds = 0.0, []
    for n in modes:
        o = blco.mttkrp(T, n, F, out=outs[n])
        rows = sampled_rows(rng, dims[n])
        M, S = oracle.mttkrp_rows_f32(coords, vals, A_ref, n, rows, dims)
        got = o[torch.from_numpy(rows.astype(np.int64)).to(dev)].cpu().numpy().astype(np.float64)
        nz = S > 0
        e = np.abs(got - M)[nz] / S[nz]
        worst = max(worst, float(e.max()) if e.size else 0.0)
        meds.append(float(np.median(e)) if e.size else 0.0)
        log(f"  oracle rows, mode {n}: max normalised error {worst:.2e}")
    return {"max": worst, "median": float(np.median(meds))}


def cpu_oracle_rate(oracle, coords, vals, A, sample, modes):
    """The fp64 oracle, single thread, over the first `sample` non-zeros of every mode."""
    S = min(sample, len(vals))
    cs = [c[:S] for c in coords]
    Ad = [a.astype(np.float64) for a in A]
    t0 = time.time()
    for n in modes:
        oracle.mttkrp(cs, vals[:S], Ad, n)
    dt = time.time() - t0
    return {"value": S * len(modes) / dt / 1e9, "unit": "Gnnz/s", "cores": 1, "kind": "oracle",
            "sample": f"first {S} non-zeros of the workload, {len(modes)} modes, fp64, "
                      f"single thread, {dt:.1f}s"}


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


# --------------------------------------------------------------------------- legs

def leg_inmemory(args, torch, blco, synth, w):
    dev = torch.device("cuda:0")
    timer = Timer(torch)
    t0 = time.time()
    coords, vals = synth.workload_tensor(w, nnz=args.nnz, log=log)
    nnz = len(vals)
    log(f"generated {nnz} non-zeros in {time.time() - t0:.1f}s")
    t0 = time.time()
    T = blco.build(coords, vals, w.dims)
    build_s = time.time() - t0
    inf = T.info()
    log(f"built BLCO in {build_s:.2f}s: T={inf['total_bits']} bits, {inf['nblocks']} block(s), "
        f"{inf['nruns']} run(s)")
    # the same construction on the GPU, from device-resident coordinates and values
    dc = [torch.from_numpy(c.view(np.int32)).to(dev) for c in coords]
    dv = torch.from_numpy(vals).to(dev)
    torch.cuda.synchronize()
    gpu_build = []
    for _ in range(3):
        t0 = time.time()
        Tg = blco.build_device(dc, dv, w.dims)
        gpu_build.append(time.time() - t0)
        Tg.free()
    del dc, dv
    log(f"built BLCO on the GPU in {min(gpu_build) * 1e3:.1f} ms (host builder {build_s * 1e3:.0f} ms)")
    N = len(w.dims)
    modes = list(range(N))
    distinct = [int(np.count_nonzero(np.bincount(c, minlength=d))) for c, d in zip(coords, w.dims)]
    results = {}
    head = None
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
            call = [timer(lambda n=n: blco.mttkrp(T, n, F, out=outs[n]), args.steps) for n in modes]
            kern = [timer(lambda n=n: blco.mttkrp_acc(T, n, F, outs[n]), args.steps) for n in modes]
            sf = 4 if tag == "fp32" else 2
            per_nnz = 12 + (N - 1) * R * sf
            mech = [T.resolution(n, R) for n in modes]
            alt = {}
            for n in modes:
                if mech[n] == "hierarchical":
                    # the other mechanism on the same mode, for the Section 5.3 comparison
                    T.set_resolution("register")
                    alt[n] = timer(lambda n=n: blco.mttkrp_acc(T, n, F, outs[n]), args.steps)
                    T.set_resolution("auto")
            results[f"R{R}_{tag}"] = {
                "ms_per_step": ms_step, "gnnz_s": nnz * N / (ms_step * 1e-3) / 1e9,
                "resolution": mech,
                "register_kernel_ms_on_hierarchical_modes": {str(n): v for n, v in alt.items()},
                "call_ms": call, "kernel_ms": kern,
                "per_mode_gnnz_s": [nnz / (x * 1e-3) / 1e9 for x in call],
                "bytes_per_nnz": per_nnz,
                "kernel_gbs": [nnz * per_nnz / (x * 1e-3) / 1e9 for x in kern],
            }
            log(f"R={R} {tag}: all-mode step {ms_step:.3f} ms, kernel ms/mode "
                f"{[round(x, 3) for x in kern]} ({mech}); register-based on the hierarchical "
                f"modes: {({n: round(v, 3) for n, v in alt.items()})}")
            if head is None:
                head = (R, ms_step, kern, per_nnz, A, F32, BF16, outs)
    R, ms_step, kern, per_nnz, A, F32, BF16, outs = head
    avg_kernel_ms = float(np.mean(kern))
    achieved = nnz * per_nnz / (avg_kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic() if w.name == "zipf3" and args.nnz is None else None
    compulsory = [nnz * 12 + sum(distinct[m] * R * 4 for m in modes if m != n) +
                  2 * w.dims[n] * R * 4 for n in modes]
    res = base_result(args, w, nnz, nnz * N / (ms_step * 1e-3) / 1e9, ms_step)
    res["config"].update({"rank": R, "key_bits": inf["total_bits"], "blocks": inf["nblocks"]})
    res["roofline"] = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
        "kernel": [short_kernel_name(R, N) if T.resolution(n, R) == "hierarchical"
                   else win_kernel_name(R, N, stash=inf["hot_rows"][n] > 0) for n in modes],
        "bytes_per_nnz": per_nnz, "avg_kernel_ms": avg_kernel_ms,
        "model": "requested bytes 12 + (N-1)*R*s_f per non-zero (the paper's Vol); "
                 "frac above 1 means factor rows are served from cache",
        "compulsory_bytes_per_launch": compulsory,
    }
    res["per_config"] = results
    res["distinct_indices"] = distinct
    res["build_s"] = build_s
    res["build_gpu_s"] = min(gpu_build)
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        import oracle

        res["cpu_baseline"] = cpu_oracle_rate(oracle, coords, vals, A, args.cpu_sample_nnz, modes)
        log(f"cpu oracle: {res['cpu_baseline']['value']:.4f} Gnnz/s")
        rng = np.random.default_rng(7)
        errs = {}
        for R in w.ranks:
            if R == head[0]:
                A_, F32_, BF16_, outs_ = A, F32, BF16, outs
            else:
                A_ = synth.workload_factors(w, R)
                F32_ = [torch.from_numpy(a).to(dev) for a in A_]
                BF16_ = [blco.cast_bf16(f) for f in F32_]
                outs_ = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in w.dims]
            Ab = [oracle.bf16_round(a) for a in A_]
            errs[f"R{R}_fp32"] = row_errors(oracle, blco, torch, T, coords, vals, A_, F32_, outs_,
                                            w.dims, modes, rng, dev)
            errs[f"R{R}_bf16"] = row_errors(oracle, blco, torch, T, coords, vals, Ab, BF16_, outs_,
                                            w.dims, modes, rng, dev)
            errs[f"R{R}_bf16_vs_fp32"] = row_errors(oracle, blco, torch, T, coords, vals, A_,
                                                    BF16_, outs_, w.dims, modes, rng, dev)
        res["errors"] = errs
        log(f"errors: {errs}")
    return res


def leg_oom(args, torch, blco, synth, w):
    dev = torch.device("cuda:0")
    timer = Timer(torch)
    t0 = time.time()
    coords, vals = synth.workload_tensor(w, nnz=args.nnz, log=log)
    nnz = len(vals)
    log(f"generated {nnz} non-zeros in {time.time() - t0:.1f}s")
    t0 = time.time()
    T = blco.build(coords, vals, w.dims, placement="pinned")
    build_s = time.time() - t0
    log(f"built pinned BLCO in {build_s:.1f}s")
    N = len(w.dims)
    modes = list(range(N))
    R = w.ranks[0]
    A = synth.workload_factors(w, R)
    F = [torch.from_numpy(a).to(dev) for a in A]
    outs = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in w.dims]
    budget = args.budget or w.budget_bytes
    per = []
    for n in modes:
        ms = timer(lambda n=n: blco.mttkrp_stream(T, n, F, out=outs[n], device_budget=budget),
                   args.steps, args.warmup)
        inf = T.info()
        copy_ms, kern_ms = inf["stream_copy_ms"], inf["stream_kernel_ms"]
        tot_ms = inf["stream_total_ms"]
        overlap = (copy_ms + kern_ms - tot_ms) / max(min(copy_ms, kern_ms), 1e-9)
        per.append({"mode": n, "call_ms": ms, "overall_gnnz_s": nnz / (ms * 1e-3) / 1e9,
                    "in_memory_gnnz_s": nnz / (kern_ms * 1e-3) / 1e9,
                    "h2d_gbs": nnz * 12 / (copy_ms * 1e-3) / 1e9,
                    "copy_ms": copy_ms, "kernel_ms": kern_ms, "total_ms": tot_ms,
                    "overlap": overlap, "chunks": inf["stream_chunks"],
                    "chunk_nnz": inf["stream_chunk_nnz"],
                    "peak_device_bytes": inf["stream_peak_bytes"]})
        log(f"mode {n}: {ms:.1f} ms/call, copy {copy_ms:.1f} ms, kernels {kern_ms:.1f} ms, "
            f"span {tot_ms:.1f} ms, overlap {overlap:.3f}, {inf['stream_chunks']} chunks")
    ms_per_mode_sum = sum(p["call_ms"] for p in per)
    # every mode in one pass: each chunk crosses the host link once
    ms_step = timer(lambda: blco.mttkrp_stream_all(T, F, outs=outs, device_budget=budget),
                    args.steps, args.warmup)
    inf = T.info()
    copy_ms, kern_ms, tot_ms = inf["stream_copy_ms"], inf["stream_kernel_ms"], inf["stream_total_ms"]
    fused = {"call_ms": ms_step, "overall_gnnz_s": nnz * N / (ms_step * 1e-3) / 1e9,
             "copy_ms": copy_ms, "kernel_ms": kern_ms, "total_ms": tot_ms,
             "overlap": (copy_ms + kern_ms - tot_ms) / max(min(copy_ms, kern_ms), 1e-9),
             "h2d_gbs": nnz * 12 / (copy_ms * 1e-3) / 1e9, "chunks": inf["stream_chunks"],
             "peak_device_bytes": inf["stream_peak_bytes"]}
    log(f"all modes in one pass: {ms_step:.1f} ms/call, copy {copy_ms:.1f} ms, kernels "
        f"{kern_ms:.1f} ms, overlap {fused['overlap']:.3f}")
    res = base_result(args, w, nnz, nnz * N / (ms_step * 1e-3) / 1e9, ms_step)
    res["per_mode_passes_ms_per_step"] = ms_per_mode_sum
    res["per_mode_passes_gnnz_s"] = nnz * N / (ms_per_mode_sum * 1e-3) / 1e9
    res["one_pass"] = fused
    kern_ms = float(np.mean([p["kernel_ms"] / p["chunks"] for p in per]))
    chunk_nnz = per[0]["chunk_nnz"]
    per_nnz = 12 + (N - 1) * R * 4
    res["config"].update({"rank": R, "device_budget_bytes": budget, "placement": "pinned"})
    res["roofline"] = {
        "bound": "hbm", "achieved": chunk_nnz * per_nnz / (kern_ms * 1e-3) / 1e9,
        "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": chunk_nnz * per_nnz / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
        "kernel": win_kernel_name(R, N) + " per chunk", "bytes_per_nnz": per_nnz,
        "avg_kernel_ms": kern_ms,
        "note": "the step itself is bound by host-to-device copies (per_mode h2d_gbs)",
    }
    res["per_mode"] = per
    res["build_s"] = build_s
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        import oracle

        res["cpu_baseline"] = cpu_oracle_rate(oracle, coords, vals, A, args.cpu_sample_nnz, modes)
        rng = np.random.default_rng(7)
        worst = 0.0
        for n in modes:
            o = blco.mttkrp_stream(T, n, F, out=outs[n], device_budget=budget)
            rows = sampled_rows(rng, w.dims[n], 40)
            M, S = oracle.mttkrp_rows_f32(coords, vals, A, n, rows, w.dims)
            got = o[torch.from_numpy(rows.astype(np.int64)).to(dev)].cpu().numpy()
            nz = S > 0
            worst = max(worst, float((np.abs(got - M)[nz] / S[nz]).max()))
        res["errors"] = {"fp32": {"max": worst}}
        log(f"max normalised error {worst:.2e}")
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


def leg_cpgrad(args, torch, blco, synth, w):
    dev = torch.device("cuda:0")
    timer = Timer(torch)
    t0 = time.time()
    coords, _ = synth.workload_tensor(w, nnz=args.nnz, log=log)
    nnz = len(coords[0])
    G = [synth.draw_u01_matrix(d, 8, w.seed, synth.S_TRUTH + m) for m, d in enumerate(w.dims)]
    vals = planted_values(torch, coords, G, 0.01, w.seed, synth)
    log(f"generated {nnz} non-zeros with planted values in {time.time() - t0:.1f}s")
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
        log(f"CP loss+gradient ({storage}): {ms:.2f} ms/step")
    ms_step = out["fp32"]["ms_per_step"]
    res = base_result(args, w, nnz, nnz / (ms_step * 1e-3) / 1e9, ms_step)
    res["metric"] = "CP loss + gradient step Gnnz/s (forward sampled reconstruction + N MTTKRPs)"
    Pd = [p.detach() for p in P]
    loss_ms = timer(lambda: blco.sampled_loss(T, Pd), args.steps)
    per_nnz = 12 + 4 + N * R * 4
    res["config"].update({"rank": R, "model_rank": 8, "noise_sigma": 0.01})
    res["roofline"] = {
        "bound": "hbm", "achieved": nnz * per_nnz / (loss_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": nnz * per_nnz / (loss_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "traffic": None, "kernel": f"k_loss_tile<32, float, {N}> (sampled reconstruction)",
        "bytes_per_nnz": per_nnz, "avg_kernel_ms": loss_ms,
    }
    res["per_storage"] = out
    res["build_s"] = build_s
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        import oracle

        S = min(args.cpu_sample_nnz, nnz)
        t0 = time.time()
        oracle.cp_grad([c[:S] for c in coords], vals[:S], [a.astype(np.float64) for a in A],
                       dims=w.dims)
        dt = time.time() - t0
        res["cpu_baseline"] = {"value": S / dt / 1e9, "unit": "Gnnz/s", "cores": 1,
                               "kind": "oracle", "sample": f"loss + {N}-mode gradient over the "
                               f"first {S} non-zeros, fp64, single thread, {dt:.1f}s"}
        f_ref, _ = oracle.cp_loss(coords, vals, [a.astype(np.float64) for a in A])
        res["errors"] = {"loss_rel_fp32": abs(out["fp32"]["loss"] - f_ref) / f_ref,
                         "loss_rel_bf16_vs_fp64": abs(out["bf16"]["loss"] - f_ref) / f_ref}
        log(f"oracle loss {f_ref:.6e}, gpu {out['fp32']['loss']:.6e}")
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
    per_nnz = 12 + (N - 1) * R * 4
    avg = float(np.mean(mk))
    res["roofline"] = {
        "bound": "hbm", "achieved": nnz * per_nnz / (avg * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": nnz * per_nnz / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
        "kernel": [short_kernel_name(R, N) if T.resolution(n, R) == "hierarchical"
                   else win_kernel_name(R, N) for n in range(N)],
        "bytes_per_nnz": per_nnz, "avg_kernel_ms": avg,
        "model": "requested bytes 12 + (N-1)*R*4 per non-zero of the MTTKRP kernels",
    }
    res["mttkrp_kernel_ms"] = mk
    res["mttkrp_share_of_iteration"] = sum(mk) / ms_iter
    res["fits"] = fits
    res["pinv_fallbacks"] = rep["pinv_fallbacks"]
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        from oracle import cpals

        S = min(args.cpu_sample_nnz, nnz)
        t0 = time.time()
        _, fw = cpals.cp_als([c[:S] for c in coords], vals[:S], [a.astype(np.float64) for a in A],
                             w.dims, max_iters=1)
        dt = time.time() - t0
        res["cpu_baseline"] = {"value": S * N / dt / 1e9, "unit": "Gnnz/s", "cores": 1,
                               "kind": "oracle", "sample": f"one CP-ALS iteration over the first "
                               f"{S} non-zeros, fp64, single thread, {dt:.1f}s"}
    return res


def win_kernel_name(R, N, ft="float", big=False, stash=True):
    """Template name of the window MTTKRP kernel the library launches for rank R
    (stash: the mode has frequent rows held in LDS)."""
    lpn, rpl = (16, 1) if R <= 16 else (16, 2) if R <= 32 else (16, 4) if R <= 64 else (64, 2)
    b = lambda v: "true" if v else "false"
    return f"k_mttkrp_win<{lpn}, {rpl}, {ft}, {N}, {b(big)}, {b(stash)}>"


def short_kernel_name(R, N, ft="float", big=False):
    """Template name of the hierarchical MTTKRP kernel for a single rank slice of width R."""
    rpl = 1 if R <= 16 else 2 if R <= 32 else 4
    return f"k_mttkrp_short<{rpl}, {ft}, {N}, {'true' if big else 'false'}>"


def summarize_pmc(fetch_csv, write_csv, copy_bytes, kernel=None, out=TRAFFIC_FILE):
    """Per-launch HBM bytes of the MTTKRP kernel from two rocprofv3 --pmc runs.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are averaged over the MTTKRP
    dispatches, and each is scaled by the ratio of the known size of a plain
    device-to-device copy to what the same counter read for that copy.
    """
    import csv

    kernel = kernel or "void " + win_kernel_name(32, 3)

    def per_kernel(path, counter):
        acc = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            key = "mttkrp" if name.startswith(kernel + "(") else (
                "copy" if "copyBuffer" in name else None)
            if key is None:
                continue
            acc.setdefault(key, []).append(float(r["Counter_Value"]))
        # the calibration copy is the largest copy dispatch
        red = {"mttkrp": np.mean, "copy": np.max}
        return ({k: float(red[k](v)) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()})

    f, fn = per_kernel(fetch_csv, "FETCH_SIZE")
    w, wn = per_kernel(write_csv, "WRITE_SIZE")
    # the largest copy dispatch is the calibration copy
    fscale = copy_bytes / (f["copy"] * 1024.0)
    wscale = copy_bytes / (w["copy"] * 1024.0)
    fetch_b = f["mttkrp"] * 1024.0 * fscale
    write_b = w["mttkrp"] * 1024.0 * wscale
    lines = [
        f"# HBM traffic of the MTTKRP kernel ({kernel[5:]}), 50M-non-zero",
        "# 2^22 x 2^21 x 2^20 Zipf(1.1) workload, R = 32, fp32 factors, per launch (one mode).",
        "# FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two rocprofv3 --pmc runs of",
        "#   python3 bench.py --workload zipf3 --steps 2 --warmup 0 --no-cpu-baseline "
        f"--calibrate-copy-bytes {copy_bytes}",
        "# each scaled by copy_bytes / (counter of the calibration copy), then summed.",
        f"kernel_source_sha256_16: {kernel_source_hash()}",
        f"mttkrp_dispatches: {fn.get('mttkrp', 0)}",
        f"fetch_kib_per_dispatch: {f['mttkrp']:.1f}",
        f"write_kib_per_dispatch: {w['mttkrp']:.1f}",
        f"copy_bytes: {copy_bytes}",
        f"copy_fetch_kib: {f['copy']:.1f}",
        f"copy_write_kib: {w['copy']:.1f}",
        f"fetch_scale: {fscale:.4f}",
        f"write_scale: {wscale:.4f}",
        f"hbm_fetch_bytes_per_launch: {fetch_b:.0f}",
        f"hbm_write_bytes_per_launch: {write_b:.0f}",
        f"hbm_bytes_per_launch: {fetch_b + write_b:.0f}",
    ]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_counters(workload, kernel, nnz, out, *csvs):
    """Per-launch and per-non-zero means of every counter in one or more rocprofv3
    --pmc CSVs, over the dispatches of one kernel (instruction counts, LDS bank
    conflicts, and the atomics the kernel sends to the L2 and on to memory)."""
    import csv

    lines = [f"# rocprofv3 counters of {kernel}, workload {workload}, {nnz} non-zeros per launch",
             "# (one mode per launch; mean over the kernel's dispatches). Commands, one per pass:"]
    vals, ndisp = {}, {}
    for path in csvs:
        names = set()
        for r in csv.DictReader(open(path)):
            if not r["Kernel_Name"].startswith("void " + kernel + "("):
                continue
            names.add(r["Counter_Name"])
            vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        for c in names:
            ndisp[c] = len(vals[c])
        lines.append(f"#   rocprofv3 --pmc {' '.join(sorted(names))} -o run --output-format csv "
                     f"-- python3 bench.py --workload {workload} --steps 2 --warmup 0 "
                     "--no-cpu-baseline")
    lines.append(f"kernel_source_sha256_16: {kernel_source_hash()}")
    lines.append(f"{'counter':40s} {'dispatches':>10s} {'per_launch':>16s} {'per_nnz':>10s}")
    for c in sorted(vals):
        m = float(np.mean(vals[c]))
        lines.append(f"{c:40s} {ndisp[c]:10d} {m:16.1f} {m / nnz:10.4f}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


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


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-pmc":
        summarize_pmc(sys.argv[2], sys.argv[3], int(sys.argv[4]))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-counters":
        # WORKLOAD KERNEL NNZ OUT CSV...
        summarize_counters(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], *sys.argv[6:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="zipf3",
                    choices=["zipf3", "uniform3", "zipf4", "oom3", "cpgrad4", "cpals4", "short4",
                             "small"])
    ap.add_argument("--nnz", type=int, default=None, help="shrink the workload (same recipe)")
    ap.add_argument("--budget", type=int, default=None, help="device budget for oom3 (bytes)")
    ap.add_argument("--cpu-sample-nnz", type=int, default=4_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    w = synth.WORKLOADS.get(args.workload)
    if args.workload == "oom3":
        res = leg_oom(args, torch, blco, synth, w)
    elif args.workload == "cpgrad4":
        res = leg_cpgrad(args, torch, blco, synth, w)
    elif args.workload == "cpals4":
        res = leg_cpals(args, torch, blco, synth, synth.WORKLOADS["cpgrad4"])
    else:
        res = leg_inmemory(args, torch, blco, synth, w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
