"""Benchmark: all-mode BLCO sparse MTTKRP on one MI355X.

Workload (default): 3-mode tensor 2^22 x 2^21 x 2^20 (63 key bits, one block),
50M distinct non-zeros with per-mode Zipf(1.1) indices, U(0,1) values, rank-32
N(0,1) factors; MTTKRP in all three modes from one BLCO copy.  A step is one
MTTKRP per mode (output zero-fill included) with fp32 factors; inputs are
resident in device memory before timing starts.  The bf16-factor form is timed
beside it, and both are checked against the fp64 oracle on sampled rows.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="zipf3")
    ap.add_argument("--nnz", type=int, default=None, help="shrink the workload (same recipe)")
    ap.add_argument("--cpu-sample-nnz", type=int, default=4_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2201_12523_amd as blco
    import synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    w = synth.WORKLOADS[args.workload]
    R = w.ranks[0]
    N = len(w.dims)
    t0 = time.time()
    coords, vals = synth.workload_tensor(w, nnz=args.nnz)
    nnz = len(vals)
    log(f"generated {nnz} non-zeros in {time.time() - t0:.1f}s")
    t0 = time.time()
    T = blco.build(coords, vals, w.dims)
    build_s = time.time() - t0
    inf = T.info()
    log(f"built BLCO in {build_s:.2f}s: T={inf['total_bits']} bits, {inf['nblocks']} block(s)")
    A = synth.workload_factors(w, R)
    F32 = [torch.from_numpy(a).to(dev) for a in A]
    BF16 = [blco.cast_bf16(f) for f in F32]
    distinct = [int(np.count_nonzero(np.bincount(c, minlength=d))) for c, d in zip(coords, w.dims)]
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    outs = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in w.dims]

    def step(F):
        for n in range(N):
            blco.mttkrp(T, n, F, out=outs[n])

    # ---- timed region: K all-mode steps, fp32 factors
    for _ in range(args.warmup):
        step(F32)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step(F32)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    log(f"fp32 all-mode step {ms_step:.3f} ms")

    def per_mode(F, acc):
        """Average ms per call for each mode: full call, or the MTTKRP kernel alone (acc)."""
        res = []
        for n in range(N):
            fn = (lambda: blco.mttkrp_acc(T, n, F, outs[n])) if acc else \
                (lambda: blco.mttkrp(T, n, F, out=outs[n]))
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            res.append(e0.elapsed_time(e1) / args.steps)
        return res

    call_f32 = per_mode(F32, False)
    kern_f32 = per_mode(F32, True)
    call_bf16 = per_mode(BF16, False)
    kern_bf16 = per_mode(BF16, True)
    # bf16 all-mode step
    for _ in range(args.warmup):
        step(BF16)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step(BF16)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step_bf16 = ev0.elapsed_time(ev1) / args.steps

    # ---- roofline of the dominant kernel (the MTTKRP kernel, fp32 factors)
    per_nnz = 12 + (N - 1) * R * 4          # key + value streamed, N-1 factor rows gathered
    alg_bytes = nnz * per_nnz                # per launch (one mode)
    avg_kernel_ms = float(np.mean(kern_f32))
    achieved = alg_bytes / (avg_kernel_ms * 1e-3) / 1e9
    compulsory = []
    for n in range(N):
        b = nnz * 12 + sum(distinct[m] * R * 4 for m in range(N) if m != n) + 2 * w.dims[n] * R * 4
        compulsory.append(b)

    # ---- CPU baseline (the oracle) and accuracy against it
    cpu = None
    errs = {}
    if not args.no_cpu_baseline:
        import oracle

        S = min(args.cpu_sample_nnz, nnz)
        cs = [c[:S] for c in coords]
        vs = vals[:S]
        Ad = [a.astype(np.float64) for a in A]
        t0 = time.time()
        for n in range(N):
            oracle.mttkrp(cs, vs, Ad, n)
        cpu_s = time.time() - t0
        cpu = {"value": S * N / cpu_s / 1e9, "unit": "Gnnz/s", "cores": 1, "kind": "oracle",
               "sample": f"first {S} non-zeros of the workload, all {N} modes, fp64, "
                         f"single thread, {cpu_s:.1f}s"}
        log(f"cpu oracle: {cpu['value']:.4f} Gnnz/s over {S} non-zeros x {N} modes")
        rng = np.random.default_rng(7)
        Ab = [oracle.bf16_round(a).astype(np.float64) for a in A]
        vd = vals.astype(np.float64)
        for label, F, Aref in (("fp32", F32, Ad), ("bf16", BF16, Ab), ("bf16_vs_fp32", BF16, Ad)):
            worst = 0.0
            med = []
            for n in range(N):
                o = blco.mttkrp(T, n, F, out=outs[n])
                rows = np.unique(np.concatenate([np.arange(8), rng.integers(0, w.dims[n], 120)])
                                 ).astype(np.uint32)
                M, Ssum = oracle.mttkrp_rows(coords, vd, Aref, n, rows, w.dims)
                got = o[torch.from_numpy(rows.astype(np.int64)).to(dev)].cpu().numpy()
                nz = Ssum > 0
                e = np.abs(got.astype(np.float64) - M)[nz] / Ssum[nz]
                worst = max(worst, float(e.max()))
                med.append(float(np.median(e)))
            errs[label] = {"max": worst, "median": float(np.median(med))}
        log(f"errors: {errs}")

    tot = nnz * N
    res = {
        "metric": "MTTKRP Gnnz/s per mode & % HBM peak; bf16 vs fp32 factors at stated rel error",
        "value": tot / (ms_step * 1e-3) / 1e9,
        "unit": "Gnnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {N}-mode {'x'.join(str(d) for d in w.dims)}, {nnz} distinct "
                        f"non-zeros, per-mode {'/'.join(map(str, w.index_dist[0]))} indices, "
                        f"U(0,1) values, rank {R} N(0,1) factors; all-mode MTTKRP from one BLCO copy",
            "nnz": nnz, "dims": list(w.dims), "rank": R, "modes": N,
            "key_bits": inf["total_bits"], "blocks": inf["nblocks"],
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_mttkrp_win<32, float, 3>" if os.environ.get("BLCO_KERNEL", "win") == "win" else os.environ.get("BLCO_KERNEL"),
            "bytes_per_nnz": per_nnz,
            "avg_kernel_ms": avg_kernel_ms,
        },
        "cpu_baseline": cpu,
        "per_mode": {
            "fp32_call_ms": call_f32, "fp32_kernel_ms": kern_f32,
            "fp32_gnnz_s": [nnz / (x * 1e-3) / 1e9 for x in call_f32],
            "bf16_call_ms": call_bf16, "bf16_kernel_ms": kern_bf16,
            "bf16_gnnz_s": [nnz / (x * 1e-3) / 1e9 for x in call_bf16],
            "compulsory_bytes": compulsory,
            "compulsory_gbs_fp32": [b / (x * 1e-3) / 1e9 for b, x in zip(compulsory, kern_f32)],
            "distinct_indices": distinct,
        },
        "bf16": {"ms_per_step": ms_step_bf16, "value": tot / (ms_step_bf16 * 1e-3) / 1e9,
                 "unit": "Gnnz/s"},
        "errors": errs,
        "build_s": build_s,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
