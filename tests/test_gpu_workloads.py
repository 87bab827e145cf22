"""The other workload recipes on the GPU against the fp64 oracle, on sampled rows.

Each runs at the full mode lengths and rank with fewer non-zeros, so the oracle
finishes in seconds (the full non-zero counts are measured by bench.py):
* 4-mode 2^24 x 2^22 x 2^20 x 2^10 (76-bit index: blocks on the top 12 bits),
  20M non-zeros, R = 32 and 64, fp32 and bf16 factors, every mode; at R = 64 the
  4 GiB mode-1 factor takes the 64-bit-addressing kernel;
* sparse CP loss and gradient on 2^20 x 2^18 x 2^16 x 2^12, 10M non-zeros
  holding a planted rank-8 model plus N(0, 0.01^2) noise, R = 32;
* out-of-memory streaming of the 2^23 x 2^23 x 2^17 Zipf(1.05) recipe, 24M
  non-zeros, under a budget that forces many chunks.
Acceptance as in test_gpu_parity: |gpu - oracle| <= tol * sum|terms| per entry; CP
gradients also carry the fp32 residual's rounding, bounded through the model's
magnitude (conftest.grad_allowed).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from conftest import grad_allowed  # noqa: E402
import paper_2201_12523_amd as blco  # noqa: E402
import synth  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rows_for(rng, I):
    return np.unique(np.concatenate([np.arange(min(6, I)), rng.integers(0, I, 40), [I - 1]])
                     ).astype(np.uint32)


def check_rows(out, coords, vals, A_ref, n, dims, rows, tol, label):
    M, S = oracle.mttkrp_rows_f32(coords, vals, A_ref, n, rows, dims)
    got = out[torch.from_numpy(rows.astype(np.int64)).to(DEV)].cpu().numpy().astype(np.float64)
    zero = S == 0
    assert np.all(got[zero] == 0.0), label
    err = float((np.abs(got - M)[~zero] / S[~zero]).max()) if (~zero).any() else 0.0
    say(f"{label}: max normalised error {err:.2e}")
    assert err <= tol, f"{label}: {err:.3e} > {tol:.1e}"


def test_zipf4_blocked():
    w = synth.WORKLOADS["zipf4"]
    say("zipf4 recipe: generating 20M non-zeros")
    coords, vals = synth.workload_tensor(w, nnz=20_000_000)
    say("zipf4: building")
    t = blco.build(coords, vals, w.dims)
    inf = t.info()
    assert inf["total_bits"] == 76 and inf["block_bits"] == 12 and inf["nruns"] > 1
    say(f"zipf4: {inf['nruns']} runs, {inf['nblocks']} blocks")
    rng = np.random.default_rng(4)
    for R in w.ranks:
        A = synth.workload_factors(w, R)
        F32 = [torch.from_numpy(a).to(DEV) for a in A]
        for dt in ("fp32", "bf16"):
            F = F32 if dt == "fp32" else [blco.cast_bf16(f) for f in F32]
            Aref = A if dt == "fp32" else [oracle.bf16_round(a) for a in A]
            for n in range(4):
                out = blco.mttkrp(t, n, F)
                torch.cuda.synchronize()
                rows = rows_for(rng, w.dims[n])
                check_rows(out, coords, vals, Aref, n, w.dims, rows, 1e-5, f"zipf4 R={R} {dt} mode {n}")
                if dt == "bf16":
                    check_rows(out, coords, vals, A, n, w.dims, rows, 3 * 2.0 ** -8 + 1e-5,
                               f"zipf4 R={R} bf16-vs-fp32 mode {n}")
                del out
            del F
        del F32
        torch.cuda.empty_cache()


def test_cpgrad4():
    w = synth.WORKLOADS["cpgrad4"]
    say("cpgrad4 recipe: generating 10M non-zeros")
    coords, _ = synth.workload_tensor(w, nnz=10_000_000)
    nnz = len(coords[0])
    G = [synth.draw_u01_matrix(d, 8, w.seed, synth.S_TRUTH + m) for m, d in enumerate(w.dims)]
    noise = synth.draw_normal_f64(nnz, 0.01, w.seed, synth.S_NOISE)
    vals = (oracle.cp_model(coords, G) + noise).astype(np.float32)
    t = blco.build(coords, vals, w.dims)
    R = 32
    A = [synth.draw_factor(d, R, w.seed, m, 0, R ** (-1.0 / 8)) for m, d in enumerate(w.dims)]
    say("cpgrad4: oracle loss")
    f_ref, e = oracle.cp_loss(coords, vals, [a.astype(np.float64) for a in A])
    xabs = oracle.cp_model(coords, [np.abs(a).astype(np.float64) for a in A])
    wvals = np.abs(e) + xabs
    rng = np.random.default_rng(5)
    for storage in ("fp32", "bf16"):
        P = [torch.from_numpy(a).to(DEV).requires_grad_(True) for a in A]
        loss = blco.CPLoss.apply(t, storage, *P)
        loss.backward()
        torch.cuda.synchronize()
        Aref = A if storage == "fp32" else [oracle.bf16_round(a) for a in A]
        f_st, e_st = (f_ref, e) if storage == "fp32" else oracle.cp_loss(
            coords, vals, [a.astype(np.float64) for a in Aref])
        rel = abs(float(loss.detach()) - f_st) / f_st
        say(f"cpgrad4 {storage}: loss {float(loss.detach()):.6e} oracle {f_st:.6e} rel {rel:.2e}")
        assert rel <= 1e-6
        negE = (-e_st).astype(np.float64)
        for n in range(4):
            rows = rows_for(rng, w.dims[n])
            Gr, Sr = oracle.mttkrp_rows(coords, negE, [a.astype(np.float64) for a in Aref], n,
                                        rows, w.dims)
            got = P[n].grad[torch.from_numpy(rows.astype(np.int64)).to(DEV)].cpu().numpy()
            # the fp32 residual's own rounding (bounded by the model's magnitude, W) on top
            # of 1e-5 of the sum of |terms|; see grad_allowed
            xa = xabs if storage == "fp32" else oracle.cp_model(
                coords, [np.abs(a).astype(np.float64) for a in Aref])
            Wr, _ = oracle.mttkrp_rows(coords, xa, [np.abs(a).astype(np.float64) for a in Aref],
                                       n, rows, w.dims)
            nz = Sr > 0
            assert np.all(got[~nz] == 0.0)
            err = float((np.abs(got - Gr)[nz] / Sr[nz]).max())
            lim = grad_allowed(Sr, Wr, 4, R)
            ratio = float((np.abs(got - Gr)[nz] / lim[nz]).max())
            say(f"cpgrad4 {storage} grad mode {n}: max normalised error {err:.2e}, "
                f"max error / allowed {ratio:.2f}")
            assert np.all(np.abs(got - Gr) <= lim)
            if storage == "bf16":
                # against the fp32-factor oracle: each bf16 factor is within 2^-9 of its
                # fp32 value, so each gradient term moves by at most about
                # N 2^-9 (|e_k| + sum_r prod_m |a|) prod_{m != n} |a|; W sums those weights
                # and the bound takes twice the first-order term
                G32, _ = oracle.mttkrp_rows(coords, -e, [a.astype(np.float64) for a in A], n,
                                            rows, w.dims)
                W, _ = oracle.mttkrp_rows(coords, wvals, [np.abs(a).astype(np.float64) for a in A],
                                          n, rows, w.dims)
                assert np.all(np.abs(got - G32) <= (4 * 2.0 ** -8 + 1e-5) * W)
        del P


def test_oom3_recipe_streamed():
    w = synth.WORKLOADS["oom3"]
    nnz = 24_000_000
    say(f"oom3 recipe: generating {nnz} non-zeros")
    coords, vals = synth.workload_tensor(w, nnz=nnz)
    t = blco.build(coords, vals, w.dims, placement="pinned", max_block_nnz=1 << 22)
    A = synth.workload_factors(w, 32)
    F = [torch.from_numpy(a).to(DEV) for a in A]
    rng = np.random.default_rng(6)
    for n in range(3):
        fixed = sum(int(np.prod(a.shape)) * 4 for m, a in enumerate(A) if m != n)
        fixed += w.dims[n] * 32 * 4 + t.info()["device_bytes"]
        budget = fixed + 2 * (3 << 20) * 12   # about 3M non-zeros per staging buffer
        out = blco.mttkrp_stream(t, n, F, device_budget=budget)
        torch.cuda.synchronize()
        inf = t.info()
        say(f"oom3 mode {n}: {inf['stream_chunks']} chunks of {inf['stream_chunk_nnz']}, "
            f"copy {inf['stream_copy_ms']:.1f} ms, kernels {inf['stream_kernel_ms']:.1f} ms, "
            f"span {inf['stream_total_ms']:.1f} ms")
        assert inf["stream_chunks"] >= 8 and inf["stream_peak_bytes"] <= budget
        check_rows(out, coords, vals, A, n, w.dims, rows_for(rng, w.dims[n]), 1e-5,
                   f"oom3 streamed mode {n}")
    # every mode in one pass over the non-zeros
    fixed = sum(int(np.prod(a.shape)) * 4 * 2 for a in A) + t.info()["device_bytes"]
    budget = fixed + 2 * (3 << 20) * 12
    outs = blco.mttkrp_stream_all(t, F, device_budget=budget)
    torch.cuda.synchronize()
    inf = t.info()
    say(f"oom3 all modes: {inf['stream_chunks']} chunks, copy {inf['stream_copy_ms']:.1f} ms, "
        f"kernels {inf['stream_kernel_ms']:.1f} ms, span {inf['stream_total_ms']:.1f} ms")
    assert inf["stream_chunks"] >= 8 and inf["stream_peak_bytes"] <= budget
    for n in range(3):
        check_rows(outs[n], coords, vals, A, n, w.dims, rows_for(rng, w.dims[n]), 1e-5,
                   f"oom3 one-pass mode {n}")
