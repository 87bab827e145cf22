"""Parity of the HIP path against the fp64 oracle at the workloads' full sizes, in the
launch configuration the benchmark times (run on an MI355X).

* 4-mode 2^24 x 2^22 x 2^20 x 2^10, 200M non-zeros (76-bit index, blocked on the top
  12 bits), R = 32 and 64, fp32 and bf16 factors, every mode: 256 rows per mode (the
  16 most frequent, rows 0-7, random rows and the last row) against the oracle, plus
  the cross-mode invariant sum(M^(n) * A^(n)) = sum_k x_k xhat_k that covers every
  entry at any size.
* 3-mode 2^22 x 2^21 x 2^20, 50M non-zeros, R = 32, fp32: every entry of every mode.
* Sparse CP loss and gradient on 2^20 x 2^18 x 2^16 x 2^12, 80M non-zeros, R = 32,
  fp32 and bf16 factor storage.

Acceptance (Eq. (1) per entry): |gpu - oracle| <= 1e-5 * S, S the sum of |terms|, and
exact zeros where no term lands; bf16 factors: the same bound against the oracle on
the bf16-rounded factors, and (N-1) * 2^-8 + 1e-5 against the fp32 factors (round to
nearest even moves each factor by at most 2^-9 of itself); CP gradients also carry the
fp32 residual's rounding, bounded through the model's magnitude (conftest.grad_allowed).
The threaded oracles used here are pinned to the serial ones in test_oracle_mttkrp.
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
TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sample_rows(counts, I, rng, k=256):
    """k distinct rows: the 16 most frequent, rows 0-7, the last row, random rows."""
    hot = np.argsort(-counts, kind="stable")[:16]
    fixed = np.unique(np.concatenate([hot, np.arange(min(8, I)), [I - 1]]))
    rest = np.setdiff1d(np.arange(I), fixed) if I <= 4096 else None
    want = max(0, min(k, I) - len(fixed))
    if rest is not None:
        extra = rng.choice(rest, size=min(want, len(rest)), replace=False)
    else:
        extra = np.setdiff1d(np.unique(rng.integers(0, I, 2 * want)), fixed)[:want]
    return np.unique(np.concatenate([fixed, extra])).astype(np.uint32)


def check(got, M, S, tol, label):
    got = np.asarray(got, dtype=np.float64)
    zero = S == 0
    assert np.all(got[zero] == 0.0), f"{label}: non-zero output where no term lands"
    err = np.abs(got - M)[~zero] / S[~zero]
    worst = float(err.max()) if err.size else 0.0
    say(f"{label}: max normalised error {worst:.2e} over {got.size} entries")
    assert worst <= tol, f"{label}: {worst:.3e} > {tol:.2e}"
    return worst


@pytest.mark.timeout(900)
def test_zipf4_full_size():
    w = synth.WORKLOADS["zipf4"]
    say("zipf4 full size: generating 200M non-zeros")
    coords, vals = synth.workload_tensor(w)
    assert len(vals) == 200_000_000
    say("zipf4: building")
    t = blco.build(coords, vals, w.dims)
    inf = t.info()
    assert inf["total_bits"] == 76 and inf["block_bits"] == 12
    counts = [np.bincount(c, minlength=d) for c, d in zip(coords, w.dims)]
    v64 = vals.astype(np.float64)
    rng = np.random.default_rng(2024)
    N = 4
    for R in w.ranks:
        A = synth.workload_factors(w, R)
        Ab = [oracle.bf16_round(a) for a in A]
        F32 = [torch.from_numpy(a).to(DEV) for a in A]
        BF = [blco.cast_bf16(f) for f in F32]
        inner = {"fp32": [], "bf16": []}
        for n in range(N):
            rows = sample_rows(counts[n], w.dims[n], rng)
            assert len(rows) >= 256 and rows.max() == w.dims[n] - 1
            ridx = torch.from_numpy(rows.astype(np.int64)).to(DEV)
            say(f"zipf4 R={R} mode {n}: oracle on {len(rows)} rows")
            M32, S32 = oracle.mttkrp_rows_omp(coords, v64, A, n, rows, w.dims)
            Mb, Sb = oracle.mttkrp_rows_omp(coords, v64, Ab, n, rows, w.dims)
            for dt, F in (("fp32", F32), ("bf16", BF)):
                out = blco.mttkrp(t, n, F)
                torch.cuda.synchronize()
                got = out[ridx].cpu().numpy()
                if dt == "fp32":
                    check(got, M32, S32, TOL, f"zipf4 R={R} fp32 mode {n}")
                else:
                    check(got, Mb, Sb, TOL, f"zipf4 R={R} bf16 mode {n}")
                    check(got, M32, S32, (N - 1) * 2.0 ** -8 + TOL,
                          f"zipf4 R={R} bf16-vs-fp32 mode {n}")
                Fn = F[n].float()
                inner[dt].append((float((out.double() * Fn.double()).sum()),
                                  float((out.double().abs() * Fn.double().abs()).sum())))
                del out
        for dt, v in inner.items():
            s = [a for a, _ in v]
            scale = max(b for _, b in v)
            say(f"zipf4 R={R} {dt}: cross-mode invariant spread {max(s) - min(s):.3e} "
                f"of {scale:.3e}")
            assert max(s) - min(s) <= TOL * scale
        del F32, BF
        torch.cuda.empty_cache()
    t.free()


@pytest.mark.timeout(900)
def test_zipf3_every_entry():
    w = synth.WORKLOADS["zipf3"]
    say("zipf3 full size: generating 50M non-zeros")
    coords, vals = synth.workload_tensor(w)
    t = blco.build(coords, vals, w.dims)
    A = synth.workload_factors(w, 32)
    F = [torch.from_numpy(a).to(DEV) for a in A]
    Ad = [a.astype(np.float64) for a in A]
    for n in range(3):
        out = blco.mttkrp(t, n, F)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        del out
        say(f"zipf3 mode {n}: full oracle")
        M, S, threads, _ = oracle.mttkrp_omp(coords, vals, Ad, n, dims=w.dims)
        check(got, M, S, TOL, f"zipf3 fp32 mode {n} (every entry, oracle on {threads} threads)")
        del M, S, got
    t.free()


@pytest.mark.timeout(900)
def test_cpgrad4_full_size():
    w = synth.WORKLOADS["cpgrad4"]
    say("cpgrad4 full size: generating 80M non-zeros")
    coords, _ = synth.workload_tensor(w)
    nnz = len(coords[0])
    assert nnz == 80_000_000
    G = [synth.draw_u01_matrix(d, 8, w.seed, synth.S_TRUTH + m) for m, d in enumerate(w.dims)]
    noise = synth.draw_normal_f64(nnz, 0.01, w.seed, synth.S_NOISE)
    vals = (oracle.cp_model_omp(coords, G) + noise).astype(np.float32)
    t = blco.build(coords, vals, w.dims)
    N, R = 4, 32
    A = [synth.draw_factor(d, R, w.seed, m, 0, R ** (-1.0 / (2 * N))) for m, d in enumerate(w.dims)]
    Ab = [oracle.bf16_round(a) for a in A]
    counts = [np.bincount(c, minlength=d) for c, d in zip(coords, w.dims)]
    v64 = vals.astype(np.float64)
    rng = np.random.default_rng(77)
    rows = [sample_rows(counts[n], w.dims[n], rng) for n in range(N)]

    def oracle_side(Aref):
        xh = oracle.cp_model_omp(coords, [a.astype(np.float64) for a in Aref])
        e = v64 - xh
        return 0.5 * float(np.dot(e, e)), e

    say("cpgrad4: oracle losses")
    f32, e32 = oracle_side(A)
    fb, eb = oracle_side(Ab)
    # the bf16 gradient against the fp32-factor oracle: rounding moves each factor by at
    # most 2^-9 of itself, so xhat_k by at most N 2^-9 sum_r prod_m |a|, and each term
    # e_k prod_{m != n} a by at most N 2^-9 (|e_k| + sum_r prod_m |a|) prod_{m != n} |a|
    # (first order); W below is that sum, and the bound takes twice the first-order term
    xabs = oracle.cp_model_omp(coords, [np.abs(a).astype(np.float64) for a in A])
    wvals = np.abs(e32) + xabs
    Aabs = [np.abs(a) for a in A]
    xabs_b = oracle.cp_model_omp(coords, [np.abs(a).astype(np.float64) for a in Ab])
    for storage in ("fp32", "bf16"):
        P = [torch.from_numpy(a).to(DEV).requires_grad_(True) for a in A]
        loss = blco.CPLoss.apply(t, storage, *P)
        loss.backward()
        torch.cuda.synchronize()
        f_ref, e_ref, Aref = (f32, e32, A) if storage == "fp32" else (fb, eb, Ab)
        got_f = float(loss.detach())
        rel = abs(got_f - f_ref) / f_ref
        say(f"cpgrad4 {storage}: loss {got_f:.9e}, oracle {f_ref:.9e}, rel {rel:.2e}")
        assert rel <= 1e-6
        for n in range(N):
            ridx = torch.from_numpy(rows[n].astype(np.int64)).to(DEV)
            got = P[n].grad[ridx].cpu().numpy().astype(np.float64)
            Gr, Sr = oracle.mttkrp_rows_omp(coords, -e_ref, Aref, n, rows[n], w.dims)
            # the fp32 residual's rounding is bounded by the model's magnitude (W), not by
            # |e_k|: conftest.grad_allowed
            xa = xabs if storage == "fp32" else xabs_b
            Wr, _ = oracle.mttkrp_rows_omp(coords, xa, [np.abs(a) for a in Aref], n, rows[n],
                                           w.dims)
            zero = Sr == 0
            assert np.all(got[zero] == 0.0)
            lim = grad_allowed(Sr, Wr, N, R)
            err = float((np.abs(got - Gr)[~zero] / Sr[~zero]).max())
            ratio = float((np.abs(got - Gr)[~zero] / lim[~zero]).max())
            say(f"cpgrad4 {storage} gradient mode {n}: max normalised error {err:.2e}, "
                f"max error / allowed {ratio:.2f}")
            assert np.all(np.abs(got - Gr) <= lim)
            if storage == "bf16":
                G32, _ = oracle.mttkrp_rows_omp(coords, -e32, A, n, rows[n], w.dims)
                W, _ = oracle.mttkrp_rows_omp(coords, wvals, Aabs, n, rows[n], w.dims)
                err = np.abs(got - G32)
                bound = (N * 2.0 ** -8 + TOL) * W
                worst = float((err / np.maximum(W, 1e-300)).max())
                say(f"cpgrad4 bf16-vs-fp32 gradient mode {n}: max error / W {worst:.2e} "
                    f"(bound {N * 2.0 ** -8 + TOL:.2e})")
                assert np.all(err <= bound)
        del P
    t.free()
